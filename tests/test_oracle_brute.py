"""The oracle against an independent brute-force simulator (no lane map,
all-pairs neighbour search) on tiny networks: full state and every binned
statistic equal at every step.

Congested settings (short edges, many trips, narrow departure windows) are
chosen so that claims, losers, queues and lane changes all occur."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as hs

import oracle
from brute_sim import BruteSim
from paper_2406_08496_amd import synth

KEYS = ("status", "edge", "lane", "x", "v", "arrival_step")


def compare_stats(o, b, where):
    so, sb = o.edge_stats(), b.stats()
    for key in sb:
        if not np.array_equal(so[key], sb[key]):
            bad = np.argwhere(so[key] != sb[key])[:5]
            raise AssertionError(f"{where} stats {key} at {bad.tolist()}")


def compare_run(inst, n_steps, **params):
    # short statistics bins (10 s = 20 steps) so that runs span many of them
    params = dict(dict(bin_seconds=10.0, n_bins=24), **params)
    o = oracle.OracleSim(**params).load(inst)
    b = BruteSim(inst, **dict(oracle.DEFAULTS, **params))
    for k in range(n_steps):
        o.step(1)
        b.step()
        vo, vb = o.vehicles(), b.state()
        for key in KEYS:
            if not np.array_equal(vo[key], vb[key]):
                bad = np.nonzero(vo[key] != vb[key])[0][:5]
                raise AssertionError(f"step {k} field {key} trips {bad}: "
                                     f"oracle {vo[key][bad]} brute {vb[key][bad]}")
        compare_stats(o, b, f"step {k}")
    return o


@pytest.mark.parametrize("seed,free_mode,n,w", [(1, 0, 200, 40), (2, 1, 300, 100), (3, 0, 300, 100)])
def test_brute_congested_grid(seed, free_mode, n, w):
    inst = synth.grid_instance(seed=seed, side=3, n_trips=n, depart_window=w,
                               len_lo=20, len_hi=100, lanes=2)
    o = compare_run(inst, 600, free_mode=free_mode)
    c = o.counters()
    assert c["claims_lost"] > 0 and c["lc_accepts"] > 0 and c["transfers"] > 0


@settings(max_examples=12, deadline=None, suppress_health_check=list(HealthCheck))
@given(seed=hs.integers(0, 10**6), side=hs.integers(2, 3), lanes=hs.integers(1, 3),
       n_trips=hs.integers(1, 150), window=hs.integers(1, 80),
       free_mode=hs.integers(0, 1), lane_change=hs.integers(0, 1))
def test_brute_random(seed, side, lanes, n_trips, window, free_mode, lane_change):
    inst = synth.grid_instance(seed=seed, side=side, n_trips=n_trips, depart_window=window,
                               len_lo=8, len_hi=40, lanes=lanes)
    compare_run(inst, 250, free_mode=free_mode, lane_change=lane_change, seed=seed)


def test_brute_mixed_lanes_and_blocking():
    """Edges with 1..4 lanes (target lane capped by the next edge's lane count)
    and a blocked edge that builds a queue."""
    rng = np.random.default_rng(5)
    inst = synth.grid_instance(seed=5, side=3, n_trips=50, depart_window=50, len_lo=12, len_hi=40)
    inst.lanes = np.repeat(rng.integers(1, 5, size=inst.n_edges // 2), 2).astype(np.uint8)
    o = oracle.OracleSim().load(inst)
    b = BruteSim(inst, **oracle.DEFAULTS)
    hot = int(np.bincount(inst.route_edges).argmax())
    o.block_edge(hot)
    b.blocked.add(hot)
    for k in range(200):
        if k == 120:
            o.block_edge(hot, False)
            b.blocked.discard(hot)
        o.step(1)
        b.step()
        vo, vb = o.vehicles(), b.state()
        for key in KEYS:
            assert np.array_equal(vo[key], vb[key]), (k, key)


@pytest.mark.parametrize("seed,green_s,allred_s", [(6, 6.0, 2.0), (7, 15.0, 0.0)])
def test_brute_signals(seed, green_s, allred_s):
    """Fixed-time signals at every 3- and 4-way node of a congested grid: the
    oracle and the brute-force simulator (its own walk through the cycle) agree
    at every step, and vehicles do queue at red lights."""
    inst = synth.grid_instance(seed=seed, side=3, n_trips=120, depart_window=60, len_lo=12, len_hi=40)
    plan = synth.signal_plan(inst, seed=seed, green_s=green_s, allred_s=allred_s)
    assert plan.n_signals > 0
    o = oracle.OracleSim().load(inst)
    o.set_signals(plan)
    b = BruteSim(inst, **oracle.DEFAULTS)
    b.signals = plan
    for k in range(300):
        o.step(1)
        b.step()
        vo, vb = o.vehicles(), b.state()
        for key in KEYS:
            assert np.array_equal(vo[key], vb[key]), (k, key)
    free = oracle.OracleSim().load(inst)
    free.step(300)
    assert o.counters()["vehicle_steps"] > free.counters()["vehicle_steps"]


@pytest.mark.parametrize("seed,eps_a,eps_b", [(8, 1.0, 0.0), (9, 0.5, 3.0), (10, 4.0, 4.0)])
def test_brute_random_gap_terms(seed, eps_a, eps_b):
    """Random lead/lag gap terms: the brute-force simulator draws them with its
    own hash code; equal state at every step."""
    inst = synth.grid_instance(seed=seed, side=3, n_trips=250, depart_window=80, len_lo=15, len_hi=60, lanes=3)
    o = compare_run(inst, 400, seed=seed * 31, eps_a=eps_a, eps_b=eps_b)
    assert o.counters()["lc_accepts"] > 0
