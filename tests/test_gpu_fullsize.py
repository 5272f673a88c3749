"""The benchmark workloads at their full sizes, in the launch configuration
the benchmark times: regional (225,150 nodes, 550,000 edges, 2.82M trips,
28,800 steps), the same with fixed-time signals, large (1M nodes, 2.5M
edges, 9M trips, 36,000 steps) and the batch of 64 scenarios (4.4M edges,
7.6M trips, 14,400 steps).

The oracle cannot run the whole horizon in test time, so the check has two
parts:
- the first 2,400 steps (tens of thousands of vehicles on the road) are
  compared with the oracle element by element, bit for bit (for the batch,
  each scenario against its own oracle);
- the GPU then runs on alone to the horizon, and properties that hold at any
  size are checked every 2,400 steps: conservation, at most one vehicle per
  cell, front-to-front spacing of at least L in a lane, positions inside their
  edge, monotone positions on an unchanged edge, no watchdog, and at the end
  the statistics identities.
"""
from types import SimpleNamespace

import numpy as np
import pytest

import oracle
from paper_2406_08496_amd import synth

from test_gpu_parity import CNT_KEYS, assert_same_counters, assert_same_state, assert_same_stats, case

pytestmark = pytest.mark.gpu

BENCH_LAUNCH = (512, 640, 64)
ST_ACTIVE = 1


@pytest.fixture(scope="module")
def Sim():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_08496_amd.lpsim import Simulator

    return Simulator


def check_properties(v, c, inst, C, speed, prev):
    n = inst.n_trips
    st = v["status"]
    act = st == ST_ACTIVE
    assert c["waiting"] + c["active"] + c["arrived"] == n
    assert int(act.sum()) == c["active"]
    assert c["watchdog"] == 0
    e = v["edge"][act].astype(np.int64)
    x = v["x"][act].astype(np.float64)
    assert np.all(x >= 0) and np.all(x < C[e])
    assert np.all(v["cell"][act] == np.floor(x))
    # speed is carried over a transfer, so it is bounded by the fastest limit
    vv = v["v"][act]
    assert np.all(vv >= 0) and np.all(vv <= speed.max())
    assert np.all(v["lane"][act] < inst.lanes[e])
    key = e * 16 + v["lane"][act]
    order = np.lexsort((x, key))
    ks, xs = key[order], x[order]
    same = ks[1:] == ks[:-1]
    assert np.all(xs[1:][same] - xs[:-1][same] >= 5.0 - 1e-4)
    arr = st == 2
    assert np.all(v["arrival_step"][arr] <= c["step"]) and np.all(v["arrival_step"][~arr] == -1)
    if prev is not None:
        pe, px = prev
        both = act & (pe == v["edge"]) & (pe >= 0)
        assert np.all(v["x"][both] >= px[both])
    return v["edge"].copy(), v["x"].copy()


def properties_to_horizon(gpu, inst, horizon, every=2400, start=2400, edge_base=None):
    """Step to the horizon checking properties; edge_base (per trip) turns the
    batch's scenario-local edge ids into batch-wide ones."""
    C = np.ceil(inst.length.astype(np.float64)).astype(np.int64)
    speed = inst.speed.astype(np.float32)
    prev = None
    done = start
    while done < horizon:
        n = min(every, horizon - done)
        gpu.step(n)
        done += n
        c = gpu.counters()
        assert c["step"] == done
        case("properties at step", done, "active", c["active"], "arrived", c["arrived"])
        v = gpu.vehicles()
        if edge_base is not None:
            on = v["edge"] >= 0
            v["edge"] = np.where(on, v["edge"] + edge_base, -1).astype(np.int32)
        prev = check_properties(v, c, inst, C, speed, prev)
    c = gpu.counters()
    s = gpu.edge_stats()
    assert s["n_exits"].sum() == c["transfers"] + c["arrived"]
    assert s["inflow_bin"].sum() == c["transfers"] + c["departures"]
    assert np.array_equal(s["exits_bin"].sum(1), s["n_exits"])
    assert np.array_equal(s["tt_bin"].sum(1), s["tt_sum"])
    assert s["occ_bin"].sum() == c["vehicle_steps"]
    return c


@pytest.mark.parametrize("workload", ["regional", "large", "regional+signals"])
def test_full_size(Sim, workload):
    inst, n_bins = (synth.large(), 60) if workload == "large" else (synth.regional(), 48)
    plan = synth.signal_plan(inst) if workload.endswith("+signals") else None
    case(workload, "full size:", inst.n_nodes, "nodes,", inst.n_edges, "edges,", inst.n_trips, "trips")
    gpu = Sim(n_bins=n_bins)
    gpu.set_launch(*BENCH_LAUNCH)
    gpu.load(inst)
    ref = oracle.OracleSim(n_bins=n_bins).load(inst)
    if plan is not None:
        case("signals at", plan.n_signals, "nodes")
        gpu.set_signals(plan)
        ref.set_signals(plan)
    for k in (1200, 2400):
        gpu.step(1200)
        ref.step(1200)
        case("compare with the oracle at step", k)
        assert_same_state(gpu.vehicles(), ref.vehicles(), f"step {k}")
        assert_same_counters(gpu.counters(), ref.counters(), f"step {k}")
    assert_same_stats(gpu.edge_stats(), ref.edge_stats(), "step 2400")
    assert gpu.counters()["active"] > 10_000
    del ref
    c = properties_to_horizon(gpu, inst, inst.n_steps)
    assert c["arrived"] > inst.n_trips // 10


def test_batch_full_size(Sim):
    insts = synth.batch_scenarios()
    case("batch full size:", len(insts), "scenarios,", sum(i.n_trips for i in insts), "trips")
    gpu = Sim(n_bins=48)
    gpu.set_launch(*BENCH_LAUNCH)
    gpu.load_batch(insts)
    gpu.step(2400)
    vg, sg = gpu.vehicles(), gpu.edge_stats()
    for s, inst in enumerate(insts):
        t0, t1 = gpu.trip_off[s], gpu.trip_off[s + 1]
        e0, e1 = gpu.edge_off[s], gpu.edge_off[s + 1]
        ref = oracle.OracleSim(n_bins=48).load(inst)
        ref.step(2400)
        case("scenario", s, "trips", inst.n_trips, "compared at step 2400")
        # the batch reports each scenario's trips with its own edge ids
        assert_same_state({k: vg[k][t0:t1] for k in vg}, ref.vehicles(), f"scenario {s}")
        assert_same_stats({k: sg[k][e0:e1] for k in sg}, ref.edge_stats(), f"scenario {s}")
        del ref
    # properties to the horizon over the concatenated instance
    cat = SimpleNamespace(n_trips=sum(i.n_trips for i in insts),
                          length=np.concatenate([i.length for i in insts]),
                          lanes=np.concatenate([i.lanes for i in insts]),
                          speed=np.concatenate([i.speed for i in insts]))
    edge_base = np.repeat(np.asarray(gpu.edge_off[:-1], np.int64), [i.n_trips for i in insts])
    c = properties_to_horizon(gpu, cat, max(i.n_steps for i in insts), edge_base=edge_base)
    assert c["arrived"] > cat.n_trips // 10
