"""Fixed-time signals (Algorithm 1 intersection branch) on the GPU against the
oracle, element by element: small grids every step in several launch shapes,
a plan installed and removed mid-run, a batch with one plan per scenario, the
line case whose entry step is known in closed form, and the validation
errors of the entry point."""
import numpy as np
import pytest

import oracle
from paper_2406_08496_amd import synth
from paper_2406_08496_amd.lpsim import EINVAL, LpsimError

from test_gpu_parity import assert_same_counters, assert_same_state, assert_same_stats, case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Sim():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_08496_amd.lpsim import Simulator

    return Simulator


def pair(Sim, inst, plan, params=None, launch=None):
    params = params or {}
    gpu = Sim(**params)
    if launch:
        gpu.set_launch(*launch)
    gpu.load(inst)
    gpu.set_signals(plan)
    ref = oracle.OracleSim(**params).load(inst)
    ref.set_signals(plan)
    return gpu, ref


def test_line_first_green(Sim):
    case("line of two 100 m edges, two-phase signal, offset 30: entry at step 71")
    inst = synth.line_instance([100, 100], [10.0, 10.0], [1, 1], [0], [[0, 1]])
    n = inst.n_nodes
    plan = synth.SignalPlan(np.zeros(n, np.int32), np.zeros(n, np.int32), np.zeros(n, np.int32),
                            np.zeros(n, np.int32), np.full(inst.n_edges, -1, np.int32))
    plan.n_phases[1], plan.green[1], plan.allred[1], plan.offset[1] = 2, 10, 90, 30
    plan.edge_phase[0] = 1
    gpu, ref = pair(Sim, inst, plan)
    for k in range(1, 101):
        gpu.step(1)
        ref.step(1)
        v = gpu.vehicles()
        assert_same_state(v, ref.vehicles(), f"step {k}")
        # enters the second edge at 71 and leaves it 20 steps of 5 m later
        assert v["edge"][0] == (0 if k < 71 else 1 if k < 91 else -1)


@pytest.mark.parametrize("seed,green_s,allred_s,launch", [
    (1, 10.0, 3.0, None), (2, 40.0, 5.0, (256, 16, 1)), (3, 6.0, 0.0, (64, 8, 0)), (4, 20.0, 4.0, (1024, 2048, 7))])
def test_signalised_grid_every_step(Sim, seed, green_s, allred_s, launch):
    case("signalised 4x4 grid", seed, green_s, allred_s, launch)
    inst = synth.grid_instance(seed=60 + seed, side=4, n_trips=600, depart_window=150,
                               len_lo=20, len_hi=90, lanes=1 + seed % 3)
    plan = synth.signal_plan(inst, seed=seed, green_s=green_s, allred_s=allred_s)
    assert plan.n_signals > 0
    gpu, ref = pair(Sim, inst, plan, params=dict(n_bins=6, bin_seconds=60.0, seed=seed), launch=launch)
    for k in range(1, 701):
        gpu.step(1)
        ref.step(1)
        if k % 3 == 0 or k < 50:
            assert_same_state(gpu.vehicles(), ref.vehicles(), f"step {k}")
    assert_same_stats(gpu.edge_stats(), ref.edge_stats())
    assert_same_counters(gpu.counters(), ref.counters())
    assert ref.counters()["claims_lost"] > 0


def test_plan_installed_and_removed_mid_run(Sim):
    case("5x5 grid: signals from step 200 (vehicles on the road), removed at 500")
    inst = synth.grid_instance(seed=71, side=5, n_trips=1200, depart_window=400, len_lo=30, len_hi=120)
    plan = synth.signal_plan(inst, seed=71, green_s=12.0, allred_s=3.0)
    gpu = Sim().load(inst)
    ref = oracle.OracleSim().load(inst)
    for k in range(800):
        if k == 200:
            gpu.set_signals(plan)
            ref.set_signals(plan)
        if k == 500:
            gpu.set_signals(None)
            ref.set_signals(None)
        gpu.step(1)
        ref.step(1)
        if k % 4 == 3 or k in (200, 201, 500, 501):
            assert_same_state(gpu.vehicles(), ref.vehicles(), f"step {k + 1}")
    assert_same_stats(gpu.edge_stats(), ref.edge_stats())
    assert_same_counters(gpu.counters(), ref.counters())


def test_graphs_after_plan_change(Sim):
    case("64-step graphs, plan changed between graph launches")
    inst = synth.grid_instance(seed=72, side=5, n_trips=1000, depart_window=300, len_lo=30, len_hi=120)
    plan = synth.signal_plan(inst, seed=72)
    gpu = Sim()
    gpu.set_launch(512, 64, 64)
    gpu.load(inst)
    ref = oracle.OracleSim().load(inst)
    gpu.step(128)
    ref.step(128)
    gpu.set_signals(plan)
    ref.set_signals(plan)
    for _ in range(6):
        gpu.step(128)
        ref.step(128)
        assert_same_state(gpu.vehicles(), ref.vehicles(), "graphs")
    assert_same_counters(gpu.counters(), ref.counters())


def test_batch_with_plans(Sim):
    case("batch of 3 grids, one plan each (one scenario without signals)")
    insts = [synth.grid_instance(seed=80 + s, side=4 + s, n_trips=300 * (s + 1), depart_window=200,
                                 len_lo=20, len_hi=100, lanes=1 + s % 2) for s in range(3)]
    plans = [synth.signal_plan(i, seed=s, green_s=15.0 + 10 * s) for s, i in enumerate(insts)]
    none = plans[1]
    none.n_phases[:] = 0
    none.edge_phase[:] = -1
    bat = Sim().load_batch(insts)
    bat.set_signals(synth.concat_signal_plans(plans, insts))
    bat.step(900)
    vb, sb = bat.vehicles(), bat.edge_stats()
    for s, inst in enumerate(insts):
        t0, t1 = bat.trip_off[s], bat.trip_off[s + 1]
        e0, e1 = bat.edge_off[s], bat.edge_off[s + 1]
        ref = oracle.OracleSim().load(inst)
        ref.set_signals(plans[s])
        ref.step(900)
        assert_same_state({k: vb[k][t0:t1] for k in vb}, ref.vehicles(), f"scenario {s}")
        assert_same_stats({k: sb[k][e0:e1] for k in sb}, ref.edge_stats(), f"scenario {s}")


def test_plan_validation(Sim):
    case("signal plan validation errors")
    inst = synth.line_instance([100, 100], [10.0, 10.0], [1, 1], [0], [[0, 1]])
    gpu = Sim().load(inst)
    n = inst.n_nodes

    def plan(**over):
        p = synth.SignalPlan(np.zeros(n, np.int32), np.zeros(n, np.int32), np.zeros(n, np.int32),
                             np.zeros(n, np.int32), np.full(inst.n_edges, -1, np.int32))
        p.n_phases[1], p.green[1], p.allred[1], p.offset[1] = 2, 10, 5, 0
        p.edge_phase[0] = 1
        for k, (i, v) in over.items():
            getattr(p, k)[i] = v
        return p

    gpu.set_signals(plan())
    for bad in (dict(n_phases=(1, 16)), dict(green=(1, 0)), dict(allred=(1, -1)),
                dict(offset=(1, 30)), dict(edge_phase=(0, 2)), dict(edge_phase=(1, 0)),
                dict(n_phases=(1, 15), green=(1, 4000), allred=(1, 370))):
        with pytest.raises(LpsimError) as e:
            gpu.set_signals(plan(**bad))
        assert e.value.code == EINVAL, bad
    gpu.set_signals(None)
    gpu.step(30)
    assert gpu.vehicles()["edge"][0] == 1  # no signal: entered at step 21


def test_restore_follows_current_plan(Sim):
    case("snapshot with signals on, restored after the plan and a block were removed")
    inst = synth.grid_instance(seed=73, side=5, n_trips=1000, depart_window=300, len_lo=30, len_hi=120)
    plan = synth.signal_plan(inst, seed=73, green_s=12.0, allred_s=3.0)
    hot = int(np.bincount(inst.route_edges).argmax())
    gpu = Sim().load(inst)
    gpu.set_signals(plan)
    gpu.block_edge(hot)
    ref = oracle.OracleSim().load(inst)
    ref.set_signals(plan)
    ref.block_edge(hot)
    gpu.step(300)
    ref.step(300)
    snap = gpu.save_state()
    gpu.step(100)
    gpu.set_signals(None)
    gpu.block_edge(hot, False)
    ref.set_signals(None)
    ref.block_edge(hot, False)
    # back to step 300: the cached flags must follow the edges as they are now
    gpu.restore_state(snap)
    for k in range(300, 500, 20):
        gpu.step(20)
        ref.step(20)
        assert_same_state(gpu.vehicles(), ref.vehicles(), f"step {k + 20}")
    assert_same_stats(gpu.edge_stats(), ref.edge_stats())


def test_signals_with_random_gap_terms(Sim):
    case("signalised 5x5 grid, 3 lanes, random gap terms, every step")
    inst = synth.grid_instance(seed=77, side=5, n_trips=1200, depart_window=300, len_lo=25, len_hi=110, lanes=3)
    plan = synth.signal_plan(inst, seed=77, green_s=15.0, allred_s=3.0)
    params = dict(eps_a=1.5, eps_b=2.5, seed=4242, n_bins=6, bin_seconds=60.0)
    gpu, ref = pair(Sim, inst, plan, params=params, launch=(256, 64, 16))
    for k in range(1, 801):
        gpu.step(1)
        ref.step(1)
        if k % 2 == 0:
            assert_same_state(gpu.vehicles(), ref.vehicles(), f"step {k}")
    assert_same_stats(gpu.edge_stats(), ref.edge_stats())
    assert_same_counters(gpu.counters(), ref.counters())
    c = ref.counters()
    assert c["lc_accepts"] > 0 and c["claims_lost"] > 0
