"""Pins for the oracle's fixed-time signals (Algorithm 1 intersection branch),
from hand-derived closed forms rather than the oracle's own formula.

A lone vehicle on a line of two 100 m edges at 10 m/s moves 5 m per step and
reaches the first stop line about 20 steps after it enters; if the light is
red it comes to rest s0 = 2 m before the line (pinned separately) and crosses
in the first green step, so it enters the second edge one step later.  The
entry steps below are worked out by hand from each plan's cycle."""
import numpy as np
import pytest

import oracle
from paper_2406_08496_amd import synth


def plan_for(inst, n_phases, green, allred, offset, phase, node=1):
    n = inst.n_nodes
    P = synth.SignalPlan(np.zeros(n, np.int32), np.zeros(n, np.int32), np.zeros(n, np.int32),
                         np.zeros(n, np.int32), np.full(inst.n_edges, -1, np.int32))
    P.n_phases[node], P.green[node], P.allred[node], P.offset[node] = n_phases, green, allred, offset
    for e in np.nonzero(inst.dst == node)[0]:
        P.edge_phase[e] = phase
    return P


def entry_step_of_second_edge(plan, horizon=400):
    inst = synth.line_instance([100, 100], [10.0, 10.0], [1, 1], [0], [[0, 1]])
    o = oracle.OracleSim().load(inst)
    if plan is not None:
        o.set_signals(plan(inst))
    prev = None
    for k in range(1, horizon + 1):
        o.step(1)
        v = o.vehicles()
        if v["edge"][0] == 1:
            # the step before: at rest behind the line (or free running)
            return k, prev
        prev = (int(v["edge"][0]), float(v["x"][0]), float(v["v"][0]))
    raise AssertionError("never entered the second edge")


def test_no_signal_reference():
    k, prev = entry_step_of_second_edge(None)
    assert k == 21 and prev == (0, 95.0, 10.0)


@pytest.mark.parametrize("n_phases,green,allred,offset,phase,expect", [
    # one phase: green at cycle positions 0..9 of 210; red from step 10 to 209
    (1, 10, 200, 0, 0, 211),
    # offset 5 moves the next green 5 steps earlier: steps 205..214
    (1, 10, 200, 5, 0, 206),
    # two phases of 100 steps (10 green, 90 all-red), cycle 200:
    # phase 1 is green at positions 100..109, phase 0 at 0..9 (next at 200)
    (2, 10, 90, 0, 1, 101),
    (2, 10, 90, 0, 0, 201),
    # offset 30: phase 1 green when k + 30 is at 100..109 of the cycle, k = 70..79
    (2, 10, 90, 30, 1, 71),
])
def test_waits_for_first_green(n_phases, green, allred, offset, phase, expect):
    k, prev = entry_step_of_second_edge(lambda i: plan_for(i, n_phases, green, allred, offset, phase))
    assert k == expect
    edge, x, v = prev
    # waiting at the line: stopped on the first edge, inside the last 5 m
    assert edge == 0 and v == 0.0 and 95.0 <= x <= 99.0


def test_green_on_arrival_and_unserved_approach():
    # a long green covering the arrival at the line: no delay
    k, _ = entry_step_of_second_edge(lambda i: plan_for(i, 1, 100, 10, 0, 0))
    assert k == 21
    # a signalised node that does not serve this approach never stops it
    k, _ = entry_step_of_second_edge(lambda i: plan_for(i, 2, 10, 90, 0, -1))
    assert k == 21


def test_arrival_passes_no_signal():
    # a signal at the end of the last edge, red almost all the time: the trip
    # still arrives at its free-flow step (3 + 1 + 20 + 20)
    inst = synth.line_instance([100, 100], [10.0, 10.0], [1, 1], [3], [[0, 1]])
    o = oracle.OracleSim().load(inst)
    o.set_signals(plan_for(inst, 1, 1, 1000, 0, 0, node=2))
    o.step(60)
    v = o.vehicles()
    assert v["status"][0] == oracle.ST_DONE and v["arrival_step"][0] == 44


def congested(seed):
    return synth.grid_instance(seed=seed, side=4, n_trips=500, depart_window=120, len_lo=20, len_hi=80)


def test_all_green_plan_changes_nothing():
    inst = congested(11)
    plan = synth.signal_plan(inst, seed=11)
    # every signal reduced to one always-green phase
    on = plan.n_phases > 0
    plan.n_phases[on] = 1
    plan.allred[on] = 0
    plan.offset[on] = 0
    plan.edge_phase[plan.edge_phase >= 0] = 0
    a = oracle.OracleSim().load(inst)
    a.set_signals(plan)
    b = oracle.OracleSim().load(inst)
    for k in range(400):
        a.step(1)
        b.step(1)
        va, vb = a.vehicles(), b.vehicles()
        for key in ("status", "edge", "lane", "x", "v"):
            assert np.array_equal(va[key], vb[key]), (k, key)


def test_no_vehicle_crosses_on_red():
    inst = congested(12)
    plan = synth.signal_plan(inst, seed=12, green_s=10.0, allred_s=3.0)
    o = oracle.OracleSim().load(inst)
    o.set_signals(plan)
    before = o.vehicles()["edge"].copy()
    crossings = red_crossings = 0
    for k in range(600):
        o.step(1)
        after = o.vehicles()["edge"]
        moved = np.nonzero((before >= 0) & (after >= 0) & (after != before))[0]
        for t in moved:
            e = int(before[t])
            ph = int(plan.edge_phase[e])
            if ph < 0:
                continue
            node = int(inst.dst[e])
            g, r, nph = int(plan.green[node]), int(plan.allred[node]), int(plan.n_phases[node])
            # the cycle laid out as a boolean track, one entry per step
            track = np.concatenate([np.concatenate([np.full(g, q == ph), np.zeros(r, bool)])
                                    for q in range(nph)])
            crossings += 1
            if not track[(k + int(plan.offset[node])) % len(track)]:
                red_crossings += 1
        before = after.copy()
    assert crossings > 100 and red_crossings == 0


@pytest.mark.parametrize("field,value", [
    ("n_phases", 16), ("green", 0), ("allred", -1), ("offset", 10_000), ("edge_phase", 2),
])
def test_plan_validation(field, value):
    inst = synth.line_instance([100, 100], [10.0, 10.0], [1, 1], [0], [[0, 1]])
    plan = plan_for(inst, 2, 10, 5, 0, 1)
    arr = getattr(plan, field)
    if field == "edge_phase":
        arr[0] = value
    else:
        arr[1] = value
    o = oracle.OracleSim().load(inst)
    with pytest.raises(oracle.OracleError):
        o.set_signals(plan)


def test_plan_validation_unsignalised_node_and_long_cycle():
    inst = synth.line_instance([100, 100], [10.0, 10.0], [1, 1], [0], [[0, 1]])
    o = oracle.OracleSim().load(inst)
    plan = plan_for(inst, 2, 10, 5, 0, 1)
    plan.edge_phase[1] = 0  # edge 1 ends at node 2, which has no signal
    with pytest.raises(oracle.OracleError):
        o.set_signals(plan)
    plan = plan_for(inst, 15, 4000, 370, 0, 1)  # cycle 65,550 > 65,535
    with pytest.raises(oracle.OracleError):
        o.set_signals(plan)
    o.set_signals(None)
