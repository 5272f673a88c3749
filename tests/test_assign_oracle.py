"""Pins of the surrogate's data-path oracle (oracle/assign.py) against
independent formulations: a step-by-step walk for the network loading,
hand-computed feature and target values, and the special cases of the
anchored estimate and the routing cost."""
import numpy as np

from oracle import assign as oa


def brute_load(route_off, route_edges, depart, tt, n_bins, bin_steps, horizon):
    """Step by step: at every step s < horizon, find the edge each trip is on
    by replaying its route from the departure (independent of the oracle's
    interval arithmetic)."""
    E = tt.shape[0]
    inflow = np.zeros((E, n_bins), np.int64)
    occ = np.zeros((E, n_bins), np.int64)
    for i in range(len(depart)):
        # schedule: (edge, enter step, leave step)
        sched = []
        t = int(depart[i]) + 1
        for j in range(route_off[i], route_off[i + 1]):
            e = int(route_edges[j])
            b = min(t // bin_steps, n_bins - 1)
            v = float(tt[e, b])
            # round half to even, at least one step
            tau = max(1, int(round(v))) if v >= 1.0 else 1
            sched.append((e, t, t + tau))
            t += tau
        for e, a, z in sched:
            if a < horizon:
                inflow[e, min(a // bin_steps, n_bins - 1)] += 1
        for s in range(horizon):
            for e, a, z in sched:
                if a <= s < z:
                    occ[e, min(s // bin_steps, n_bins - 1)] += 1
    return inflow, occ


def test_load_matches_step_by_step_walk():
    rng = np.random.default_rng(5)
    E, B, bs, H = 9, 6, 7, 40
    n = 25
    lens = rng.integers(1, 5, size=n)
    off = np.r_[0, np.cumsum(lens)].astype(np.int64)
    edges = rng.integers(0, E, size=off[-1]).astype(np.int32)
    dep = rng.integers(0, 30, size=n).astype(np.int32)
    tt = rng.uniform(0.2, 9.0, size=(E, B)).astype(np.float32)
    tt[0, :] = 2.5  # exact half: rounds to 2
    tt[1, :] = 3.5  # rounds to 4
    a = oa.load(off, edges, dep, tt, B, bs, H)
    b = brute_load(off, edges, dep, tt, B, bs, H)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_load_single_trip_closed_form():
    # one trip over edges 0, 1, 2 with 3, 4 and 5 steps each; departs at 0
    tt = np.array([[3.0], [4.0], [5.0]], np.float32)
    inflow, occ = oa.load(np.array([0, 3]), np.array([0, 1, 2]), np.array([0]), tt, 1, 100, 100)
    assert list(inflow[:, 0]) == [1, 1, 1]
    assert list(occ[:, 0]) == [3, 4, 5]
    # horizon cuts the last edge after 2 of its 5 steps (enters at 8)
    inflow, occ = oa.load(np.array([0, 3]), np.array([0, 1, 2]), np.array([0]), tt, 1, 100, 10)
    assert list(occ[:, 0]) == [3, 4, 2]


def test_features_hand_values():
    inflow = np.zeros((1, 12), np.int64)
    inflow[0, 3] = 1
    occ = np.zeros((1, 12), np.int64)
    occ[0, 5] = 600 * 100 * 2  # one vehicle per metre of lane through the bin
    x = oa.features(inflow, occ, np.array([100.0]), np.array([2]), np.array([22.4]), 600, 7.0)
    assert x.shape == (1, 32)
    assert x[0, 3] == np.log(2.0) and x[0, 0] == 0.0
    assert x[0, 12 + 5] == 7.0
    assert np.isclose(x[0, 24], np.log(100.0)) and x[0, 25] == 0.5 and x[0, 26] == 1.0
    assert np.all(x[0, 27:] == 0)


def test_targets_hand_values():
    ex = np.zeros((1, 12), np.int64)
    ts = np.zeros((1, 12), np.int64)
    ex[0, 2], ts[0, 2] = 4, 4 * 30  # mean 30 steps over free flow 10 -> log 3
    y, m = oa.targets(ex, ts, np.array([10.0]))
    assert m[0, 2] and m.sum() == 1
    assert np.isclose(y[0, 2], np.log(3.0)) and y[0, 0] == 0.0


def test_shift_special_cases():
    rng = np.random.default_rng(1)
    E, B = 4, 24
    anc = rng.uniform(1.0, 50.0, size=(E, B))
    y = rng.normal(size=(E * 2, 16))
    # no predicted change: the anchor itself
    assert np.array_equal(oa.shift(y, y, anc, 1.0, 1e9), anc)
    # a change of +log 2 in sample (edge 1, window 1), output 3 -> bin 15
    y2 = y.copy()
    y2[1 * 2 + 1, 3] += np.log(2.0)
    out = oa.shift(y2, y, anc, 1.0, 1e9)
    diff = np.argwhere(out != anc)
    assert diff.tolist() == [[1, 15]] and np.isclose(out[1, 15], 2 * anc[1, 15])
    # clamped change and clamped result
    y3 = y + 5.0
    assert np.allclose(oa.shift(y3, y, anc, 1.0, 1e9), anc * np.e)
    assert oa.shift(y3, y, anc, 1.0, 10.0).max() == 10.0
    assert oa.shift(y - 5.0, y, np.ones((E, B)), 1.0, 10.0).min() == 1.0


def test_edge_tt_special_cases():
    tt = np.full((3, 12), 8.0)
    tt[1, :6] = 4.0
    inflow = np.zeros((3, 12), np.int64)
    inflow[0, :] = 1
    inflow[1, 0], inflow[1, 6] = 3, 1  # 3 at 4 steps, 1 at 8 steps -> 5
    out = oa.edge_tt(inflow, tt, np.array([2.0, 2.0, 0.25]), 0.5)
    assert out[0] == 4.0 and out[1] == 2.5
    # nobody entered: free flow, at least one step
    assert out[2] == 0.5
