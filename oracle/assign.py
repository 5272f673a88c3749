"""CPU oracle of the surrogate's data path -- test infrastructure only.

Plain numpy versions of: network loading under estimated travel times,
perceptron features, training targets and the damped travel-time update.
Loading is integer work (exact); features and targets are computed in
float64 (the GPU rounds float32 results to bfloat16, compared within one
bfloat16 step)."""
from __future__ import annotations

import numpy as np

WIN = 12


def load(route_off, route_edges, depart, tt, n_bins, bin_steps, horizon):
    """Walk every trip's route: enter the first edge at depart + 1, spend
    max(1, round-half-even(tt[e][bin])) steps on an edge entered in `bin`, stop
    at the horizon.  Returns (entries per entry bin, vehicle-steps per bin)."""
    E = tt.shape[0]
    inflow = np.zeros((E, n_bins), np.int64)
    occ = np.zeros((E, n_bins), np.int64)
    n = len(depart)
    for i in range(n):
        t = int(depart[i]) + 1
        for j in range(route_off[i], route_off[i + 1]):
            if t >= horizon:
                break
            e = int(route_edges[j])
            b0 = min(t // bin_steps, n_bins - 1)
            inflow[e, b0] += 1
            est = float(np.float32(tt[e, b0]))
            tau = int(np.rint(est)) if est >= 1.0 else 1
            t_out = min(t + tau, horizon)
            for st in range(t, t_out):
                occ[e, min(st // bin_steps, n_bins - 1)] += 1
            t += tau
    return inflow, occ


def features(inflow, occ, length, lanes, speed, bin_steps, jam):
    E, B = inflow.shape
    nw = B // WIN
    x = np.zeros((E * nw, 32))
    cap = bin_steps * np.ceil(length.astype(np.float64)) * lanes
    for w in range(nw):
        rows = np.arange(E) * nw + w
        x[rows, 0:12] = np.log1p(inflow[:, w * WIN:(w + 1) * WIN])
        x[rows, 12:24] = occ[:, w * WIN:(w + 1) * WIN] / cap[:, None] * jam
        x[rows, 24] = np.log(length.astype(np.float64))
        x[rows, 25] = lanes / 4.0
        x[rows, 26] = speed.astype(np.float64) / 22.4
    return x


def targets(exits_bin, tt_sum_bin, tt_free):
    E, B = exits_bin.shape
    nw = B // WIN
    y = np.zeros((E * nw, 16))
    m = np.zeros((E * nw, 16), bool)
    for w in range(nw):
        rows = np.arange(E) * nw + w
        ex = exits_bin[:, w * WIN:(w + 1) * WIN]
        ts = tt_sum_bin[:, w * WIN:(w + 1) * WIN]
        ok = ex > 0
        y[rows, :12] = np.where(ok, np.log(ts / np.maximum(ex, 1) / tt_free[:, None]), 0.0)
        m[rows, :12] = ok
    return y, m


def tt_update(tt, y, tt_free, damping, tt_max):
    E, B = tt.shape
    nw = B // WIN
    out = tt.astype(np.float64).copy()
    for w in range(nw):
        rows = np.arange(E) * nw + w
        p = np.clip(tt_free[:, None] * np.exp(y[rows, :12]), 1.0, tt_max)
        out[:, w * WIN:(w + 1) * WIN] = (1 - damping) * out[:, w * WIN:(w + 1) * WIN] + damping * p
    return out


def shift(y_new, y_anchor, anchor_tt, max_shift, tt_max):
    """Anchored estimate: anchor_tt[e][b] * exp(clamped predicted change of
    log travel time for the sample (e, b // 12), output b % 12), clamped to
    [1, tt_max]."""
    E, B = anchor_tt.shape
    nw = B // WIN
    out = np.empty((E, B))
    for w in range(nw):
        rows = np.arange(E) * nw + w
        d = np.clip(y_new[rows, :WIN] - y_anchor[rows, :WIN], -max_shift, max_shift)
        out[:, w * WIN:(w + 1) * WIN] = np.clip(anchor_tt[:, w * WIN:(w + 1) * WIN] * np.exp(d), 1.0, tt_max)
    return out


def edge_tt(inflow, tt, tt_free, dt):
    """Routing cost per edge (seconds): entry-weighted mean of the per-bin
    travel time (steps), free flow where nobody entered, at least one step."""
    f = inflow.astype(np.float64)
    den = f.sum(1)
    num = (f * tt.astype(np.float64)).sum(1)
    t = np.where(den > 0, num / np.maximum(den, 1.0), tt_free.astype(np.float64))
    return np.maximum(t, 1.0) * dt
