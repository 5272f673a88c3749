"""Brute-force reference for tiny networks, written independently of the C oracle.

It keeps no lane map at all: every occupancy question ("what is the first
vehicle ahead of cell c in lane l of edge e?") is answered by looking at every
vehicle.  The arithmetic is numpy binary32 scalars, one rounding per
operation, in the same order as the method's definition, so its state must
equal the oracle's bit for bit.  Only tiny instances (tens of vehicles) are
feasible.

The model (paper Section 3.1 equations, Algorithm 1, Remarks; the
deterministic reading used throughout this project):
  * occupancy: a vehicle occupies the one metre cell floor(x) of its lane and
    shows its speed truncated to an integer (capped at 254);
  * each step, every active vehicle looks ahead D cells in its own lane; a
    vehicle there is its leader (gap = cell - x - L, speed = its shown
    speed); otherwise, if the stop line is within reach and the next edge's
    entry cells (first W cells of the target lane) are taken, the stop line
    is a standing obstacle (gap = C - x); otherwise the road is free;
  * IDM with delta = 4 for the leader and stop-line cases, the jump to the
    speed limit (or IDM free road) otherwise, then the no-overlap clamp;
  * crossing the end: arrive on the last edge, else request the target lane
    (lane index capped by the next edge's lane count); departures request the
    lane (trip id mod lanes) of the first edge when its entry cells are free;
    per target lane the lowest trip id wins;
  * a fixed-time signal at the end of an edge that is not serving it makes
    the stop line a standing obstacle too (departures and arrivals pass no
    signal);
  * lane change on the post-move positions, toward the lane given by the
    rank of the next edge among the node's out-edges, even steps toward lane
    0 only, odd steps away from it, with a hashed Bernoulli draw and lead/lag
    gap acceptance; the critical gaps' random terms are uniform on
    [-eps, eps) from a second hashed stream, added before the clamp at zero;
  * statistics (Algorithm 1 records the entry time t_start of each edge):
    entries in the bin of the entry step, finished traversals and their
    times in the bin of their entry step, and occupancy counted step by step
    (every vehicle on an edge at the start of a step, in that step's bin),
    where a step's bin is floor(step * dt / bin_seconds), capped at the last.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

f32 = np.float32
MASK64 = (1 << 64) - 1
EPS_STREAM = 0xD6E8FEB86659FD93  # key of the random gap terms' stream


def splitmix_out(z: int) -> int:
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


class BruteSim:
    def __init__(self, inst, dt=0.5, a=1.0, b=1.5, s0=2.0, T=1.5, veh_len=5.0,
                 x0=100.0, g_a=2.0, g_b=2.0, alpha_i=1.0, alpha_a=1.0, alpha_b=1.0,
                 seed=0x5EED, free_mode=0, lane_change=1, eps_a=0.0, eps_b=0.0,
                 bin_seconds=300.0, n_bins=12, **_ignored):
        self.inst = inst
        # statistics: a step's bin is floor(step * dt / bin_seconds) in exact
        # rational arithmetic, the last bin taking every later step
        self.bin_dt = Fraction(float(f32(dt)))
        self.bin_len = Fraction(float(bin_seconds))
        self.n_bins = int(n_bins)
        E = inst.n_edges
        self.st = {k: np.zeros((E, self.n_bins), np.int64)
                   for k in ("inflow_bin", "exits_bin", "tt_bin", "occ_bin")}
        self.tt_sum = np.zeros(E, np.int64)
        self.n_exits = np.zeros(E, np.int64)
        self.dt, self.a, self.b, self.s0, self.T = f32(dt), f32(a), f32(b), f32(s0), f32(T)
        self.L, self.x0 = f32(veh_len), f32(x0)
        self.g_a, self.g_b = f32(g_a), f32(g_b)
        self.al_i, self.al_a, self.al_b = f32(alpha_i), f32(alpha_a), f32(alpha_b)
        self.seed = seed
        self.eps_a, self.eps_b = f32(eps_a), f32(eps_b)
        self.free_mode = free_mode
        self.lane_change = lane_change
        self.W = math.ceil(float(f32(veh_len)) + float(f32(s0)))
        vmax = max(float(v) for v in inst.speed)
        self.D = math.ceil(float(f32(veh_len)) + max(2.0 * float(f32(dt)) * vmax,
                                                      float(f32(s0)) + float(f32(T)) * vmax))
        self.tsab = f32(2.0 * math.sqrt(float(f32(a)) * float(f32(b))))
        self.C = [int(math.ceil(float(l))) for l in inst.length]
        self.nl = [int(l) for l in inst.lanes]
        self.v0 = [f32(v) for v in inst.speed]
        outs = {}
        for e in range(inst.n_edges):
            outs.setdefault(int(inst.src[e]), []).append(e)
        self.rank = {}
        self.deg = {}
        for u, es in outs.items():
            for r, e in enumerate(sorted(es)):
                self.rank[e] = r
                self.deg[e] = len(es)
        n = inst.n_trips
        self.routes = [list(map(int, inst.route(i))) for i in range(n)]
        self.depart = [int(d) for d in inst.depart_step]
        self.status = [0] * n
        self.e = [-1] * n
        self.l = [0] * n
        self.x = [f32(0)] * n
        self.v = [f32(0)] * n
        self.rp = [0] * n
        self.enter = [-1] * n
        self.arr = [-1] * n
        self.blocked = set()
        self.signals = None  # synth.SignalPlan or None
        self.k = 0

    def _green(self, e, k):
        """Walk the node's cycle phase by phase (green, then all-red) from the
        cycle position of step k; True if edge e is served at that moment."""
        sp = self.signals
        if sp is None or int(sp.edge_phase[e]) < 0:
            return True
        n = int(self.inst.dst[e])
        g, r, nph = int(sp.green[n]), int(sp.allred[n]), int(sp.n_phases[n])
        pos = (k + int(sp.offset[n])) % (nph * (g + r))
        for ph in range(nph):
            if pos < g:
                return ph == int(sp.edge_phase[e])
            pos -= g
            if pos < r:
                return False
            pos -= r
        raise AssertionError("position outside the cycle")

    # -- statistics ---------------------------------------------------------------
    def _bin(self, step):
        return min(math.floor(step * self.bin_dt / self.bin_len), self.n_bins - 1)

    def _record_exit(self, e, enter, exit_step):
        """A finished traversal: counted, with its time, in its entry step's bin."""
        b = self._bin(enter)
        self.st["exits_bin"][e, b] += 1
        self.st["tt_bin"][e, b] += exit_step - enter
        self.n_exits[e] += 1
        self.tt_sum[e] += exit_step - enter

    def _record_entry(self, e, step):
        self.st["inflow_bin"][e, self._bin(step)] += 1

    def stats(self):
        out = {k: v.copy() for k, v in self.st.items()}
        out["tt_sum"] = self.tt_sum.copy()
        out["n_exits"] = self.n_exits.copy()
        return out

    # -- occupancy queries without a map ---------------------------------------
    def _occ(self, e, l, cells=None):
        """{cell: shown speed} of the active vehicles in lane l of edge e."""
        out = {}
        for i, st in enumerate(self.status):
            if st == 1 and self.e[i] == e and self.l[i] == l:
                vv = self.v[i]
                shown = int(min(float(vv), 254.0))
                out[int(math.floor(float(self.x[i])))] = shown
        return out

    def _first_ahead(self, occ, lo, hi):
        best = None
        for c in occ:
            if lo <= c <= hi and (best is None or c < best):
                best = c
        return best

    def _first_behind(self, occ, hi, lo):
        best = None
        for c in occ:
            if lo <= c <= hi and (best is None or c > best):
                best = c
        return best

    def _entry_taken(self, e, l):
        if e in self.blocked:
            return True
        occ = self._occ(e, l)
        return any(0 <= c < self.W for c in occ)

    # -- dynamics ---------------------------------------------------------------
    def _idm(self, x, v, v0, gap, vl):
        if gap <= f32(0):
            return x, f32(0)
        dv = v - vl
        t = (v * self.T) + ((v * dv) / self.tsab)
        ss = self.s0 + (t if t > f32(0) else f32(0))
        r = v / v0
        r2 = r * r
        r4 = r2 * r2
        q = ss / gap
        q2 = q * q
        acc = self.a * ((f32(1) - r4) - q2)
        nv = v + acc * self.dt
        vn = nv if nv > f32(0) else f32(0)
        return x + (v + vn) * (f32(0.5) * self.dt), vn

    def _free(self, x, v, v0):
        if self.free_mode == 0:
            return x + v0 * self.dt, v0
        r = v / v0
        r2 = r * r
        r4 = r2 * r2
        acc = self.a * (f32(1) - r4)
        nv = v + acc * self.dt
        vn = nv if nv > f32(0) else f32(0)
        return x + (v + vn) * (f32(0.5) * self.dt), vn

    def step(self):
        k = self.k
        n = len(self.status)
        active0 = [i for i in range(n) if self.status[i] == 1]
        occ_cache = {}

        def occ(e, l):
            if (e, l) not in occ_cache:
                occ_cache[(e, l)] = self._occ(e, l)
            return occ_cache[(e, l)]

        # occupancy: every vehicle on an edge at the start of step k counts
        # one step in that edge's bin of step k
        for i in active0:
            self.st["occ_bin"][self.e[i], self._bin(k)] += 1
        intents = {}
        requests = {}  # (edge, lane) -> list of ids
        for i in active0:
            e, l, x, v = self.e[i], self.l[i], self.x[i], self.v[i]
            C = self.C[e]
            c = int(math.floor(float(x)))
            route = self.routes[i]
            last = self.rp[i] == len(route) - 1
            o = occ(e, l)
            lead = self._first_ahead(o, c + 1, min(c + self.D, C - 1))
            if lead is not None:
                vl = f32(o[lead])
                xn, vn = self._idm(x, v, self.v0[e], (f32(lead) - x) - self.L, vl)
                if xn > f32(lead) - self.L:
                    xn = max(x, f32(lead) - self.L)
                    vn = vn if vn < vl else vl
            else:
                blocked = False
                if not last and c + self.D >= C:
                    en = route[self.rp[i] + 1]
                    blocked = (not self._green(e, k)) or self._entry_taken(en, min(l, self.nl[en] - 1))
                if blocked:
                    xn, vn = self._idm(x, v, self.v0[e], f32(C) - x, f32(0))
                    if xn > f32(C - 1):
                        xn = max(x, f32(C - 1))
                        vn = f32(0)
                else:
                    xn, vn = self._free(x, v, self.v0[e])
            kind = "move"
            tgt = None
            if xn >= f32(C):
                if last:
                    kind = "arrive"
                else:
                    en = route[self.rp[i] + 1]
                    tgt = (en, min(l, self.nl[en] - 1))
                    kind = "claim"
                    requests.setdefault(tgt, []).append(i)
            intents[i] = (kind, xn, vn, tgt)
        deps = []
        for i in range(n):
            if self.status[i] == 0 and self.depart[i] <= k:
                e0 = self.routes[i][0]
                l0 = i % self.nl[e0]
                if not self._entry_taken(e0, l0):
                    requests.setdefault((e0, l0), []).append(i)
                    deps.append(i)
        winners = {t: min(ids) for t, ids in requests.items()}
        entered = set()
        for i in active0:
            kind, xn, vn, tgt = intents[i]
            if kind == "arrive":
                self._record_exit(self.e[i], self.enter[i], k + 1)
                self.status[i] = 2
                self.arr[i] = k + 1
                self.e[i] = -1
            elif kind == "claim":
                if winners[tgt] == i:
                    self._record_exit(self.e[i], self.enter[i], k + 1)
                    self._record_entry(tgt[0], k + 1)
                    self.e[i], self.l[i] = tgt
                    self.x[i], self.v[i] = f32(0), vn
                    self.rp[i] += 1
                    self.enter[i] = k + 1
                    entered.add(i)
                else:
                    lim = f32(self.C[self.e[i]] - 1)
                    self.x[i] = self.x[i] if self.x[i] > lim else lim
                    self.v[i] = f32(0)
            else:
                self.x[i], self.v[i] = xn, vn
        for i in deps:
            e0 = self.routes[i][0]
            if winners[(e0, i % self.nl[e0])] == i:
                self.status[i] = 1
                self.e[i], self.l[i] = e0, i % self.nl[e0]
                self.x[i], self.v[i] = f32(0), f32(0)
                self.rp[i] = 0
                self.enter[i] = k + 1
                self._record_entry(e0, k + 1)
                entered.add(i)
        if self.lane_change:
            new_l = {}
            occ_cache.clear()
            for i in range(n):
                if self.status[i] != 1 or i in entered:
                    continue
                route = self.routes[i]
                if self.rp[i] == len(route) - 1:
                    continue
                e, l, x, v = self.e[i], self.l[i], self.x[i], self.v[i]
                en = route[self.rp[i] + 1]
                want = (self.rank[en] * self.nl[e]) // self.deg[en]
                if want == l:
                    continue
                d = 1 if want > l else -1
                if (k % 2 == 0) != (d < 0):
                    continue
                dist = f32(self.C[e]) - x
                p = f32(0) if dist >= self.x0 else f32(1) - dist / self.x0
                h = splitmix_out(self.seed ^ ((i << 32) | (k & 0xFFFFFFFF)))
                if not (f32(h >> 40) < p * f32(16777216.0)):
                    continue
                ea = eb = f32(0)
                if self.eps_a > 0 or self.eps_b > 0:
                    # second stream, same (trip, step) key: 24 bits per term
                    h2 = splitmix_out(self.seed ^ EPS_STREAM ^ ((i << 32) | (k & 0xFFFFFFFF)))
                    ua, ub = h2 >> 40, (h2 >> 16) & 0xFFFFFF
                    ea = self.eps_a * (f32(ua) / f32(2 ** 23) - f32(1))
                    eb = self.eps_b * (f32(ub) / f32(2 ** 23) - f32(1))
                lt = l + d
                c = int(math.floor(float(x)))
                o = occ(e, lt)
                if c in o:
                    continue
                ok = True
                ca = self._first_ahead(o, c + 1, min(c + self.D, self.C[e] - 1))
                if ca is not None:
                    va = f32(o[ca])
                    need = self.g_a + max(f32(0), ((self.al_i * v) - (self.al_a * va)) + ea)
                    if not ((f32(ca) - x) - self.L >= need):
                        ok = False
                cb = self._first_behind(o, c - 1, max(0, c - self.D))
                if ok and cb is not None:
                    vb = f32(o[cb])
                    need = self.g_b + max(f32(0), ((self.al_b * vb) - (self.al_i * v)) + eb)
                    if not ((x - self.L) - f32(cb + 1) >= need):
                        ok = False
                if ok:
                    new_l[i] = lt
            for i, lt in new_l.items():
                self.l[i] = lt
        self.k = k + 1

    def state(self):
        n = len(self.status)
        act = [self.status[i] == 1 for i in range(n)]
        return dict(
            status=np.array(self.status, np.uint8),
            edge=np.array([self.e[i] if act[i] else -1 for i in range(n)], np.int32),
            lane=np.array([self.l[i] if act[i] else 0 for i in range(n)], np.uint8),
            x=np.array([self.x[i] if act[i] else 0 for i in range(n)], np.float32),
            v=np.array([self.v[i] if act[i] else 0 for i in range(n)], np.float32),
            arrival_step=np.array(self.arr, np.int32),
        )
