"""Traffic assignment by the method of successive averages (MSA), with the
full simulation or the learned surrogate as the travel-time evaluator.

The paper's title promises accelerated traffic assignment; routes are the
simulator's input (Section 3.1, vehicle data) and rerouting is left open
(Section 5).  This driver alternates:

    evaluate(routes) -> edge travel times        (simulation or surrogate)
    best = shortest-time routes on those times    (native router)
    switch a deterministic 1/(n+1) share of trips to `best`

Everything numeric on the path runs in the library: the simulation kernels,
the router (host C++), network loading, feature and target construction,
and the perceptron's forward, backward and Adam kernels.  Python orchestrates
and moves arrays between host and device (PyTorch owns device memory).
"""
from __future__ import annotations

import ctypes
import time

import numpy as np

from .lpsim import LpsimError, Simulator, load_library

MASK64 = (1 << 64) - 1
WIN = 12  # statistics bins per perceptron sample


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def mix64(z):
    """SplitMix64 output function (Steele, Lea & Flood 2014), uint64 arrays."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def msa_switch(n_trips, n, seed):
    """Trip i moves to its new route at iteration n (1-based) iff
    mix64(seed ^ i<<8 ^ n) mod (n+1) == 0: a deterministic 1/(n+1) share."""
    i = np.arange(n_trips, dtype=np.uint64)
    h = mix64(np.uint64(seed) ^ (i << np.uint64(8)) ^ np.uint64(n))
    return (h % np.uint64(n + 1) == 0).astype(np.uint8)


class Router:
    """Shortest-time routes (library host code, lpsim_router_*)."""

    def __init__(self, n_nodes, src, dst, n_threads=0):
        self.lib = load_library()
        self.src = np.ascontiguousarray(src, np.int32)
        self.dst = np.ascontiguousarray(dst, np.int32)
        h = ctypes.c_void_p()
        rc = self.lib.lpsim_router_create(int(n_nodes), len(self.src), _p(self.src), _p(self.dst),
                                          int(n_threads), ctypes.byref(h))
        if rc:
            raise LpsimError(rc, "router create")
        self._h = h

    def __del__(self):
        if getattr(self, "_h", None):
            self.lib.lpsim_router_destroy(self._h)
            self._h = None

    def routes(self, cost, origin, dest, old=None, take_new=None):
        cost = np.ascontiguousarray(cost, np.float64)
        origin = np.ascontiguousarray(origin, np.int32)
        dest = np.ascontiguousarray(dest, np.int32)
        n = len(origin)
        rc = self.lib.lpsim_router_solve(self._h, _p(cost), n, _p(origin), _p(dest))
        if rc:
            raise LpsimError(rc, "router solve (bad cost, ids, or unreachable destination)")
        off = np.empty(n + 1, np.int64)
        oo = oe = tk = None
        if take_new is not None:
            oo = np.ascontiguousarray(old[0], np.int64)
            oe = np.ascontiguousarray(old[1], np.int32)
            tk = np.ascontiguousarray(take_new, np.uint8)
        rc = self.lib.lpsim_router_fill(self._h, _p(oo), _p(oe), _p(tk), _p(off), None)
        if rc:
            raise LpsimError(rc, "router fill")
        edges = np.empty(max(int(off[-1]), 1), np.int32)
        rc = self.lib.lpsim_router_fill(self._h, _p(oo), _p(oe), _p(tk), _p(off), _p(edges))
        if rc:
            raise LpsimError(rc, "router fill")
        return off, edges[:off[-1]]


def free_flow_steps(inst, dt):
    """Steps to cross an empty edge under the jump-to-speed-limit rule."""
    return np.ceil(np.ceil(inst.length.astype(np.float64)) / (inst.speed.astype(np.float64) * dt))


class Assignment:
    """One MSA run on an instance; `evaluate` is the full simulation or the
    surrogate depending on the mode."""

    def __init__(self, inst, n_bins=48, seed=0xA55, sim_params=None, n_threads=0, horizon=None):
        import torch

        self.torch = torch
        self.inst = inst
        self.n_bins = n_bins
        self.seed = seed
        self.horizon = horizon or inst.n_steps
        self.sim = Simulator(n_bins=n_bins, **(sim_params or {}))
        self.sim.load_network(inst.n_nodes, inst.src, inst.dst, inst.length, inst.lanes, inst.speed,
                              node_xy=inst.node_xy)
        self.dt = float(self.sim.params["dt"])
        self.bin_steps = int(round(self.sim.params["bin_seconds"] / self.dt))
        self.router = Router(inst.n_nodes, inst.src, inst.dst, n_threads=n_threads)
        self.tt_free = free_flow_steps(inst, self.dt)
        self.origin = inst.meta["origin"]
        self.dest = inst.meta["dest"]
        self.timings = {}

    # -- evaluation by simulation -------------------------------------------
    def simulate(self, off, edges):
        t0 = time.perf_counter()
        self.sim.load_trips(self.inst.depart_step, off, edges)
        self.sim.step(self.horizon)
        st = self.sim.edge_stats()
        self._add("simulate", time.perf_counter() - t0)
        return st

    def edge_tt_from_stats(self, st):
        """Mean simulated travel time per edge in seconds (free flow if unused)."""
        n = st["n_exits"].astype(np.float64)
        mean = np.where(n > 0, st["tt_sum"] / np.maximum(n, 1), self.tt_free)
        return np.maximum(mean, 1.0) * self.dt

    def _add(self, k, v):
        self.timings[k] = self.timings.get(k, 0.0) + v

    def reroute(self, cost_s, off, edges, n):
        t0 = time.perf_counter()
        take = msa_switch(len(self.origin), n, self.seed)
        new = self.router.routes(cost_s, self.origin, self.dest, old=(off, edges), take_new=take)
        self._add("route", time.perf_counter() - t0)
        return new

    # -- plain MSA -------------------------------------------------------------
    def run_plain(self, n_iter):
        t0 = time.perf_counter()
        off, edges = self.inst.route_off, self.inst.route_edges
        hist = []
        for n in range(1, n_iter + 1):
            st = self.simulate(off, edges)
            tt = self.edge_tt_from_stats(st)
            hist.append({"n": n, "mode": "sim", "mean_tt": float(np.average(tt, weights=st["n_exits"] + 1e-9))})
            off, edges = self.reroute(tt, off, edges, n)
        wall = time.perf_counter() - t0
        st = self.simulate(off, edges)
        return {"wall_s": wall, "tt": self.edge_tt_from_stats(st), "exits": st["n_exits"], "hist": hist,
                "routes": (off, edges)}

    # -- surrogate-assisted MSA -------------------------------------------------
    def run_surrogate(self, n_iter, judge_every=5, tol=0.05, train_steps=300, batch=8192, lr=2e-3,
                      passes=3, damping=0.5, mlp_seed=0):
        from .surrogate import EdgeMLP

        torch = self.torch
        dev = "cuda"
        lib = load_library()
        E, B = self.inst.n_edges, self.n_bins
        nw = B // WIN
        stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        length_d = torch.from_numpy(self.inst.length.astype(np.float32)).to(dev)
        lanes_d = torch.from_numpy(self.inst.lanes.astype(np.uint8)).to(dev)
        speed_d = torch.from_numpy(self.inst.speed.astype(np.float32)).to(dev)
        tt_free_d = torch.from_numpy(self.tt_free.astype(np.float32)).to(dev)
        dep_d = torch.from_numpy(self.inst.depart_step.astype(np.int32)).to(dev)
        jam = float(self.sim.params["veh_len"] + self.sim.params["s0"])
        net = EdgeMLP(seed=mlp_seed)
        vp = lambda t: ctypes.c_void_p(t.data_ptr())

        def check(rc, what):
            if rc:
                raise LpsimError(rc, what)

        def features(inflow_d, occ_d):
            x = torch.empty((E * nw, 32), dtype=torch.bfloat16, device=dev)
            check(lib.lpsim_surrogate_features(E, B, self.bin_steps, ctypes.c_float(jam), vp(inflow_d), vp(occ_d),
                                               vp(length_d), vp(lanes_d), vp(speed_d), vp(x), stream), "features")
            return x

        t0 = time.perf_counter()
        off, edges = self.inst.route_off, self.inst.route_edges
        hist = []
        buf_x, buf_y, buf_m = [], [], []
        use_sur = False
        tt_bins = torch.from_numpy(np.repeat(self.tt_free[:, None], B, 1).astype(np.float32)).to(dev)
        for n in range(1, n_iter + 1):
            judge = (n - 1) % judge_every == 0
            if judge or not use_sur:
                st = self.simulate(off, edges)
                tt = self.edge_tt_from_stats(st)
                ts = time.perf_counter()
                inflow_d = torch.from_numpy(st["inflow_bin"]).to(dev)
                occ_d = torch.from_numpy(st["occ_bin"]).to(dev)
                exits_d = torch.from_numpy(st["exits_bin"]).to(dev)
                ttb_d = torch.from_numpy(st["tt_bin"]).to(dev)
                x = features(inflow_d, occ_d)
                y = torch.empty((E * nw, 16), dtype=torch.float32, device=dev)
                m = torch.empty((E * nw, 16), dtype=torch.uint8, device=dev)
                check(lib.lpsim_surrogate_targets(E, B, vp(exits_d), vp(ttb_d), vp(tt_free_d), vp(y), vp(m), stream),
                      "targets")
                # judge: flow-weighted mean relative error of the current model
                # (host, float64)
                pred = net.forward(x)[:, :WIN].cpu().numpy().astype(np.float64)
                yh = y[:, :WIN].cpu().numpy().astype(np.float64)
                mh = m[:, :WIN].cpu().numpy().astype(bool)
                w = st["exits_bin"].reshape(E * nw, WIN).astype(np.float64)
                rel = np.abs(np.expm1(pred - yh)) * mh
                err = float((rel * w).sum() / max(w.sum(), 1.0))
                # keep samples that carry a target; train on the recent ones
                keep = m[:, :WIN].any(dim=1)
                buf_x.append(x[keep])
                buf_y.append(y[keep])
                buf_m.append(m[keep])
                buf_x, buf_y, buf_m = buf_x[-3:], buf_y[-3:], buf_m[-3:]
                X = torch.cat(buf_x)
                Y = torch.cat(buf_y)
                M = torch.cat(buf_m)
                g = torch.Generator(device=dev)
                g.manual_seed(n)
                for s in range(train_steps):
                    idx = torch.randint(0, X.shape[0], (min(batch, X.shape[0]),), device=dev, generator=g)
                    net.train_step(X[idx].contiguous(), Y[idx].contiguous(), M[idx].contiguous(), lr=lr)
                torch.cuda.synchronize()
                use_sur = err <= tol
                self._add("train", time.perf_counter() - ts)
                # estimates for the next surrogate passes start from the simulation
                ttb = st["tt_bin"] / np.maximum(st["exits_bin"], 1)
                tt_bins = torch.from_numpy(np.where(st["exits_bin"] > 0, ttb,
                                                    self.tt_free[:, None]).astype(np.float32)).to(dev)
                hist.append({"n": n, "mode": "sim", "judge_err": err, "samples": int(X.shape[0])})
            else:
                ts = time.perf_counter()
                off_d = torch.from_numpy(off).to(dev)
                edges_d = torch.from_numpy(edges).to(dev)
                inflow_d = torch.empty((E, B), dtype=torch.int32, device=dev)
                occ_d = torch.empty((E, B), dtype=torch.int64, device=dev)
                for _ in range(passes):
                    check(lib.lpsim_surrogate_load(vp(off_d), vp(edges_d), vp(dep_d), len(self.origin), vp(tt_bins),
                                                   E, B, self.bin_steps, self.horizon, vp(inflow_d), vp(occ_d),
                                                   stream), "load")
                    x = features(inflow_d, occ_d)
                    yp = net.forward(x)
                    check(lib.lpsim_surrogate_tt(E, B, vp(yp), vp(tt_free_d), ctypes.c_float(damping),
                                                 ctypes.c_float(float(self.horizon)), vp(tt_bins), stream), "tt")
                fl = inflow_d.cpu().numpy().astype(np.float64)
                tb = tt_bins.cpu().numpy().astype(np.float64)
                tot = fl.sum(1)
                tt_steps = np.where(tot > 0, (fl * tb).sum(1) / np.maximum(tot, 1.0), self.tt_free)
                tt = np.maximum(tt_steps, 1.0) * self.dt
                self._add("surrogate", time.perf_counter() - ts)
                hist.append({"n": n, "mode": "surrogate"})
            off, edges = self.reroute(tt, off, edges, n)
        wall = time.perf_counter() - t0
        st = self.simulate(off, edges)
        return {"wall_s": wall, "tt": self.edge_tt_from_stats(st), "exits": st["n_exits"], "hist": hist,
                "routes": (off, edges)}


def agreement(tt_a, tt_b, weights):
    """Flow-weighted relative L2 difference ||a - b||_w / ||b||_w."""
    w = np.asarray(weights, np.float64)
    return float(np.sqrt(np.sum(w * (tt_a - tt_b) ** 2)) / max(np.sqrt(np.sum(w * tt_b ** 2)), 1e-300))
