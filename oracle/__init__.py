"""CPU oracle for the LPSim vehicle update -- test infrastructure only.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg use
this package.  It wraps `lpsim_oracle.c` (plain C, binary32, no contraction)
through ctypes and shares nothing with the GPU library.

Every function is documented in `lpsim_oracle.c` with the passage of the paper
it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_build", "liblpsim_oracle.so")
# the same source built with OpenMP: its two per-vehicle loops run on all host
# cores, with results identical to the single-threaded build
_SO_OMP = os.path.join(_HERE, "_build", "liblpsim_oracle_omp.so")
_libs = {}

ST_WAIT, ST_ACTIVE, ST_DONE = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle: gcc -O2 -ffp-contract=off, no fast-math; once
    single-threaded and once with OpenMP."""
    os.makedirs(os.path.dirname(_SO), exist_ok=True)
    for so, extra in ((_SO, ["-Wno-unknown-pragmas"]), (_SO_OMP, ["-fopenmp"])):
        if force or not os.path.exists(so):
            tmp = so + ".tmp%d" % os.getpid()
            subprocess.check_call([
                "gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math",
                "-Wall", *extra, "-shared", "-fPIC", os.path.join(_HERE, "lpsim_oracle.c"),
                "-o", tmp, "-lm",
            ])
            os.replace(tmp, so)
    return _SO


class OrParams(ctypes.Structure):
    _fields_ = [
        ("dt", ctypes.c_float), ("a", ctypes.c_float), ("b", ctypes.c_float),
        ("s0", ctypes.c_float), ("T", ctypes.c_float), ("veh_len", ctypes.c_float),
        ("x0", ctypes.c_float), ("g_a", ctypes.c_float), ("g_b", ctypes.c_float),
        ("alpha_i", ctypes.c_float), ("alpha_a", ctypes.c_float), ("alpha_b", ctypes.c_float),
        ("bin_seconds", ctypes.c_double), ("delta", ctypes.c_int32),
        ("n_bins", ctypes.c_int32), ("seed", ctypes.c_uint64),
        ("free_mode", ctypes.c_int32), ("lane_change", ctypes.c_int32),
        ("eps_a", ctypes.c_float), ("eps_b", ctypes.c_float),
    ]


class OrCounters(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "step", "active", "waiting", "arrived", "vehicle_steps", "transfers",
        "departures", "claims_lost", "lc_attempts", "lc_accepts", "watchdog")]


def _load(parallel: bool = False):
    so = _SO_OMP if parallel else _SO
    if so not in _libs:
        if not os.path.exists(so):
            build(force=False)
        lib = ctypes.CDLL(so)
        vp = ctypes.c_void_p
        lib.or_create.argtypes = [ctypes.POINTER(OrParams), ctypes.POINTER(vp)]
        lib.or_destroy.argtypes = [vp]
        lib.or_destroy.restype = None
        lib.or_load_network.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp, vp]
        lib.or_load_trips.argtypes = [vp, ctypes.c_int64, vp, vp, vp]
        lib.or_block_edge.argtypes = [vp, ctypes.c_int32, ctypes.c_int32]
        lib.or_set_signals.argtypes = [vp] + [vp] * 5
        lib.or_step.argtypes = [vp, ctypes.c_int32]
        lib.or_place.argtypes = [vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.c_float, ctypes.c_float]
        lib.or_get_vehicles.argtypes = [vp] + [vp] * 7
        lib.or_get_progress.argtypes = [vp, vp, vp]
        lib.or_edge_stats.argtypes = [vp] + [vp] * 6
        lib.or_get_counters.argtypes = [vp, ctypes.POINTER(OrCounters)]
        lib.or_invariant_broken.argtypes = [vp]
        lib.or_window.argtypes = [vp, ctypes.c_int32]
        lib.or_window.restype = ctypes.c_int32
        lib.or_map_bytes.argtypes = [vp]
        lib.or_map_bytes.restype = ctypes.c_int64
        lib.or_threads.argtypes = []
        lib.or_threads.restype = ctypes.c_int32
        _libs[so] = lib
    return _libs[so]


DEFAULTS = dict(dt=0.5, a=1.0, b=1.5, s0=2.0, T=1.5, veh_len=5.0, x0=100.0,
                g_a=2.0, g_b=2.0, alpha_i=1.0, alpha_a=1.0, alpha_b=1.0,
                bin_seconds=300.0, delta=4, n_bins=12, seed=0x5EED, free_mode=0,
                lane_change=1, eps_a=0.0, eps_b=0.0)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


class OracleError(RuntimeError):
    pass


class OracleSim:
    """One simulation instance on the CPU oracle.  parallel=True runs the
    OpenMP build (all host cores, OMP_NUM_THREADS if set); its results are
    identical to the single-threaded build's."""

    def __init__(self, parallel=False, **params):
        self.parallel = bool(parallel)
        self._lib = lib = _load(self.parallel)
        kw = dict(DEFAULTS)
        kw.update(params)
        self.params = kw
        self._p = OrParams(**kw)
        h = ctypes.c_void_p()
        self._check(lib.or_create(ctypes.byref(self._p), ctypes.byref(h)), "create")
        self._h = h
        self.n_edges = 0
        self.n_trips = 0

    def _check(self, rc, what):
        if rc != 0:
            raise OracleError(f"oracle {what} failed: {rc}")

    def close(self):
        if getattr(self, "_h", None):
            self._lib.or_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load_network(self, n_nodes, src, dst, length, lanes, speed):
        src = np.ascontiguousarray(src, np.int32)
        dst = np.ascontiguousarray(dst, np.int32)
        length = np.ascontiguousarray(length, np.float32)
        lanes = np.ascontiguousarray(lanes, np.uint8)
        speed = np.ascontiguousarray(speed, np.float32)
        self._check(self._lib.or_load_network(self._h, n_nodes, len(src), _ptr(src), _ptr(dst),
                                            _ptr(length), _ptr(lanes), _ptr(speed)), "load_network")
        self.n_edges = len(src)

    def load_trips(self, depart_step, route_off, route_edges):
        d = np.ascontiguousarray(depart_step, np.int32)
        o = np.ascontiguousarray(route_off, np.int64)
        r = np.ascontiguousarray(route_edges, np.int32)
        if len(r) == 0:
            r = np.zeros(1, np.int32)
        self._check(self._lib.or_load_trips(self._h, len(d), _ptr(d), _ptr(o), _ptr(r)), "load_trips")
        self.n_trips = len(d)

    def load(self, inst):
        self.load_network(inst.n_nodes, inst.src, inst.dst, inst.length, inst.lanes, inst.speed)
        self.load_trips(inst.depart_step, inst.route_off, inst.route_edges)
        return self

    def block_edge(self, e, on=True):
        self._check(self._lib.or_block_edge(self._h, e, 1 if on else 0), "block_edge")

    def set_signals(self, plan):
        """Fixed-time signal plan (`synth.SignalPlan`), or None to remove it."""
        if plan is None:
            self._check(self._lib.or_set_signals(self._h, None, None, None, None, None), "set_signals")
            return
        arrs = [np.ascontiguousarray(getattr(plan, k), np.int32)
                for k in ("n_phases", "green", "allred", "offset", "edge_phase")]
        self._check(self._lib.or_set_signals(self._h, *[_ptr(a) for a in arrs]), "set_signals")

    def place(self, trip, rp, lane, x, v):
        """Test hook: put waiting `trip` on its route edge `rp` at (lane, x, v)."""
        self._check(self._lib.or_place(self._h, trip, rp, lane, float(np.float32(x)),
                                     float(np.float32(v))), "place")

    @property
    def threads(self):
        """Threads the per-vehicle loops run on (1 for the single-threaded build)."""
        return int(self._lib.or_threads())

    def step(self, n=1):
        self._check(self._lib.or_step(self._h, n), "step")

    @property
    def W(self):
        return self._lib.or_window(self._h, 0)

    @property
    def D(self):
        return self._lib.or_window(self._h, 1)

    @property
    def bin_steps(self):
        return self._lib.or_window(self._h, 2)

    def vehicles(self):
        n = self.n_trips
        out = dict(edge=np.empty(n, np.int32), lane=np.empty(n, np.uint8),
                   cell=np.empty(n, np.int32), x=np.empty(n, np.float32),
                   v=np.empty(n, np.float32), arrival_step=np.empty(n, np.int32),
                   status=np.empty(n, np.uint8))
        self._check(self._lib.or_get_vehicles(self._h, *[_ptr(out[k]) for k in (
            "edge", "lane", "cell", "x", "v", "arrival_step", "status")]), "get_vehicles")
        return out

    def progress(self):
        n = self.n_trips
        rp = np.empty(n, np.int32)
        en = np.empty(n, np.int32)
        self._check(self._lib.or_get_progress(self._h, _ptr(rp), _ptr(en)), "get_progress")
        return rp, en

    def edge_stats(self):
        E, B = self.n_edges, self.params["n_bins"]
        out = dict(tt_sum=np.empty(E, np.int64), n_exits=np.empty(E, np.int32),
                   inflow_bin=np.empty((E, B), np.int32), exits_bin=np.empty((E, B), np.int32),
                   tt_bin=np.empty((E, B), np.int64), occ_bin=np.empty((E, B), np.int64))
        self._check(self._lib.or_edge_stats(self._h, *[_ptr(out[k]) for k in (
            "tt_sum", "n_exits", "inflow_bin", "exits_bin", "tt_bin", "occ_bin")]), "edge_stats")
        return out

    def counters(self):
        c = OrCounters()
        self._check(self._lib.or_get_counters(self._h, ctypes.byref(c)), "counters")
        return {n: int(getattr(c, n)) for n, _ in OrCounters._fields_}

    @property
    def invariant_broken(self):
        return bool(self._lib.or_invariant_broken(self._h))
