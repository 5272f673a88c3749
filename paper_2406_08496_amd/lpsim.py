"""Python binding of the gfx950 LPSim library (argument marshalling only).

Every step of the simulation runs in the HIP kernels of `liblpsim.so`; this
module converts numpy arrays to pointers and status codes to exceptions.
PyTorch is used only to hand the library a HIP stream.  There is no CPU
fallback: if the library is missing or no GPU is present, construction fails.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "liblpsim.so")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, ECAPACITY = 0, -1, -2, -3, -4, -5
WAITING, ACTIVE, ARRIVED = 0, 1, 2
PHASES = ("move", "resolve", "lanechange", "commit", "reorder")

_lib = None


class LpsimError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lpsim error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
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


class Counters(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "step", "active", "waiting", "arrived", "vehicle_steps", "transfers",
        "departures", "claims_lost", "lc_attempts", "lc_accepts", "watchdog",
        "scan_bytes")]


DEFAULT_PARAMS = dict(dt=0.5, a=1.0, b=1.5, s0=2.0, T=1.5, veh_len=5.0, x0=100.0,
                      g_a=2.0, g_b=2.0, alpha_i=1.0, alpha_a=1.0, alpha_b=1.0,
                      bin_seconds=300.0, delta=4, n_bins=12, seed=0x5EED,
                      free_mode=0, lane_change=1, eps_a=0.0, eps_b=0.0)

# exported symbol -> (argtypes, restype)
_vp = ctypes.c_void_p
_i32, _i64 = ctypes.c_int32, ctypes.c_int64
SIGNATURES = {
    "lpsim_create": ([ctypes.POINTER(Params), ctypes.POINTER(_vp)], _i32),
    "lpsim_destroy": ([_vp], None),
    "lpsim_set_allocator": ([_vp, _vp, _vp, _vp], _i32),
    "lpsim_load_network": ([_vp, _i32, _vp, _i32, _vp, _vp, _vp, _vp, _vp], _i32),
    "lpsim_load_trips": ([_vp, _i64, _vp, _vp, _vp], _i32),
    "lpsim_batch_load": ([_vp, _i32] + [_vp] * 13, _i32),
    "lpsim_step": ([_vp, _i32, _vp], _i32),
    "lpsim_prepare_steps": ([_vp, _i32], _i32),
    "lpsim_edge_stats": ([_vp] + [_vp] * 6, _i32),
    "lpsim_edge_stats_device": ([_vp] * 6, _i32),
    "lpsim_get_vehicles": ([_vp] + [_vp] * 7, _i32),
    "lpsim_get_counters": ([_vp, ctypes.POINTER(Counters)], _i32),
    "lpsim_block_edge": ([_vp, _i32, _i32], _i32),
    "lpsim_set_signals": ([_vp, _vp, _vp, _vp, _vp, _vp], _i32),
    "lpsim_set_launch": ([_vp, _i32, _i32, _i32], _i32),
    "lpsim_set_timing": ([_vp, _i32], _i32),
    "lpsim_kernel_times": ([_vp, _vp, _vp, _i32], _i32),
    "lpsim_state_size": ([_vp, ctypes.POINTER(ctypes.c_size_t)], _i32),
    "lpsim_save_state": ([_vp, _vp, ctypes.c_size_t], _i32),
    "lpsim_restore_state": ([_vp, _vp, ctypes.c_size_t], _i32),
    "lpsim_query": ([_vp, _i32], _i32),
    "lpsim_autotune": ([_vp, _i32, _vp, _i32, _vp, _i32, _vp, _vp], _i32),
    "lpsim_router_create": ([_i32, _i32, _vp, _vp, _i32, ctypes.POINTER(_vp)], _i32),
    "lpsim_router_destroy": ([_vp], None),
    "lpsim_router_solve": ([_vp, _vp, _i64, _vp, _vp], _i32),
    "lpsim_router_solve_gpu": ([_vp, _vp, _i64, _vp, _vp, _vp], _i32),
    "lpsim_msa_switch": ([_i64, _i32, ctypes.c_uint64, _vp], _i32),
    "lpsim_edge_tt": ([_i32, _vp, _vp, _vp, ctypes.c_double, _vp], _i32),
    "lpsim_edge_tt_bins": ([_i32, _i32, _vp, _vp, _vp, _vp], _i32),
    "lpsim_edge_tt_bins_device": ([_i32, _i32, _vp, _vp, _vp, _vp, _vp], _i32),
    "lpsim_router_fill": ([_vp, _vp, _vp, _vp, _vp, _vp], _i32),
    "lpsim_surrogate_load": ([_vp, _vp, _vp, _i64, _vp, _i32, _i32, _i32, _i32, _vp, _vp, _vp], _i32),
    "lpsim_surrogate_features": ([_i32, _i32, _i32, ctypes.c_float, _vp, _vp, _vp, _vp, _vp, _vp, _vp], _i32),
    "lpsim_surrogate_targets": ([_i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp], _i32),
    "lpsim_surrogate_tt": ([_i32, _i32, _vp, _vp, ctypes.c_float, ctypes.c_float, _vp, _vp], _i32),
    "lpsim_surrogate_shift": ([_i32, _i32, _vp, _vp, _vp, ctypes.c_float, ctypes.c_float, _vp, _vp], _i32),
    "lpsim_surrogate_edge_tt": ([_i32, _i32, _vp, _vp, _vp, ctypes.c_float, _vp, _vp], _i32),
    "lpsim_mlp_shape": ([_vp, _vp, _vp], _i32),
    "lpsim_mlp_forward": ([_vp, _vp, _vp, _vp, _vp, _i64, _vp], _i32),
    "lpsim_mlp_loss_grad": ([_vp, _vp, _vp, _i64, ctypes.c_float, _vp, _vp, _vp], _i32),
    "lpsim_mlp_workspace_bytes": ([_i64, _i32], ctypes.c_size_t),
    "lpsim_mlp_backward": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp, _i32, _i64, _vp], _i32),
    "lpsim_mlp_backward_noalloc": ([_vp, _vp, _vp, _vp, _vp, _vp, _i32, _i64, _vp], _i32),
    "lpsim_mlp_adam": ([_vp, _vp, _vp, _vp, _vp, _vp, _i32, _i32, ctypes.c_float, ctypes.c_float,
                        ctypes.c_float, ctypes.c_float, _i32, _vp], _i32),
    "lpsim_last_error": ([_vp], ctypes.c_char_p),
}


def load_library():
    """Load liblpsim.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2406_08496_amd.build")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(int(stream.cuda_stream))  # torch.cuda.Stream


class Simulator:
    """One GPU simulation context (one scenario or a batch)."""

    def __init__(self, **params):
        lib = load_library()
        kw = dict(DEFAULT_PARAMS)
        kw.update(params)
        self.params = kw
        self._pp = Params(**kw)
        h = ctypes.c_void_p()
        rc = lib.lpsim_create(ctypes.byref(self._pp), ctypes.byref(h))
        if rc != OK:
            raise LpsimError(rc, "lpsim_create failed (no usable GPU or bad parameters)")
        self._h = h
        self.n_edges = 0
        self.n_trips = 0

    # -- plumbing
    def _check(self, rc):
        if rc != OK:
            msg = load_library().lpsim_last_error(self._h)
            raise LpsimError(rc, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "_h", None):
            load_library().lpsim_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- loading
    def load_network(self, n_nodes, src, dst, length, lanes, speed, node_xy=None):
        src = np.ascontiguousarray(src, np.int32)
        dst = np.ascontiguousarray(dst, np.int32)
        length = np.ascontiguousarray(length, np.float32)
        lanes = np.ascontiguousarray(lanes, np.uint8)
        speed = np.ascontiguousarray(speed, np.float32)
        xy = None if node_xy is None else np.ascontiguousarray(node_xy, np.float32)
        self._check(load_library().lpsim_load_network(
            self._h, int(n_nodes), _p(xy), len(src), _p(src), _p(dst), _p(length), _p(lanes), _p(speed)))
        self.n_edges = len(src)

    def load_trips(self, depart_step, route_off, route_edges):
        d = np.ascontiguousarray(depart_step, np.int32)
        o = np.ascontiguousarray(route_off, np.int64)
        r = np.ascontiguousarray(route_edges, np.int32)
        if len(r) == 0:
            r = np.zeros(1, np.int32)
        self._check(load_library().lpsim_load_trips(self._h, len(d), _p(d), _p(o), _p(r)))
        self.n_trips = len(d)

    def load(self, inst, reorder=True):
        self.load_network(inst.n_nodes, inst.src, inst.dst, inst.length, inst.lanes, inst.speed,
                          node_xy=inst.node_xy if reorder else None)
        self.load_trips(inst.depart_step, inst.route_off, inst.route_edges)
        return self

    def load_batch(self, insts, seeds=None, reorder=True):
        """Independent scenarios in one context (arrays concatenated)."""
        S = len(insts)
        node_off = np.zeros(S + 1, np.int32)
        edge_off = np.zeros(S + 1, np.int32)
        trip_off = np.zeros(S + 1, np.int64)
        node_off[1:] = np.cumsum([i.n_nodes for i in insts])
        edge_off[1:] = np.cumsum([i.n_edges for i in insts])
        trip_off[1:] = np.cumsum([i.n_trips for i in insts])
        cat = lambda f, dt: np.ascontiguousarray(np.concatenate([f(i) for i in insts]), dt)
        xy = cat(lambda i: i.node_xy.reshape(-1), np.float32) if reorder else None
        src, dst = cat(lambda i: i.src, np.int32), cat(lambda i: i.dst, np.int32)
        length, lanes = cat(lambda i: i.length, np.float32), cat(lambda i: i.lanes, np.uint8)
        speed = cat(lambda i: i.speed, np.float32)
        dep = cat(lambda i: i.depart_step, np.int32)
        roff = cat(lambda i: i.route_off, np.int64)
        redges = cat(lambda i: i.route_edges, np.int32)
        sd = None if seeds is None else np.ascontiguousarray(seeds, np.uint64)
        self._check(load_library().lpsim_batch_load(
            self._h, S, _p(node_off), _p(edge_off), _p(trip_off), _p(xy), _p(src), _p(dst),
            _p(length), _p(lanes), _p(speed), _p(dep), _p(roff), _p(redges), _p(sd)))
        self.n_edges = int(edge_off[-1])
        self.n_trips = int(trip_off[-1])
        self.trip_off, self.edge_off = trip_off, edge_off
        return self

    # -- running
    def block_edge(self, e, on=True):
        self._check(load_library().lpsim_block_edge(self._h, int(e), 1 if on else 0))

    def set_signals(self, plan):
        """Fixed-time signal plan with fields n_phases, green, allred, offset
        (per node) and edge_phase (per edge), or None to remove it."""
        if plan is None:
            self._check(load_library().lpsim_set_signals(self._h, None, None, None, None, None))
            return
        arrs = [np.ascontiguousarray(getattr(plan, k), np.int32)
                for k in ("n_phases", "green", "allred", "offset", "edge_phase")]
        self._check(load_library().lpsim_set_signals(self._h, *[_p(a) for a in arrs]))

    def set_launch(self, block_size=512, n_blocks=640, graph_steps=64):
        self._check(load_library().lpsim_set_launch(self._h, block_size, n_blocks, graph_steps))

    def step(self, n=1, stream=None):
        self._check(load_library().lpsim_step(self._h, int(n), _stream_handle(stream)))

    def prepare(self, n):
        """Capture the graphs a step(n) call made next would launch."""
        self._check(load_library().lpsim_prepare_steps(self._h, int(n)))

    def autotune(self, n_steps=64, block_sizes=(256, 512),
                 block_counts=(512, 640, 768, 1024, 1280, 1536, 2048)):
        """Pick the fastest launch shape on the current state (state unchanged)."""
        bs = np.ascontiguousarray(block_sizes, np.int32)
        bc = np.ascontiguousarray(block_counts, np.int32)
        best = np.zeros(3, np.int32)
        trials = np.zeros(len(bs) * len(bc), np.float64)
        self._check(load_library().lpsim_autotune(self._h, int(n_steps), _p(bs), len(bs), _p(bc),
                                                  len(bc), _p(best), _p(trials)))
        return {"block_size": int(best[0]), "blocks": int(best[1]),
                "us_per_step": {(int(b), int(g)): float(trials[i * len(bc) + j])
                                for i, b in enumerate(bs) for j, g in enumerate(bc)}}

    def set_timing(self, on=True):
        self._check(load_library().lpsim_set_timing(self._h, 1 if on else 0))

    def kernel_times(self):
        ms = np.zeros(len(PHASES), np.float64)
        cnt = np.zeros(len(PHASES), np.int64)
        self._check(load_library().lpsim_kernel_times(self._h, _p(ms), _p(cnt), len(PHASES)))
        return {ph: (float(ms[i]), int(cnt[i])) for i, ph in enumerate(PHASES)}

    # -- read-back
    @property
    def W(self):
        return load_library().lpsim_query(self._h, 0)

    @property
    def D(self):
        return load_library().lpsim_query(self._h, 1)

    def vehicles(self):
        n = self.n_trips
        out = dict(edge=np.empty(n, np.int32), lane=np.empty(n, np.uint8),
                   cell=np.empty(n, np.int32), x=np.empty(n, np.float32),
                   v=np.empty(n, np.float32), arrival_step=np.empty(n, np.int32),
                   status=np.empty(n, np.uint8))
        self._check(load_library().lpsim_get_vehicles(self._h, *[_p(out[k]) for k in (
            "edge", "lane", "cell", "x", "v", "arrival_step", "status")]))
        return out

    def edge_stats(self, binned=True, device=False):
        """Per-edge statistics in input edge order (lpsim_edge_stats).  With
        device=True the binned arrays are torch tensors on the GPU, written
        by kernels queued on the current stream (lpsim_edge_stats_device);
        the unbinned ones are host arrays either way."""
        E, B = self.n_edges, self.params["n_bins"]
        out = dict(tt_sum=np.empty(E, np.int64), n_exits=np.empty(E, np.int32))
        if binned and not device:
            out.update(inflow_bin=np.empty((E, B), np.int32), exits_bin=np.empty((E, B), np.int32),
                       tt_bin=np.empty((E, B), np.int64), occ_bin=np.empty((E, B), np.int64))
        g = lambda k: _p(out.get(k))
        self._check(load_library().lpsim_edge_stats(self._h, g("tt_sum"), g("n_exits"), g("inflow_bin"),
                                                    g("exits_bin"), g("tt_bin"), g("occ_bin")))
        if binned and device:
            import torch

            t = dict(inflow_bin=torch.empty((E, B), dtype=torch.int32, device="cuda"),
                     exits_bin=torch.empty((E, B), dtype=torch.int32, device="cuda"),
                     tt_bin=torch.empty((E, B), dtype=torch.int64, device="cuda"),
                     occ_bin=torch.empty((E, B), dtype=torch.int64, device="cuda"))
            vp = lambda k: ctypes.c_void_p(t[k].data_ptr())
            self._check(load_library().lpsim_edge_stats_device(
                self._h, vp("inflow_bin"), vp("exits_bin"), vp("tt_bin"), vp("occ_bin"),
                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
            out.update(t)
        return out

    def counters(self):
        c = Counters()
        self._check(load_library().lpsim_get_counters(self._h, ctypes.byref(c)))
        return {n: int(getattr(c, n)) for n, _ in Counters._fields_}

    def save_state(self):
        n = ctypes.c_size_t()
        self._check(load_library().lpsim_state_size(self._h, ctypes.byref(n)))
        buf = np.empty(n.value, np.uint8)
        self._check(load_library().lpsim_save_state(self._h, _p(buf), n.value))
        return buf

    def restore_state(self, buf):
        buf = np.ascontiguousarray(buf, np.uint8)
        self._check(load_library().lpsim_restore_state(self._h, _p(buf), buf.nbytes))
