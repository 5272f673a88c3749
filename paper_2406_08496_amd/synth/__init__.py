"""Seeded synthetic instances: road networks and routed demand.

The paper's workloads (the SF Bay network and the SFCTA demand, Section 4.1)
are not available, so every input here is generated from a seed with the
shapes the paper describes: a planar regional road graph of about 225k nodes
and 550k directed edges (Section 1) and about 2.8M routed car trips
(abstract).  Demand arrives already routed, as the method expects
(Section 3.1, data layout: route and first edge per vehicle), and trips are
sorted by departure time before ids are assigned (Section 4.2, sorting study).

This module holds no simulation arithmetic.  It is the one piece shared by the
CPU oracle and the GPU path: both read the same instance.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROUTING_SO = os.path.join(_HERE, "_routing.so")
_lib = None

SPEEDS_CFG = np.array([13.4, 17.9, 22.4], dtype=np.float32)


def build_routing(force: bool = True) -> str:
    """Compile the routing helper (plain C, OpenMP)."""
    import subprocess

    src = os.path.join(_HERE, "routing.c")
    if force or not os.path.exists(_ROUTING_SO):
        tmp = _ROUTING_SO + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", src, "-o", tmp]
        )
        os.replace(tmp, _ROUTING_SO)
    return _ROUTING_SO


def _routing():
    global _lib
    if _lib is None:
        if not os.path.exists(_ROUTING_SO):
            build_routing(force=False)
        _lib = ctypes.CDLL(_ROUTING_SO)
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Instance:
    """A network plus routed demand.  Edge e runs src[e] -> dst[e]."""

    n_nodes: int
    node_xy: np.ndarray  # float32 [n_nodes, 2]
    src: np.ndarray  # int32 [E]
    dst: np.ndarray  # int32 [E]
    length: np.ndarray  # float32 [E], integer metres
    lanes: np.ndarray  # uint8 [E]
    speed: np.ndarray  # float32 [E], m/s
    depart_step: np.ndarray  # int32 [N]
    route_off: np.ndarray  # int64 [N+1]
    route_edges: np.ndarray  # int32 [route_off[-1]]
    n_steps: int = 0  # horizon in steps
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_edges(self) -> int:
        return int(self.src.shape[0])

    @property
    def n_trips(self) -> int:
        return int(self.depart_step.shape[0])

    def route(self, i: int) -> np.ndarray:
        return self.route_edges[self.route_off[i]: self.route_off[i + 1]]


# ----------------------------------------------------------------------------
# routing

def in_csr(n_nodes: int, dst: np.ndarray):
    order = np.argsort(dst, kind="stable").astype(np.int32)
    counts = np.bincount(dst, minlength=n_nodes)
    off = np.zeros(n_nodes + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    return off, order


def route_trips(n_nodes, src, dst, length, speed, origin, dest_node):
    """Shortest-time routes (fp64 length/speed, ties to the lower edge id).

    Returns (route_off int64[N+1], route_edges int32[...]).
    """
    lib = _routing()
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    w = np.ascontiguousarray(
        length.astype(np.float64) / speed.astype(np.float64), dtype=np.float64
    )
    dests, dest_idx = np.unique(dest_node, return_inverse=True)
    dests = dests.astype(np.int32)
    dest_idx = dest_idx.astype(np.int32)
    off, order = in_csr(n_nodes, dst)
    nxt = np.empty((len(dests), n_nodes), dtype=np.int32)
    rc = lib.synth_route_trees(
        ctypes.c_int32(n_nodes), ctypes.c_int32(len(src)), _p(src), _p(dst), _p(w),
        _p(off), _p(order), ctypes.c_int32(len(dests)), _p(dests), _p(nxt),
    )
    if rc != 0:
        raise MemoryError("routing trees failed")
    origin = np.ascontiguousarray(origin, dtype=np.int32)
    n = len(origin)
    lens = np.empty(n, dtype=np.int32)
    rc = lib.synth_route_lengths(
        ctypes.c_int32(n_nodes), _p(dst), _p(nxt), _p(dests), ctypes.c_int64(n),
        _p(origin), _p(dest_idx), _p(lens),
    )
    if rc != 0:
        raise ValueError("some trip has no route (unreachable or origin == destination)")
    route_off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=route_off[1:])
    route_edges = np.empty(int(route_off[-1]), dtype=np.int32)
    lib.synth_route_fill(
        ctypes.c_int32(n_nodes), _p(dst), _p(nxt), _p(dests), ctypes.c_int64(n),
        _p(origin), _p(dest_idx), _p(route_off), _p(route_edges),
    )
    return route_off, route_edges


def sort_trips(depart_step, origin, dest):
    """Trip ids are ranks after sorting by (departure, origin, destination)."""
    order = np.lexsort((dest, origin, depart_step))
    return depart_step[order], origin[order], dest[order]


def streets_to_edges(a, b, rng, length_fn, lanes_fn):
    """Undirected streets (a[s], b[s]) -> directed edges 2s: a->b, 2s+1: b->a.

    Length, lanes and speed limit are drawn per street, equal both ways.
    """
    ns = len(a)
    length = length_fn(ns)
    lanes = lanes_fn(ns)
    speed = SPEEDS_CFG[rng.integers(0, 3, size=ns)]
    src = np.empty(2 * ns, np.int32)
    dst = np.empty(2 * ns, np.int32)
    src[0::2], dst[0::2] = a, b
    src[1::2], dst[1::2] = b, a
    rep = lambda x: np.repeat(x, 2)
    return src, dst, rep(length).astype(np.float32), rep(lanes).astype(np.uint8), rep(speed).astype(np.float32)


# ----------------------------------------------------------------------------
# grid instance (16x16, 2,000 trips)

def grid_instance(seed: int = 1, side: int = 16, n_trips: int = 2000,
                  depart_window: int = 1200, n_steps: int = 7200,
                  lanes: int = 2, len_lo: int = 100, len_hi: int = 500,
                  speeds=None) -> Instance:
    """side x side grid, 4-neighbour streets, integer lengths U[len_lo, len_hi],
    speed limit per street from {13.4, 17.9, 22.4} m/s (or `speeds`), uniform
    random OD pairs (origin != destination), departures uniform in
    [0, depart_window) steps."""
    rng = np.random.default_rng(seed)
    n_nodes = side * side
    a, b = [], []
    for i in range(side):
        for j in range(side):
            u = i * side + j
            if j + 1 < side:
                a.append(u); b.append(u + 1)
            if i + 1 < side:
                a.append(u); b.append(u + side)
    a = np.array(a, np.int32)
    b = np.array(b, np.int32)
    src, dst, length, ln, sp = streets_to_edges(
        a, b, rng,
        lambda ns: rng.integers(len_lo, len_hi + 1, size=ns).astype(np.float32),
        lambda ns: np.full(ns, lanes, np.uint8),
    )
    if speeds is not None:
        sp = np.repeat(np.asarray(speeds, np.float32)[rng.integers(0, len(speeds), size=len(a))], 2)
    xy = np.stack(np.meshgrid(np.arange(side), np.arange(side), indexing="ij"), -1)
    xy = xy.reshape(-1, 2)[:, ::-1].astype(np.float32)  # (x=j, y=i)
    origin = rng.integers(0, n_nodes, size=n_trips).astype(np.int32)
    dest = rng.integers(0, n_nodes - 1, size=n_trips).astype(np.int32)
    dest = np.where(dest >= origin, dest + 1, dest).astype(np.int32)
    dep = rng.integers(0, depart_window, size=n_trips).astype(np.int32)
    dep, origin, dest = sort_trips(dep, origin, dest)
    route_off, route_edges = route_trips(n_nodes, src, dst, length, sp, origin, dest)
    return Instance(n_nodes, xy, src, dst, length, ln, sp, dep, route_off,
                    route_edges, n_steps=n_steps, name=f"grid{side}x{side}-{n_trips}",
                    meta={"origin": origin, "dest": dest})


# ----------------------------------------------------------------------------
# planar regional instances (Delaunay + MST + extras, gravity demand)

def planar_network(seed: int, nx: int, ny: int, n_undirected: int,
                   jitter: float = 0.35):
    """Jittered nx x ny lattice, Delaunay triangulation, Euclidean MST plus
    random extra Delaunay edges up to n_undirected streets.  Lengths are
    lognormal(ln 150, 0.5) clamped to [20, 2000] m (integer), lanes uniform in
    {1..4}, speed limit per street from {13.4, 17.9, 22.4} m/s."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import minimum_spanning_tree
    from scipy.spatial import Delaunay

    rng = np.random.default_rng(seed)
    gx, gy = np.meshgrid(np.arange(nx, dtype=np.float64), np.arange(ny, dtype=np.float64), indexing="xy")
    xy = np.stack([gx.ravel(), gy.ravel()], 1)
    xy += rng.uniform(-jitter, jitter, size=xy.shape)
    n = xy.shape[0]
    tri = Delaunay(xy)
    s = tri.simplices
    pairs = np.concatenate([s[:, [0, 1]], s[:, [1, 2]], s[:, [0, 2]]], 0)
    pairs.sort(axis=1)
    key = pairs[:, 0].astype(np.int64) * n + pairs[:, 1]
    key = np.unique(key)
    pa = (key // n).astype(np.int32)
    pb = (key % n).astype(np.int32)
    d = np.hypot(xy[pa, 0] - xy[pb, 0], xy[pa, 1] - xy[pb, 1])
    g = coo_matrix((d, (pa, pb)), shape=(n, n)).tocsr()
    mst = minimum_spanning_tree(g).tocoo()
    ma = np.minimum(mst.row, mst.col).astype(np.int64)
    mb = np.maximum(mst.row, mst.col).astype(np.int64)
    mkey = np.unique(ma * n + mb)
    rest = np.setdiff1d(key, mkey, assume_unique=True)
    n_extra = max(0, min(len(rest), n_undirected - len(mkey)))
    extra = rng.choice(rest, size=n_extra, replace=False)
    skey = np.sort(np.concatenate([mkey, extra]))
    a = (skey // n).astype(np.int32)
    b = (skey % n).astype(np.int32)

    def lengths(ns):
        l = np.exp(rng.normal(np.log(150.0), 0.5, size=ns))
        return np.rint(np.clip(l, 20.0, 2000.0)).astype(np.float32)

    src, dst, length, ln, sp = streets_to_edges(
        a, b, rng, lengths, lambda ns: rng.integers(1, 5, size=ns).astype(np.uint8)
    )
    return n, xy.astype(np.float32), src, dst, length, ln, sp, rng


def gravity_demand(rng, xy, nx, ny, n_trips, zx, zy, peaks_min, sigma_min,
                   window_min, dt, dist_scale=40.0):
    """Gravity OD over zx*zy rectangular zones.  T_ij ~ P_i A_j exp(-d_ij/40)
    with P, A lognormal(0, 0.5); origin uniform among the nodes of zone i,
    destination the centroid (node nearest the cell centre) of zone j.
    Departures: equal mixture of normals at `peaks_min`, truncated to
    [0, window_min)."""
    from scipy.spatial import cKDTree

    n = xy.shape[0]
    cw, ch = nx / zx, ny / zy
    cx = np.clip(np.floor((xy[:, 0] + 0.5) / cw), 0, zx - 1).astype(np.int64)
    cy = np.clip(np.floor((xy[:, 1] + 0.5) / ch), 0, zy - 1).astype(np.int64)
    zone = (cy * zx + cx).astype(np.int64)
    nz = zx * zy
    centres = np.stack(np.meshgrid((np.arange(zx) + 0.5) * cw - 0.5,
                                   (np.arange(zy) + 0.5) * ch - 0.5, indexing="xy"), -1).reshape(-1, 2)
    centroid = cKDTree(xy).query(centres)[1].astype(np.int32)
    P = rng.lognormal(0.0, 0.5, size=nz)
    A = rng.lognormal(0.0, 0.5, size=nz)
    dzz = np.hypot(centres[:, None, 0] - centres[None, :, 0], centres[:, None, 1] - centres[None, :, 1])
    T = P[:, None] * A[None, :] * np.exp(-dzz / dist_scale)
    T = (T / T.sum()).ravel()
    counts = rng.multinomial(n_trips, T)
    od = np.repeat(np.arange(nz * nz), counts)
    zi, zj = od // nz, od % nz
    order = np.argsort(zone, kind="stable")
    zcount = np.bincount(zone, minlength=nz)
    zoff = np.zeros(nz + 1, np.int64)
    np.cumsum(zcount, out=zoff[1:])
    if np.any(zcount[np.unique(zi)] == 0):
        raise ValueError("empty origin zone")
    dest = centroid[zj]
    origin = np.empty(n_trips, np.int32)
    todo = np.arange(n_trips)
    while len(todo):
        zz = zi[todo]
        pick = zoff[zz] + (rng.random(len(todo)) * zcount[zz]).astype(np.int64)
        origin[todo] = order[pick]
        todo = todo[origin[todo] == dest[todo]]
    # departures: two-peak mixture, truncated
    t = np.empty(n_trips)
    todo = np.arange(n_trips)
    while len(todo):
        comp = rng.integers(0, len(peaks_min), size=len(todo))
        t[todo] = rng.normal(np.asarray(peaks_min)[comp], sigma_min) * 60.0
        todo = todo[(t[todo] < 0) | (t[todo] >= window_min * 60.0)]
    dep = np.floor(t / dt).astype(np.int32)
    return origin, dest.astype(np.int32), dep, centroid, zone


def planar_instance(seed: int, nx: int, ny: int, n_undirected: int, n_trips: int,
                    zones=(25, 20), peaks_min=(60.0, 120.0), sigma_min=20.0,
                    window_min=180.0, n_steps=28800, dt=0.5, name="planar") -> Instance:
    n, xy, src, dst, length, ln, sp, rng = planar_network(seed, nx, ny, n_undirected)
    origin, dest, dep, centroid, zone = gravity_demand(
        rng, xy, nx, ny, n_trips, zones[0], zones[1], peaks_min, sigma_min, window_min, dt
    )
    dep, origin, dest = sort_trips(dep, origin, dest)
    route_off, route_edges = route_trips(n, src, dst, length, sp, origin, dest)
    return Instance(n, xy, src, dst, length, ln, sp, dep, route_off, route_edges,
                    n_steps=n_steps, name=name,
                    meta={"origin": origin, "dest": dest, "centroid": centroid, "zone": zone})


# ----------------------------------------------------------------------------
# the named workloads

def tiny_grid() -> Instance:
    """16x16 grid, 960 directed edges, 2 lanes, 2,000 trips, 3,600 s at dt=0.5."""
    return grid_instance(seed=1)


def regional(scale: float = 1.0, demand: float = 1.0) -> Instance:
    """Planar regional graph: 475x474 jittered lattice (225,150 nodes), 550,000
    directed edges, 2.82M gravity trips over a two-peak 3 h morning profile,
    horizon 3 h + 1 h drain.  `scale` < 1 shrinks every size (for tests);
    `demand` scales only the number of trips (same network)."""
    if scale == 1.0:
        n = int(round(2_820_000 * demand))
        name = "regional-225k-2.82M" if demand == 1.0 else f"regional-225k-{n / 1e6:.3g}M"
        return planar_instance(2, 475, 474, 275_000, n, name=name)
    side = max(8, int(round(475 * np.sqrt(scale))))
    nodes = side * side
    return planar_instance(2, side, side, int(nodes * 275_000 / 225_150),
                           max(10, int(2_820_000 * scale * demand)),
                           zones=(max(2, int(25 * np.sqrt(scale))), max(2, int(20 * np.sqrt(scale)))),
                           name=f"regional-x{scale}" + ("" if demand == 1.0 else f"-d{demand}"))


def large(scale: float = 1.0) -> Instance:
    """1000x1000 lattice (1M nodes), 2.5M directed edges, 9M trips, peaks at
    80 and 160 min (sigma 25) over 4 h, horizon 5 h."""
    side = max(8, int(round(1000 * np.sqrt(scale))))
    return planar_instance(3, side, side, int(1_250_000 * scale), max(10, int(9_000_000 * scale)),
                           peaks_min=(80.0, 160.0), sigma_min=25.0, window_min=240.0,
                           n_steps=36000, name=f"large-x{scale}")


def batch_scenarios(n_scen: int = 64, seed: int = 4, node_range=(8_000, 60_000),
                    trip_range=(10_000, 500_000), n_steps: int = 14400, scale: float = 1.0):
    """Independent scenarios with log-uniform node and trip counts, each its
    own planar graph and two-peak demand over 90 min."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(n_scen):
        nodes = int(np.exp(rng.uniform(np.log(node_range[0]), np.log(node_range[1]))) * scale)
        trips = int(np.exp(rng.uniform(np.log(trip_range[0]), np.log(trip_range[1]))) * scale)
        side = max(6, int(round(np.sqrt(max(nodes, 36)))))
        nodes = side * side
        zones = max(20, nodes // 450)
        zx = max(2, int(round(np.sqrt(zones * 1.25))))
        zy = max(2, zones // zx)
        out.append(planar_instance(seed + s, side, side, int(nodes * 275_000 / 225_150),
                                   max(10, trips), zones=(zx, zy), peaks_min=(30.0, 60.0),
                                   sigma_min=15.0, window_min=90.0, n_steps=n_steps,
                                   name=f"scen{s}"))
    return out


def line_instance(lengths, speeds, lanes, departs, routes, n_nodes=None,
                  extra_edges=()) -> Instance:
    """Hand-built instance for closed-form cases.

    `lengths/speeds/lanes` describe a chain of edges 0..m-1 (node i -> i+1);
    `extra_edges` adds (src, dst, length, speed, lanes) tuples.  `routes` is a
    list of edge-id lists, one per trip, `departs` their departure steps (trips
    are NOT re-sorted: ids are list positions).
    """
    m = len(lengths)
    src = list(range(m))
    dst = list(range(1, m + 1))
    length = list(lengths)
    speed = list(speeds)
    ln = list(lanes)
    nn = m + 1
    for (a, b, L, v, l) in extra_edges:
        src.append(a); dst.append(b); length.append(L); speed.append(v); ln.append(l)
        nn = max(nn, a + 1, b + 1)
    if n_nodes is not None:
        nn = max(nn, n_nodes)
    off = np.zeros(len(routes) + 1, np.int64)
    off[1:] = np.cumsum([len(r) for r in routes])
    re = np.array([e for r in routes for e in r], np.int32)
    xy = np.stack([np.arange(nn, dtype=np.float32), np.zeros(nn, np.float32)], 1)
    return Instance(nn, xy, np.array(src, np.int32), np.array(dst, np.int32),
                    np.array(length, np.float32), np.array(ln, np.uint8),
                    np.array(speed, np.float32), np.array(departs, np.int32), off, re,
                    name="hand")


# ----------------------------------------------------------------------------
# fixed-time signal plans

@dataclass
class SignalPlan:
    """Fixed-time signals: per node the number of phases (0 = no signal),
    green and all-red steps per phase and the cycle offset in steps; per edge
    the phase of its downstream node that serves it (-1 = none)."""

    n_phases: np.ndarray  # int32 [n_nodes]
    green: np.ndarray  # int32 [n_nodes]
    allred: np.ndarray  # int32 [n_nodes]
    offset: np.ndarray  # int32 [n_nodes]
    edge_phase: np.ndarray  # int32 [E]

    @property
    def n_signals(self) -> int:
        return int((self.n_phases > 0).sum())


def signal_plan(inst: Instance, seed: int = 7, green_s: float = 40.0, allred_s: float = 5.0,
                min_in: int = 3, dt: float = 0.5) -> SignalPlan:
    """Two-phase fixed-time signals at every node with at least `min_in`
    incoming edges: approaches arriving mostly along x are served in phase 0,
    mostly along y in phase 1 (a node whose approaches all share one axis gets
    no signal).  Cycle offsets are uniform over the cycle, seeded."""
    rng = np.random.default_rng(seed)
    n, E = inst.n_nodes, inst.n_edges
    xy = inst.node_xy.astype(np.float64)
    dxy = xy[inst.dst] - xy[inst.src]
    axis = np.where(np.abs(dxy[:, 0]) >= np.abs(dxy[:, 1]), 0, 1).astype(np.int32)
    indeg = np.bincount(inst.dst, minlength=n)
    has = np.zeros((n, 2), bool)
    has[inst.dst, axis] = True
    sig = (indeg >= min_in) & has[:, 0] & has[:, 1]
    green = max(1, int(round(green_s / dt)))
    allred = max(0, int(round(allred_s / dt)))
    cycle = 2 * (green + allred)
    n_phases = np.where(sig, 2, 0).astype(np.int32)
    offset = np.where(sig, rng.integers(0, cycle, size=n), 0).astype(np.int32)
    edge_phase = np.where(sig[inst.dst], axis, -1).astype(np.int32)
    return SignalPlan(n_phases, np.where(sig, green, 0).astype(np.int32),
                      np.where(sig, allred, 0).astype(np.int32), offset, edge_phase)


def concat_signal_plans(plans, insts) -> SignalPlan:
    """One plan over a batch's concatenated nodes and edges."""
    return SignalPlan(*[np.concatenate([getattr(p, k) for p in plans]).astype(np.int32)
                        for k in ("n_phases", "green", "allred", "offset", "edge_phase")])
