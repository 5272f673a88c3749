"""The assignment loop's shortest-time router (host code in the library):
route costs equal Dijkstra distances from an independent library routine,
routes are contiguous and end at their destination, ties go to the lower
edge id, and old routes are kept where asked."""
import ctypes

import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import dijkstra

from paper_2406_08496_amd import synth
from paper_2406_08496_amd.assign import Router
from paper_2406_08496_amd.lpsim import LpsimError


def check_routes(inst, cost, origin, dest, off, edges):
    n = inst.n_nodes
    # shortest distance to each destination (reverse graph), independent routine
    g = csr_matrix((cost, (inst.dst, inst.src)), shape=(n, n))
    # parallel edges: keep the cheaper one (csr would sum duplicates)
    order = np.lexsort((cost, inst.dst, inst.src))
    key = inst.src[order].astype(np.int64) * n + inst.dst[order]
    first = np.ones(len(order), bool)
    first[1:] = key[1:] != key[:-1]
    o = order[first]
    g = csr_matrix((cost[o], (inst.dst[o], inst.src[o])), shape=(n, n))
    dests = np.unique(dest)
    dist = dijkstra(g, indices=dests)
    di = np.searchsorted(dests, dest)
    for i in range(len(origin)):
        r = edges[off[i]:off[i + 1]]
        assert len(r) > 0
        assert inst.src[r[0]] == origin[i] and inst.dst[r[-1]] == dest[i]
        assert np.all(inst.dst[r[:-1]] == inst.src[r[1:]])
        assert abs(cost[r].sum() - dist[di[i], origin[i]]) <= 1e-9 * max(1.0, dist[di[i], origin[i]])


def test_routes_are_shortest_on_grid():
    inst = synth.grid_instance(seed=4, side=7, n_trips=300)
    rng = np.random.default_rng(0)
    cost = (inst.length / inst.speed).astype(np.float64) * rng.uniform(0.5, 3.0, size=inst.n_edges)
    o, d = inst.meta["origin"], inst.meta["dest"]
    r = Router(inst.n_nodes, inst.src, inst.dst, n_threads=4)
    off, edges = r.routes(cost, o, d)
    check_routes(inst, cost, o, d, off, edges)


def test_routes_match_generator_free_flow():
    """With free-flow costs the router reproduces the generator's routes
    (both take ties to the lower edge id)."""
    inst = synth.regional(0.003)
    cost = inst.length.astype(np.float64) / inst.speed.astype(np.float64)
    r = Router(inst.n_nodes, inst.src, inst.dst)
    off, edges = r.routes(cost, inst.meta["origin"], inst.meta["dest"])
    assert np.array_equal(off, inst.route_off) and np.array_equal(edges, inst.route_edges)


def test_ties_go_to_lower_edge_id():
    # two parallel two-edge paths 0->1->3 and 0->2->3 with equal cost
    src = np.array([0, 1, 0, 2], np.int32)
    dst = np.array([2, 3, 1, 3], np.int32)
    cost = np.ones(4)
    r = Router(4, src, dst, n_threads=1)
    off, edges = r.routes(cost, np.array([0], np.int32), np.array([3], np.int32))
    # path via node 2 uses edges 0 then 3; via node 1 uses 2 then 1: first edge 0 < 2
    assert list(edges) == [0, 3]


def test_keep_old_routes_and_errors():
    inst = synth.grid_instance(seed=5, side=5, n_trips=50)
    cost = (inst.length / inst.speed).astype(np.float64) * 2.0
    cost[inst.route_edges[:3]] *= 10.0
    o, d = inst.meta["origin"], inst.meta["dest"]
    r = Router(inst.n_nodes, inst.src, inst.dst)
    take = np.zeros(50, np.uint8)
    take[::2] = 1
    off, edges = r.routes(cost, o, d, old=(inst.route_off, inst.route_edges), take_new=take)
    for i in range(1, 50, 2):
        assert np.array_equal(edges[off[i]:off[i + 1]], inst.route(i))
    with pytest.raises(LpsimError):
        r.routes(-cost, o, d)
    with pytest.raises(LpsimError):
        r.routes(cost, o, o)


def test_msa_switch_share():
    """The deterministic switch picks about 1/(n+1) of the trips (binomial
    tolerance) and differs between iterations."""
    from paper_2406_08496_amd.assign import msa_switch

    N = 200_000
    prev = None
    for n in (1, 2, 5, 29):
        s = msa_switch(N, n, 0xA55)
        p = 1.0 / (n + 1)
        assert abs(s.mean() - p) <= 5 * np.sqrt(p * (1 - p) / N)
        if prev is not None:
            assert not np.array_equal(s, prev)
        prev = s


def test_fill_in_one_call():
    """Writing the edges without a sizing call first gives the same routes
    (the lengths are measured on every call)."""
    inst = synth.grid_instance(seed=6, side=6, n_trips=400)
    cost = (inst.length / inst.speed).astype(np.float64)
    origin = np.ascontiguousarray(inst.meta["origin"], np.int32)
    dest = np.ascontiguousarray(inst.meta["dest"], np.int32)
    r = Router(inst.n_nodes, inst.src, inst.dst, n_threads=3)
    take = (np.arange(inst.n_trips) % 3 == 0).astype(np.uint8)
    old = (np.ascontiguousarray(inst.route_off, np.int64), np.ascontiguousarray(inst.route_edges, np.int32))
    off2, edges2 = r.routes(cost * 1.7, origin, dest, old=old, take_new=take)
    # a fresh solve, then one call with a buffer sized by the two-call result
    vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    c2 = np.ascontiguousarray(cost * 1.7)
    assert r.lib.lpsim_router_solve(r._h, vp(c2), inst.n_trips, vp(origin), vp(dest)) == 0
    off1 = np.zeros(inst.n_trips + 1, np.int64)
    edges1 = np.zeros(len(edges2), np.int32)
    assert r.lib.lpsim_router_fill(r._h, vp(old[0]), vp(old[1]), vp(take), vp(off1), vp(edges1)) == 0
    assert np.array_equal(off1, off2) and np.array_equal(edges1, edges2)


def test_routes_into_a_reused_buffer():
    """routes(out=...) writes into the caller's buffer when it is large
    enough and is not the old routes' memory, else into a new array with
    room to spare; the routes are the same either way."""
    inst = synth.grid_instance(seed=7, side=6, n_trips=300)
    cost = (inst.length / inst.speed).astype(np.float64) * np.linspace(1.0, 2.0, inst.n_edges)
    o, d = inst.meta["origin"], inst.meta["dest"]
    r = Router(inst.n_nodes, inst.src, inst.dst, n_threads=2)
    take = (np.arange(inst.n_trips) % 2 == 0).astype(np.uint8)
    old = (inst.route_off, inst.route_edges)
    want = r.routes(cost, o, d, old=old, take_new=take)
    # too small: a new array with room, whose base can be reused
    a = r.routes(cost, o, d, old=old, take_new=take, out=np.empty(0, np.int32))
    assert np.array_equal(a[0], want[0]) and np.array_equal(a[1], want[1])
    buf = a[1].base
    assert buf is not None and len(buf) > len(a[1])
    buf[:] = -5
    b = r.routes(cost, o, d, old=old, take_new=take, out=buf)
    assert np.shares_memory(b[1], buf)
    assert np.array_equal(b[0], want[0]) and np.array_equal(b[1], want[1])
    assert (buf[len(b[1]):] == -5).all()
    # the old routes' own memory is never written
    old2 = (b[0], b[1])
    c = r.routes(cost * 1.3, o, d, old=old2, take_new=take, out=buf)
    assert not np.shares_memory(c[1], buf)
    c_want = r.routes(cost * 1.3, o, d, old=(b[0].copy(), b[1].copy()), take_new=take)
    assert np.array_equal(c[0], c_want[0]) and np.array_equal(c[1], c_want[1])


def test_fill_refuses_to_overwrite_the_old_routes():
    """Writing the new routes over the old routes' memory, which the fill
    still reads, is an argument error (nothing is written), and so are old
    offsets that run backwards for a route that is kept."""
    inst = synth.grid_instance(seed=6, side=6, n_trips=200)
    cost = (inst.length / inst.speed).astype(np.float64) * 1.5
    origin = np.ascontiguousarray(inst.meta["origin"], np.int32)
    dest = np.ascontiguousarray(inst.meta["dest"], np.int32)
    r = Router(inst.n_nodes, inst.src, inst.dst, n_threads=2)
    take = (np.arange(inst.n_trips) % 2 == 0).astype(np.uint8)
    old_off = np.ascontiguousarray(inst.route_off, np.int64)
    buf = np.zeros(int(old_off[-1]) * 2 + 64, np.int32)
    buf[:old_off[-1]] = inst.route_edges
    vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    c = np.ascontiguousarray(cost)
    assert r.lib.lpsim_router_solve(r._h, vp(c), inst.n_trips, vp(origin), vp(dest)) == 0
    off = np.zeros(inst.n_trips + 1, np.int64)
    assert r.lib.lpsim_router_fill(r._h, vp(old_off), vp(buf), vp(take), vp(off), None) == 0
    keep = buf.copy()
    # out_edges starting inside the old routes
    out = buf[10:]
    assert r.lib.lpsim_router_fill(r._h, vp(old_off), vp(buf), vp(take), vp(off), vp(out)) != 0
    assert np.array_equal(buf, keep)
    # old offsets that run backwards for a kept route
    bad_off = old_off.copy()
    k = int(np.nonzero(take == 0)[0][0])
    bad_off[k + 1] = bad_off[k] - 1
    assert r.lib.lpsim_router_fill(r._h, vp(bad_off), vp(buf), vp(take), vp(off), None) != 0
    # the spare space after them is fine
    assert r.lib.lpsim_router_fill(r._h, vp(old_off), vp(buf), vp(take), vp(off), None) == 0
    out = buf[int(old_off[-1]):]
    assert off[-1] <= len(out)
    assert r.lib.lpsim_router_fill(r._h, vp(old_off), vp(buf), vp(take), vp(off), vp(out)) == 0
    want = r.routes(cost, origin, dest, old=(old_off, inst.route_edges.copy()), take_new=take)
    assert np.array_equal(off, want[0]) and np.array_equal(out[:off[-1]], want[1])


def test_fill_over_many_chunks():
    """More trips than one chunk of the fill's parallel prefix sums (65,536):
    the offsets equal a plain cumulative sum of the route lengths (new routes
    where taken, old ones elsewhere) and every route is where they say."""
    from paper_2406_08496_amd.assign import msa_switch

    inst = synth.grid_instance(seed=9, side=7, n_trips=150_000)
    o, d = inst.meta["origin"], inst.meta["dest"]
    r = Router(inst.n_nodes, inst.src, inst.dst, n_threads=4)
    cost = (inst.length / inst.speed).astype(np.float64) * np.linspace(1.0, 3.0, inst.n_edges)
    take = msa_switch(inst.n_trips, 2, 0x5EED)
    off, edges = r.routes(cost, o, d, old=(inst.route_off, inst.route_edges), take_new=take)
    new_off, new_edges = r.routes(cost, o, d)
    lens = np.where(take == 1, np.diff(new_off), np.diff(inst.route_off))
    assert off[0] == 0 and np.array_equal(off[1:], np.cumsum(lens))
    for i in list(range(0, inst.n_trips, 9973)) + [65535, 65536, 131072, inst.n_trips - 1]:
        want = new_edges[new_off[i]:new_off[i + 1]] if take[i] else inst.route_edges[inst.route_off[i]:inst.route_off[i + 1]]
        assert np.array_equal(edges[off[i]:off[i + 1]], want), i


def test_msa_switch_definition():
    """lpsim_msa_switch against its definition written out with Python
    integers: SplitMix64 of seed ^ i << 8 ^ n, modulo n + 1."""
    from paper_2406_08496_amd.assign import msa_switch

    M = (1 << 64) - 1

    def mix(z):
        z &= M
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        return z ^ (z >> 31)

    for n, seed in ((1, 0xA55), (7, 0xA55), (30, (1 << 63) + 12345)):
        s = msa_switch(3000, n, seed)
        want = [1 if mix(seed ^ (i << 8) ^ n) % (n + 1) == 0 else 0 for i in range(3000)]
        assert s.tolist() == want


def test_edge_travel_times_from_statistics():
    """Routing costs and per-bin times from the statistics (library host
    code) against their definitions."""
    from paper_2406_08496_amd.assign import _p
    from paper_2406_08496_amd.lpsim import load_library

    lib = load_library()
    rng = np.random.default_rng(2)
    E, B = 500, 12
    n = rng.integers(0, 5, E).astype(np.int32)
    tts = (n * rng.integers(0, 90, E)).astype(np.int64)
    free = rng.uniform(0.2, 40.0, E)
    out = np.empty(E)
    assert lib.lpsim_edge_tt(E, _p(tts), _p(n), _p(free), ctypes.c_double(0.5), _p(out)) == 0
    mean = np.where(n > 0, tts / np.maximum(n, 1), free)
    assert np.array_equal(out, np.maximum(mean, 1.0) * 0.5)
    ex = rng.integers(0, 4, (E, B)).astype(np.int32)
    ttb = (ex * rng.integers(1, 70, (E, B))).astype(np.int64)
    outb = np.empty((E, B), np.float32)
    assert lib.lpsim_edge_tt_bins(E, B, _p(ttb), _p(ex), _p(free), _p(outb)) == 0
    want = np.where(ex > 0, ttb / np.maximum(ex, 1), free[:, None]).astype(np.float32)
    assert np.array_equal(outb, want)
