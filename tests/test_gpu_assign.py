"""Surrogate data path and assignment loop on the GPU, against the oracle.

Loading is integer work and must match exactly; features are float32 results
rounded to bfloat16 and must match the float64 oracle within one bfloat16
step; targets and the damped travel-time update within float32 rounding."""
import ctypes

import numpy as np
import pytest

from oracle import assign as oa
from oracle import mlp
from paper_2406_08496_amd import synth

pytestmark = pytest.mark.gpu


def case(*a):
    print("CASE:", *a, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t

    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def vp(t):
    return ctypes.c_void_p(t.data_ptr())


@pytest.mark.parametrize("seed,n_bins,bin_steps,horizon", [(1, 12, 50, 700), (2, 24, 30, 400)])
def test_load_exact(torch, seed, n_bins, bin_steps, horizon):
    case("surrogate loading", seed, n_bins, bin_steps, horizon)
    from paper_2406_08496_amd.lpsim import load_library

    lib = load_library()
    inst = synth.grid_instance(seed=seed, side=5, n_trips=400, depart_window=300)
    rng = np.random.default_rng(seed)
    tt = rng.uniform(0.2, 60.0, size=(inst.n_edges, n_bins)).astype(np.float32)
    tt[rng.random(tt.shape) < 0.05] = 2.5  # exact ties of the rounding rule
    inflow_ref, occ_ref = oa.load(inst.route_off, inst.route_edges, inst.depart_step, tt, n_bins, bin_steps, horizon)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    inflow = torch.empty((inst.n_edges, n_bins), dtype=torch.int32, device="cuda")
    occ = torch.empty((inst.n_edges, n_bins), dtype=torch.int64, device="cuda")
    off, edges, dep, ttd = d(inst.route_off), d(inst.route_edges), d(inst.depart_step), d(tt)
    rc = lib.lpsim_surrogate_load(vp(off), vp(edges), vp(dep), inst.n_trips, vp(ttd), inst.n_edges, n_bins,
                                  bin_steps, horizon, vp(inflow), vp(occ), None)
    assert rc == 0
    torch.cuda.synchronize()
    assert np.array_equal(inflow.cpu().numpy(), inflow_ref)
    assert np.array_equal(occ.cpu().numpy(), occ_ref)


def test_features_targets_tt(torch):
    case("surrogate features, targets, travel-time update")
    from paper_2406_08496_amd.lpsim import load_library

    lib = load_library()
    rng = np.random.default_rng(3)
    E, B, bs = 700, 24, 600
    inflow = rng.integers(0, 200, size=(E, B)).astype(np.int32)
    occ = rng.integers(0, 10 ** 6, size=(E, B)).astype(np.int64)
    length = rng.integers(20, 2000, size=E).astype(np.float32)
    lanes = rng.integers(1, 5, size=E).astype(np.uint8)
    speed = rng.choice([13.4, 17.9, 22.4], size=E).astype(np.float32)
    exits = rng.integers(0, 50, size=(E, B)).astype(np.int32)
    ttsum = (exits * rng.uniform(5, 400, size=(E, B))).astype(np.int64)
    tt_free = np.ceil(np.ceil(length) / (speed * 0.5)).astype(np.float32)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    nw = B // 12
    # device inputs stay referenced until the kernels have run
    dev = {k: d(v) for k, v in dict(inflow=inflow, occ=occ, length=length, lanes=lanes, speed=speed, exits=exits,
                                     ttsum=ttsum, tt_free=tt_free).items()}
    x = torch.empty((E * nw, 32), dtype=torch.bfloat16, device="cuda")
    assert lib.lpsim_surrogate_features(E, B, bs, ctypes.c_float(7.0), vp(dev["inflow"]), vp(dev["occ"]),
                                        vp(dev["length"]), vp(dev["lanes"]), vp(dev["speed"]), vp(x), None) == 0
    y = torch.empty((E * nw, 16), dtype=torch.float32, device="cuda")
    m = torch.empty((E * nw, 16), dtype=torch.uint8, device="cuda")
    assert lib.lpsim_surrogate_targets(E, B, vp(dev["exits"]), vp(dev["ttsum"]), vp(dev["tt_free"]), vp(y), vp(m),
                                       None) == 0
    tt = rng.uniform(1, 300, size=(E, B)).astype(np.float32)
    ttd = d(tt)
    yp = rng.normal(scale=0.5, size=(E * nw, 16)).astype(np.float32)
    ypd = d(yp)
    assert lib.lpsim_surrogate_tt(E, B, vp(ypd), vp(dev["tt_free"]), ctypes.c_float(0.5), ctypes.c_float(5000.0),
                                  vp(ttd), None) == 0
    torch.cuda.synchronize()
    xf = oa.features(inflow, occ, length, lanes, speed, bs, 7.0)
    xg = mlp.from_bits(x.view(torch.int16).cpu().numpy().view(np.uint16))
    assert np.all(np.abs(xg - xf) <= 2.0 ** -7 * np.abs(xf) + 1e-30)
    yr, mr = oa.targets(exits, ttsum, tt_free.astype(np.float64))
    assert np.array_equal(m.cpu().numpy().astype(bool), mr)
    assert np.allclose(y.cpu().numpy(), yr, rtol=1e-5, atol=2e-6)
    tr = oa.tt_update(tt, yp.astype(np.float64), tt_free.astype(np.float64), 0.5, 5000.0)
    assert np.allclose(ttd.cpu().numpy(), tr, rtol=2e-6)


def test_shift_and_edge_tt(torch):
    case("surrogate anchored shift and routing cost")
    from paper_2406_08496_amd.lpsim import load_library

    lib = load_library()
    rng = np.random.default_rng(8)
    E, B = 513, 36
    nw = B // 12
    yn = rng.normal(scale=0.8, size=(E * nw, 16)).astype(np.float32)
    ya = rng.normal(scale=0.8, size=(E * nw, 16)).astype(np.float32)
    anc = rng.uniform(0.5, 900.0, size=(E, B)).astype(np.float32)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    out = torch.empty((E, B), dtype=torch.float32, device="cuda")
    ynd, yad, ancd = d(yn), d(ya), d(anc)  # referenced until the kernels have run
    assert lib.lpsim_surrogate_shift(E, B, vp(ynd), vp(yad), vp(ancd), ctypes.c_float(1.0),
                                     ctypes.c_float(1000.0), vp(out), None) == 0
    inflow = rng.integers(0, 30, size=(E, B)).astype(np.int32)
    inflow[::7] = 0  # edges nobody enters: free flow
    tt_free = rng.uniform(0.5, 60.0, size=E).astype(np.float32)
    et = torch.empty(E, dtype=torch.float64, device="cuda")
    infd, tfd = d(inflow), d(tt_free)
    assert lib.lpsim_surrogate_edge_tt(E, B, vp(infd), vp(out), vp(tfd), ctypes.c_float(0.5), vp(et), None) == 0
    torch.cuda.synchronize()
    ref = oa.shift(yn.astype(np.float64), ya.astype(np.float64), anc.astype(np.float64), 1.0, 1000.0)
    got = out.cpu().numpy()
    assert np.allclose(got, ref, rtol=2e-6)
    assert np.all(got >= 1.0) and np.all(got <= 1000.0)
    er = oa.edge_tt(inflow, got, tt_free, 0.5)
    assert np.allclose(et.cpu().numpy(), er, rtol=1e-12)
    assert lib.lpsim_surrogate_shift(E, 30, vp(ynd), vp(yad), vp(ancd), ctypes.c_float(1.0),
                                     ctypes.c_float(1000.0), vp(out), None) != 0


def test_device_stats_equal_host(torch):
    """The binned statistics handed over on the device (lpsim_edge_stats_device)
    equal the host copies element by element, with vehicles still on their
    edges (occupancy completed up to the current step) and again later in the
    run; the per-bin travel times computed from them on the device
    (lpsim_edge_tt_bins_device) equal the host routine's."""
    from paper_2406_08496_amd.assign import Assignment

    inst = synth.grid_instance(seed=13, side=8, n_trips=3000, depart_window=1200, len_lo=100, len_hi=300)
    a = Assignment(inst, n_bins=24)
    a.sim.load_trips(inst.depart_step, inst.route_off, inst.route_edges)
    for steps in (700, 900):
        a.sim.step(steps)
        host = a.sim.edge_stats(binned=True)
        dev = a.sim.edge_stats(binned=True, device=True)
        case("device statistics vs host after", steps, "more steps,", a.sim.counters()["vehicle_steps"],
             "vehicle-steps")
        assert np.array_equal(host["tt_sum"], dev["tt_sum"]) and np.array_equal(host["n_exits"], dev["n_exits"])
        for k in ("inflow_bin", "exits_bin", "tt_bin", "occ_bin"):
            assert torch.is_tensor(dev[k])
            got = dev[k].cpu().numpy()
            assert got.dtype == host[k].dtype and np.array_equal(got, host[k]), k
        assert host["occ_bin"].sum() > 0 and host["exits_bin"].sum() > 0
        tb_h = a.tt_bins_from_stats(host).cpu().numpy()
        tb_d = a.tt_bins_from_stats(dev).cpu().numpy()
        assert np.array_equal(tb_h.view(np.uint32), tb_d.view(np.uint32))


def test_msa_small_end_to_end(torch):
    case("MSA, 6 iterations, plain vs surrogate, 8x8 grid")
    from paper_2406_08496_amd.assign import Assignment, agreement

    inst = synth.grid_instance(seed=13, side=8, n_trips=3000, depart_window=1200, len_lo=100, len_hi=300)
    inst.n_steps = 4800
    a = Assignment(inst, n_bins=24)
    plain = a.run_plain(6)
    b = Assignment(inst, n_bins=24)
    sur = b.run_surrogate(6, judge_every=3, tol=10.0, train_steps=50, batch=2048)
    modes = [h["mode"] for h in sur["hist"]]
    assert modes[0] == "sim" and "surrogate" in modes
    assert sur["n_sim"] < len(plain["hist"])
    for res in (plain, sur):
        off, edges = res["routes"]
        assert off[-1] == len(edges)
        for i in range(0, inst.n_trips, 97):
            r = edges[off[i]:off[i + 1]]
            assert inst.src[r[0]] == inst.meta["origin"][i] and inst.dst[r[-1]] == inst.meta["dest"][i]
            assert np.all(inst.dst[r[:-1]] == inst.src[r[1:]])
    g = agreement(sur["tt"], plain["tt"], plain["exits"])
    assert np.isfinite(g)
    # the loops write routes into two buffers in turn; a second run on the
    # same object leaves the routes the first one returned untouched, and
    # the same routes come out again
    keep = (plain["routes"][0].copy(), plain["routes"][1].copy())
    again = a.run_plain(6)
    assert np.array_equal(plain["routes"][0], keep[0]) and np.array_equal(plain["routes"][1], keep[1])
    assert np.array_equal(again["routes"][0], keep[0]) and np.array_equal(again["routes"][1], keep[1])


def test_trained_network_gain(torch):
    """What the trained perceptron adds over the method without it.

    (1) On an assignment that converges (8x8 grid), the surrogate-assisted
    loop reaches the plain loop's final edge travel times within 2% while
    running the full simulation on fewer iterations.  (2) On a congested
    planar graph, the anchored estimate of the next routes' travel times is,
    over five MSA transitions, closer to the simulation than reusing the last
    simulation (what the loop would do without a model): by a wide margin
    where the queues respond to the route changes (a quarter of the
    demand), narrowly where gridlock noise dominates (full demand)."""
    case("trained network gain: MSA on an 8x8 grid; anchored vs stale on regional at 2%")
    from paper_2406_08496_amd.assign import Assignment, agreement

    inst = synth.grid_instance(seed=13, side=8, n_trips=3000, depart_window=1200, len_lo=100, len_hi=300)
    inst.n_steps = 4800
    plain = Assignment(inst, n_bins=24).run_plain(10)
    sur = Assignment(inst, n_bins=24).run_surrogate(10)
    g = agreement(sur["tt"], plain["tt"], plain["exits"])
    print("grid: surrogate sims", sur["n_sim"], "of", len(plain["hist"]), "agreement", g,
          "wall", sur["wall_s"], "vs", plain["wall_s"], flush=True)
    assert sur["n_sim"] <= len(plain["hist"]) // 2
    assert g <= 0.02

    for demand, bar in ((0.25, 0.8), (1.0, 0.97)):
        e_anc, e_stale = anchored_vs_stale(torch, synth.regional(0.02, demand))
        print(f"regional 2%, demand x{demand}: anchored", e_anc, "stale", e_stale, flush=True)
        assert np.mean(e_anc) < bar * np.mean(e_stale)
        if demand < 1.0:
            assert sum(a < b for a, b in zip(e_anc, e_stale)) >= 4


def anchored_vs_stale(torch, reg, n=5):
    """Errors of the anchored estimate and of the last simulation against
    the simulation of the next routes, over n MSA transitions, with the
    perceptron trained on the simulations so far (the last three)."""
    from paper_2406_08496_amd.assign import WIN, Assignment
    from paper_2406_08496_amd.surrogate import EdgeMLP

    a = Assignment(reg, n_bins=48)
    routes = [(reg.route_off, reg.route_edges)]
    sims = []
    for j in range(n + 1):
        st = a.simulate(*routes[-1])
        sims.append(st)
        routes.append(a.reroute(a.edge_tt_from_stats(st), *routes[-1], j + 1))
    net = EdgeMLP(seed=0)
    buf = []
    e_anc, e_stale = [], []
    for j in range(n):
        anc = a.anchor(sims[j], *routes[j])
        _, y, m = a.samples(sims[j])
        assert bool(torch.isfinite(y).all())
        keep = m[:, :WIN].any(1)
        buf = (buf + [(anc["x"][keep], y[keep], m[keep])])[-3:]
        X = torch.cat([b[0] for b in buf])
        Y = torch.cat([b[1] for b in buf])
        M = torch.cat([b[2] for b in buf])
        gen = torch.Generator(device="cuda")
        gen.manual_seed(j)
        for _ in range(300):
            idx = torch.randint(0, X.shape[0], (min(8192, X.shape[0]),), device="cuda", generator=gen)
            loss = net.train_step(X[idx].contiguous(), Y[idx].contiguous(), M[idx].contiguous(), lr=2e-3)
        assert np.isfinite(float(loss.item()))
        est = a.estimate(net, anc, *routes[j + 1])
        truth = a.edge_tt_from_stats(sims[j + 1])
        w = sims[j + 1]["n_exits"].astype(np.float64)
        err = lambda t: float((w * np.abs(t - truth) / truth).sum() / w.sum())
        e_anc.append(err(est))
        e_stale.append(err(a.edge_tt_from_stats(sims[j])))
    return e_anc, e_stale
