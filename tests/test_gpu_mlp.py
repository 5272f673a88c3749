"""Perceptron kernels (bfloat16 MFMA, binary32 accumulation) vs the CPU
oracle, through the C ABI.

* integer networks: every binary32 sum is exact, so forward activations,
  outputs and backward gradients must equal the oracle exactly;
* realistic random networks: differences stay inside the rigorous
  propagated bound of the oracle, and typical differences are tiny;
* Adam against the float64 update; a short training run lowers the loss.
"""
import numpy as np
import pytest

from oracle import mlp

pytestmark = pytest.mark.gpu


def case(*a):
    print("CASE:", *a, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t

    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def bf(torch, a):
    """numpy values (already bfloat16-representable) -> torch bfloat16 tensor"""
    bits = mlp.bf16_bits(a).astype(np.int16)
    return torch.from_numpy(bits).cuda().view(torch.bfloat16)


def to_np(t):
    import torch as T

    if t.dtype == T.bfloat16:
        return mlp.from_bits(t.view(T.int16).cpu().numpy().view(np.uint16))
    return t.cpu().numpy().astype(np.float64)


def integer_net(seed):
    rng = np.random.default_rng(seed)
    wt = [np.where(rng.random((o, i)) < 0.1, rng.choice([-1.0, 1.0], size=(o, i)), 0.0) for i, o in mlp.DIMS]
    b = [rng.integers(-3, 4, size=o).astype(np.float64) for _, o in mlp.DIMS]
    return wt, b


@pytest.mark.parametrize("n", [1, 127, 300, 1024])
def test_forward_integer_exact(torch, n):
    case("mlp forward, integer network, n =", n)
    from paper_2406_08496_amd.surrogate import EdgeMLP

    wt, b = integer_net(11)
    x = np.random.default_rng(n).integers(0, 9, size=(n, 32)).astype(np.float64)
    y_ref, hs_ref = mlp.forward(x, wt, b)
    net = EdgeMLP(wt, b)
    y, hs = net.forward(bf(torch, x), keep=True)
    torch.cuda.synchronize()
    rows = EdgeMLP.hidden_rows(hs, n)
    for l in range(3):
        assert hs[l].numel() == (n + 63) // 64 * 64 * 256
        assert np.array_equal(to_np(rows[l].contiguous()), hs_ref[l]), f"hidden layer {l + 1}"
    assert np.array_equal(to_np(y), y_ref)


def test_forward_empty(torch):
    from paper_2406_08496_amd.surrogate import EdgeMLP

    net = EdgeMLP(seed=1)
    y = net.forward(torch.zeros((0, 32), dtype=torch.bfloat16, device="cuda"))
    torch.cuda.synchronize()
    assert y.shape == (0, 16)


def test_forward_realistic_within_bound(torch):
    case("mlp forward, He-initialised network, n = 5000")
    from paper_2406_08496_amd.surrogate import EdgeMLP

    wt, b = mlp.init_params(5)
    x = mlp.bf16(np.random.default_rng(3).normal(size=(5000, 32)))
    y_ref, hs_ref = mlp.forward(x, wt, b)
    bound = mlp.forward_bound(x, wt, b, y_ref, hs_ref)
    net = EdgeMLP(wt, b)
    y = to_np(net.forward(bf(torch, x)))
    err = np.abs(y - y_ref)
    assert np.all(err <= bound)
    assert np.median(err) < 1e-5 * np.median(np.abs(y_ref))


def test_backward_integer_exact(torch):
    case("mlp backward, integer network, n = 200")
    from paper_2406_08496_amd.surrogate import EdgeMLP

    wt, b = integer_net(21)
    rng = np.random.default_rng(22)
    n = 200
    x = rng.integers(0, 4, size=(n, 32)).astype(np.float64)
    _, hs = mlp.forward(x, wt, b)
    dz = rng.integers(-2, 3, size=(n, 16)).astype(np.float64)
    dwt, db = mlp.backward(x, hs, dz, wt)
    # every partial sum is an integer below 2^24: exact in binary32
    ins = [x] + hs
    for l in range(4):
        assert np.all(np.abs(dz).T @ np.abs(ins[l]) < 2 ** 24)
    net = EdgeMLP(wt, b, n_split=4)
    net.backward(bf(torch, x), [net.pack_hidden(bf(torch, h)) for h in hs], bf(torch, dz))
    torch.cuda.synchronize()
    for l in range(4):
        assert np.array_equal(to_np(net.g_w[l]), dwt[l]), f"dW layer {l + 1}"
        assert np.array_equal(to_np(net.g_b[l]), db[l]), f"db layer {l + 1}"


# the training batch with its default slices, a row count that is not a
# multiple of 8, and more slices than the rows fill
@pytest.mark.parametrize("n,n_split", [(4096, 8), (1000, 3), (8192, None), (1001, 16), (77, 24)])
def test_backward_realistic_within_bound(torch, n, n_split):
    case("mlp backward, realistic, n =", n, "splits", n_split)
    from paper_2406_08496_amd.surrogate import EdgeMLP

    wt, b = mlp.init_params(6)
    rng = np.random.default_rng(8)
    x = mlp.bf16(rng.normal(size=(n, 32)))
    y, hs = mlp.forward(x, wt, b)
    t = rng.normal(size=y.shape)
    dz, _ = mlp.loss_grad(y, t, None, 1.0 / y.size)
    dwt, db = mlp.backward(x, hs, dz, wt)
    net = EdgeMLP(wt, b, n_split=n_split)
    bw, bb = mlp.backward_bound(x, hs, dz, wt, n_split=net.splits(n))
    net.backward(bf(torch, x), [net.pack_hidden(bf(torch, h)) for h in hs], bf(torch, dz))
    torch.cuda.synchronize()
    for l in range(4):
        e = np.abs(to_np(net.g_w[l]) - dwt[l])
        assert np.all(e <= bw[l] + 1e-30), f"dW layer {l + 1}: max excess {np.max(e - bw[l])}"
        assert np.median(e) <= 1e-4 * np.median(np.abs(dwt[l])) + 1e-12
        eb = np.abs(to_np(net.g_b[l]) - db[l])
        assert np.all(eb <= bb[l] + 1e-30), f"db layer {l + 1}"


def test_backward_through_forward_and_empty(torch):
    """The backward on the forward's own kept activations (rows past n in
    them hold the activations of a zero input) equals the backward on the
    same rows repacked with zero padding; no rows gives zero gradients."""
    case("mlp backward on kept activations, n = 1003, and n = 0")
    from paper_2406_08496_amd.surrogate import EdgeMLP

    wt, b = mlp.init_params(9)
    rng = np.random.default_rng(10)
    n = 1003
    x = mlp.bf16(rng.normal(size=(n, 32)))
    dz = mlp.bf16(rng.normal(size=(n, 16)) * 1e-3)
    net = EdgeMLP(wt, b, n_split=5)
    _, kept = net.forward(bf(torch, x), keep=True)
    pad = EdgeMLP.hidden_rows(kept, EdgeMLP.padded_rows(n))[0][n:]
    assert torch.count_nonzero(pad).item() > 0  # padding rows: relu(bias) of a zero input
    net.backward(bf(torch, x), kept, bf(torch, dz))
    got = [t.clone() for t in net.g_w + net.g_b]
    repacked = [net.pack_hidden(r.contiguous()) for r in EdgeMLP.hidden_rows(kept, n)]
    net.backward(bf(torch, x), repacked, bf(torch, dz))
    torch.cuda.synchronize()
    for u, v in zip(got, net.g_w + net.g_b):
        assert torch.equal(u, v)
    x0 = torch.zeros((0, 32), dtype=torch.bfloat16, device="cuda")
    _, kept0 = net.forward(x0, keep=True)
    for t in net.g_w + net.g_b:
        t.fill_(float("nan"))
    net.backward(x0, kept0, torch.zeros((0, 16), dtype=torch.bfloat16, device="cuda"))
    torch.cuda.synchronize()
    for t in net.g_w + net.g_b:
        assert torch.count_nonzero(t).item() == 0


def test_full_size_sampled(torch):
    """The benchmark's inference batch (2,200,000 rows) with the default
    slice count: sampled forward rows against the oracle within its bound,
    and the output layer's weight and bias gradients (whose inputs, dz_out and
    the kept last hidden layer, are exact) against float64 sums over all rows
    within the binary32 bound of an n/S + S + 32 chain, for sampled weights
    and every bias."""
    case("mlp full size, 2.2M rows, sampled")
    from paper_2406_08496_amd.surrogate import EdgeMLP

    n = 2_200_000
    wt, b = mlp.init_params(12)
    rng = np.random.default_rng(13)
    x = mlp.bf16(rng.normal(size=(n, 32)).astype(np.float32))
    net = EdgeMLP(wt, b)
    xt = bf(torch, x)
    y, hs = net.forward(xt, keep=True)
    rows = np.sort(rng.choice(n, 3000, replace=False))
    y_ref, hs_ref = mlp.forward(x[rows], wt, b)
    bound = mlp.forward_bound(x[rows], wt, b, y_ref, hs_ref)
    err = np.abs(to_np(y[torch.from_numpy(rows).cuda()]) - y_ref)
    assert np.all(err <= bound)
    dz = mlp.bf16(rng.normal(size=(n, 16)).astype(np.float32) * 1e-3)
    dzt = bf(torch, dz)
    net.backward(xt, hs, dzt)
    torch.cuda.synchronize()
    S = net.splits(n)
    g = mlp.gamma(n // S + S + 32)
    h2 = EdgeMLP.hidden_rows(hs, n)[2]
    gw, gb = to_np(net.g_w[3]), to_np(net.g_b[3])
    db_ref = dz.sum(axis=0)
    assert np.all(np.abs(gb - db_ref) <= g * np.abs(dz).sum(axis=0) + 1e-30)
    for i in rng.choice(256, 12, replace=False):
        col = to_np(h2[:, int(i)].contiguous())
        ref = dz.T @ col
        err = np.abs(gw[:, i] - ref)
        assert np.all(err <= g * (np.abs(dz).T @ np.abs(col)) + 1e-30), f"dW layer 4, input {i}"


def test_adam_matches_float64(torch):
    case("adam, 5 steps")
    from paper_2406_08496_amd.surrogate import EdgeMLP

    wt, b = mlp.init_params(9)
    net = EdgeMLP(wt, b)
    rng = np.random.default_rng(10)
    w_ref = [w.astype(np.float32).astype(np.float64) for w in wt]
    m_ref = [np.zeros_like(w) for w in wt]
    v_ref = [np.zeros_like(w) for w in wt]
    for t in range(1, 6):
        gs = [rng.normal(scale=0.01, size=w.shape).astype(np.float32) for w in wt]
        for l in range(4):
            net.g_w[l].copy_(torch.from_numpy(gs[l]))
            net.g_b[l].zero_()
            w_ref[l], m_ref[l], v_ref[l] = mlp.adam(w_ref[l], gs[l].astype(np.float64), m_ref[l], v_ref[l], t,
                                                    lr=1e-3)
        net.adam_step(lr=1e-3)
    torch.cuda.synchronize()
    for l in range(4):
        w = to_np(net.w[l])
        assert np.allclose(w, w_ref[l], rtol=1e-5, atol=1e-6)
        wt_m, w_m = net.weight_matrices(l)
        assert np.array_equal(to_np(wt_m.contiguous()), mlp.bf16(w).T)
        assert np.array_equal(to_np(w_m.contiguous()), mlp.bf16(w))


def test_training_lowers_loss(torch):
    case("train 300 steps on a smooth synthetic target")
    from paper_2406_08496_amd.surrogate import EdgeMLP

    rng = np.random.default_rng(12)
    n = 4096
    x = mlp.bf16(rng.uniform(-1, 1, size=(n, 32)))
    a = rng.normal(size=(32, 16)) / 6
    tgt = np.tanh(x @ a) + 0.1 * np.sin(3 * x[:, :16])
    xt = bf(torch, x)
    tt = torch.from_numpy(tgt.astype(np.float32)).cuda()
    net = EdgeMLP(seed=3)
    first = None
    for s in range(300):
        loss = net.train_step(xt, tt, lr=2e-3)
        if s == 0:
            first = float(loss.item())
    last = float(net.train_step(xt, tt, lr=2e-3).item())
    assert last < 0.1 * first, (first, last)
