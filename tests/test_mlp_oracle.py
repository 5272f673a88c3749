"""Pins for the perceptron oracle: closed forms and finite differences."""
import numpy as np

from oracle import mlp


def test_bf16_rounding_ties_to_even():
    # 1 + 2^-8 lies halfway between bfloat16 neighbours 1 and 1 + 2^-7: even (1)
    assert mlp.bf16(1.0 + 2.0 ** -8) == 1.0
    # 1 + 3*2^-8 lies halfway between 1 + 2^-7 and 1 + 2^-6: even (1 + 2^-6)
    assert mlp.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert mlp.bf16(-(1.0 + 2.0 ** -7 + 2.0 ** -9)) == -(1.0 + 2.0 ** -7)
    v = np.array([0.1, -3.75, 1e-3, 123456.0])
    assert np.array_equal(mlp.from_bits(mlp.bf16_bits(mlp.bf16(v))), mlp.bf16(v))


def permutation_net(seed=0):
    """Weights that route input features through the hidden layers unchanged
    (0/1 permutation matrices, zero bias): y[o] = x[pi(o)] for o < 16."""
    rng = np.random.default_rng(seed)
    p1 = rng.permutation(32)
    p2 = rng.permutation(32)
    p3 = rng.permutation(32)
    p4 = rng.permutation(32)[:16]
    wt = [np.zeros((o, i)) for i, o in mlp.DIMS]
    for n in range(32):
        wt[0][n, p1[n]] = 1.0
        wt[1][n, p2[n]] = 1.0
        wt[2][n, p3[n]] = 1.0
    for o in range(16):
        wt[3][o, p4[o]] = 1.0
    b = [np.zeros(o) for _, o in mlp.DIMS]
    # composed routing: y[o] = h3[p4[o]] = h2[p3[p4[o]]] = h1[p2[..]] = x[p1[..]]
    pi = p1[p2[p3[p4]]]
    return wt, b, pi


def test_forward_permutation_network_closed_form():
    wt, b, pi = permutation_net(3)
    rng = np.random.default_rng(1)
    x = mlp.bf16(rng.uniform(0.0, 4.0, size=(50, 32)))  # non-negative: ReLU passes
    y, hs = mlp.forward(x, wt, b)
    assert np.array_equal(y, x[:, pi])
    assert np.all(hs[0][:, 32:] == 0.0)


def test_backward_matches_finite_differences():
    """Without rounding, the analytic gradient equals central differences of
    the float64 loss (relative 1e-6)."""
    rng = np.random.default_rng(2)
    wt, b = mlp.init_params(4)
    x = rng.normal(size=(6, 32))
    t = rng.normal(size=(6, 16))
    mask = rng.random((6, 16)) < 0.8
    inv = 1.0 / mask.sum()

    def loss_of(wt_, b_):
        y, _ = mlp.forward(x, wt_, b_, rnd=False)
        return mlp.loss_grad(y, t, mask, inv, rnd=False)[1]

    y, hs = mlp.forward(x, wt, b, rnd=False)
    dz, _ = mlp.loss_grad(y, t, mask, inv, rnd=False)
    dwt, db = mlp.backward(x, hs, dz, wt, rnd=False)
    h = 1e-6
    for l in range(4):
        for _ in range(6):
            i = rng.integers(0, wt[l].shape[0])
            j = rng.integers(0, wt[l].shape[1])
            wp = [w.copy() for w in wt]
            wm = [w.copy() for w in wt]
            wp[l][i, j] += h
            wm[l][i, j] -= h
            fd = (loss_of(wp, b) - loss_of(wm, b)) / (2 * h)
            assert abs(fd - dwt[l][i, j]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8
        i = rng.integers(0, b[l].shape[0])
        bp = [v.copy() for v in b]
        bm = [v.copy() for v in b]
        bp[l][i] += h
        bm[l][i] -= h
        fd = (loss_of(wt, bp) - loss_of(wt, bm)) / (2 * h)
        assert abs(fd - db[l][i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8


def test_adam_first_step_closed_form():
    """From zero moments the bias-corrected first step is lr * g / (|g| + eps)."""
    w = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    w1, m, v = mlp.adam(w, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    assert np.allclose(w1, w - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_bounds_cover_binary32_reimplementation():
    """A binary32-accumulating re-evaluation stays inside the stated bounds."""
    rng = np.random.default_rng(7)
    wt, b = mlp.init_params(5)
    x = mlp.bf16(rng.normal(size=(40, 32)))
    y, hs = mlp.forward(x, wt, b)
    bound = mlp.forward_bound(x, wt, b, y, hs)
    a = x.astype(np.float32)
    for l in range(3):
        z = (a @ mlp.bf16(wt[l]).T.astype(np.float32)) + b[l].astype(np.float32)
        a = mlp.bf16(np.maximum(z, 0.0)).astype(np.float32)
    y32 = (a @ mlp.bf16(wt[3]).T.astype(np.float32)) + b[3].astype(np.float32)
    assert np.all(np.abs(y32 - y) <= bound)
    # typical errors sit far below the output scale (rare bfloat16 flips only)
    assert np.median(np.abs(y32 - y)) < 1e-5 * np.median(np.abs(y))


def integer_net(seed):
    """Integer inputs, sparse {-1, 0, 1} weights and small integer biases:
    every partial sum is an integer below 2^24, so binary32 accumulation in any
    order is exact and an implementation must agree with the oracle exactly."""
    rng = np.random.default_rng(seed)
    wt = [np.where(rng.random((o, i)) < 0.1, rng.choice([-1.0, 1.0], size=(o, i)), 0.0) for i, o in mlp.DIMS]
    b = [rng.integers(-3, 4, size=o).astype(np.float64) for _, o in mlp.DIMS]
    return wt, b


def test_integer_network_is_exact_in_binary32():
    wt, b = integer_net(11)
    rng = np.random.default_rng(12)
    x = rng.integers(0, 9, size=(300, 32)).astype(np.float64)
    y, hs = mlp.forward(x, wt, b)
    assert np.all(np.abs(y) < 2 ** 24) and np.all(y == np.round(y))
    a = x.astype(np.float32)
    for l in range(3):
        z = (a @ wt[l].T.astype(np.float32)) + b[l].astype(np.float32)
        a = mlp.bf16(np.maximum(z, 0.0)).astype(np.float32)
        assert np.array_equal(a, hs[l])
    y32 = (a @ wt[3].T.astype(np.float32)) + b[3].astype(np.float32)
    assert np.array_equal(y32, y)
