"""CPU oracle of the edge travel-time perceptron -- test infrastructure only.

Plain numpy, float64 accumulation, with the bfloat16 rounding points of the
GPU path made explicit (round to nearest even): hidden activations after
bias and ReLU, the output-gradient, and the gradient after each ReLU mask.
With `rnd=False` every rounding is skipped and the code is the textbook
float64 perceptron, which the tests check against central finite
differences (the gradient pin) and a permutation network with a closed-form
output (the wiring pin).

Shapes: x [n][32]; layer l weight "wt" [out_l][in_l], bias [out_l];
(in, out) = (32,256), (256,256), (256,256), (256,16).
"""
from __future__ import annotations

import numpy as np

IN, HID, OUT = 32, 256, 16
DIMS = [(IN, HID), (HID, HID), (HID, HID), (HID, OUT)]


def bf16(a):
    """Round to the nearest bfloat16 (ties to even), via binary32."""
    f = np.asarray(a, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def bf16_bits(a):
    """bfloat16 bit patterns (uint16) of values that are already bfloat16."""
    return (np.asarray(a, dtype=np.float64).astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)


def from_bits(b):
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def init_params(seed=0):
    """He-style random weights (binary32 master values)."""
    rng = np.random.default_rng(seed)
    wt = [rng.normal(0.0, np.sqrt(2.0 / i), size=(o, i)).astype(np.float32).astype(np.float64) for i, o in DIMS]
    b = [rng.normal(0.0, 0.05, size=o).astype(np.float32).astype(np.float64) for _, o in DIMS]
    return wt, b


def forward(x, wt, b, rnd=True):
    """y = W4 relu(W3 relu(W2 relu(W1 x + b1) + b2) + b3) + b4, row-wise.

    Operands are bfloat16 (x, the weights, the hidden activations) when rnd.
    Returns (y, [h1, h2, h3])."""
    r = bf16 if rnd else (lambda v: np.asarray(v, dtype=np.float64))
    a = r(x)
    hs = []
    for l in range(3):
        z = a @ r(wt[l]).T + b[l]
        a = r(np.maximum(z, 0.0))
        hs.append(a)
    y = a @ r(wt[3]).T + b[3]
    return y, hs


def loss_grad(y, t, mask, inv_count, rnd=True):
    """Masked mean squared error and its gradient at the output (bfloat16)."""
    m = np.ones_like(y, dtype=bool) if mask is None else mask.astype(bool)
    d = np.where(m, y - t, 0.0)
    loss = float(np.sum(d * d) * inv_count)
    g = 2.0 * d * inv_count
    return (bf16(g) if rnd else g), loss


def backward(x, hs, dz_out, wt, rnd=True):
    """Gradients of the loss for the given output gradient.

    dW_l = dz_l^T a_{l-1};  db_l = sum_rows dz_l;
    dz_{l-1} = round(relu'(a_{l-1}) * (dz_l W_l)).
    Returns (dwt[4] in "wt" layout, db[4])."""
    r = bf16 if rnd else (lambda v: np.asarray(v, dtype=np.float64))
    ins = [r(x)] + list(hs)
    dz = dz_out
    dwt, db = [None] * 4, [None] * 4
    for l in range(3, -1, -1):
        dwt[l] = dz.T @ ins[l]
        db[l] = dz.sum(axis=0)
        if l == 0:
            break
        da = dz @ r(wt[l])
        dz = r(np.where(ins[l] > 0.0, da, 0.0))
    return dwt, db


def adam(w, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba 2015) in float64; returns (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------------------
# error bounds of a binary32-accumulating implementation against this oracle


def bf16_ulp(a):
    a = np.maximum(np.abs(a), 2.0 ** -126)
    return 2.0 ** (np.floor(np.log2(a)) - 7)


def gamma(k):
    """Accumulating k exact products in binary32 in any order: relative to the
    sum of magnitudes, at most 2 k 2^-24 (first order, with slack 2)."""
    return 2.0 * k * 2.0 ** -24


def forward_bound(x, wt, b, y, hs):
    """Per-element bound on |y_impl - y_oracle| for an implementation that
    accumulates in binary32 and rounds the hidden activations to bfloat16.

    If the implementation's hidden input differs by at most d, its
    pre-activation differs by at most dz = |W| d + gamma(K) (|a| + d) |W| +
    2^-23 |z| (bias add).  Rounding (binary32 then bfloat16) and ReLU are
    monotone, so its rounded activation lies between the roundings of
    relu(z - dz) and relu(z + dz), as does the oracle's: their difference
    bounds d for the next layer (zero unless a rounding boundary is within
    reach)."""
    a = bf16(x)
    d = np.zeros_like(a)
    for l in range(4):
        w = bf16(wt[l])
        wa = np.abs(w)
        k = w.shape[1]
        ref = a @ w.T + b[l]
        lin = d @ wa.T
        dz = lin + gamma(k) * ((np.abs(a) + d) @ wa.T) + (np.abs(ref) + lin) * 2.0 ** -23
        if l == 3:
            return dz
        d = bf16(np.maximum(ref + dz, 0.0)) - bf16(np.maximum(ref - dz, 0.0))
        a = hs[l]
    return None


def backward_bound(x, hs, dz_out, wt, n_split=1):
    """Per-element bounds on |dwt_impl - dwt_oracle| and |db_impl - db_oracle|
    when the implementation gets the same x, hs and dz_out (bfloat16) and
    accumulates in binary32 (contraction over rows in n_split partial sums).
    The ReLU masks are the same on both sides (same hs); the bfloat16
    rounding of each back-propagated gradient is bracketed as in the
    forward bound."""
    ins = [bf16(x)] + list(hs)
    dz = dz_out
    d = np.zeros_like(dz)
    n = x.shape[0]
    g_rows = gamma(n // n_split + n_split + 32)
    bw, bb = [None] * 4, [None] * 4
    for l in range(3, -1, -1):
        ai = np.abs(ins[l])
        bw[l] = d.T @ ai + g_rows * ((np.abs(dz) + d).T @ ai)
        bb[l] = d.sum(axis=0) + g_rows * (np.abs(dz) + d).sum(axis=0)
        if l == 0:
            break
        w = bf16(wt[l])
        wa = np.abs(w)
        k = w.shape[0]
        da = dz @ w
        dda = d @ wa + gamma(k) * ((np.abs(dz) + d) @ wa)
        live = ins[l] > 0.0
        d = np.where(live, bf16(da + dda) - bf16(da - dda), 0.0)
        dz = bf16(np.where(live, da, 0.0))
    return bw, bb
