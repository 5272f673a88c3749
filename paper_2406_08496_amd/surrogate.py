"""Edge travel-time surrogate: the perceptron of the library, driven from Python.

Weights and activations live in torch tensors on the GPU (PyTorch provides
device memory and the stream); every arithmetic step -- forward, loss
gradient, backward, Adam -- runs in the library's HIP kernels through the C
ABI (`lpsim_mlp_*`).  bfloat16 tensors are passed by their bit patterns.

Shape: x[32] -> 256 -> 256 -> 256 -> y[16]; layer l's binary32 master weight
is [out_l][in_l].  The matrix cores read bfloat16 matrices in fragment order
(blocks of 32 rows x 16 features, `to_matrix` / `from_matrix` convert): the
weight copies, the kept activations and the backward's gradients.
"""
from __future__ import annotations

import ctypes

import numpy as np

from .lpsim import LpsimError, load_library

IN, HID, OUT = 32, 256, 16
DIMS = [(IN, HID), (HID, HID), (HID, HID), (HID, OUT)]


def _ptrs(tensors):
    arr = (ctypes.c_void_p * len(tensors))()
    for i, t in enumerate(tensors):
        arr[i] = None if t is None else t.data_ptr()
    return arr


def _check(rc, what):
    if rc != 0:
        raise LpsimError(rc, what)


def to_matrix(t, rows, feats):
    """A fragment-order array (rows a multiple of 32, feats of 16) -> the
    [rows][feats] matrix.  Element (r, f) sits at
    ((r//32) * (feats//16) + f//16) * 512 + (f%16 + 16 * ((r%32)//8)) * 8 + r%8."""
    v = t.reshape(rows // 32, feats // 16, 4, 16, 8)  # step, feature block, row group, feature, row
    return v.permute(0, 2, 4, 1, 3).reshape(rows, feats)


def from_matrix(m):
    """[rows][feats] matrix (rows a multiple of 32) -> fragment order (flat)."""
    rows, feats = m.shape
    v = m.reshape(rows // 32, 4, 8, feats // 16, 16)  # step, row group, row, feature block, feature
    return v.permute(0, 3, 1, 4, 2).reshape(-1).contiguous()


def _pad32(n):
    return (n + 31) // 32 * 32


def _stream():
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class EdgeMLP:
    """Binary32 master weights, bfloat16 copies in both layouts, Adam state."""

    def __init__(self, wt=None, b=None, seed=0, device="cuda", n_split=None):
        import torch

        self.torch = torch
        self.device = device
        # batch slices of the weight-gradient kernels: fixed if given, else
        # chosen from the row count (the result depends only on the count)
        self.n_split = n_split
        if wt is None:
            rng = np.random.default_rng(seed)
            wt = [rng.normal(0.0, np.sqrt(2.0 / i), size=(o, i)) for i, o in DIMS]
            b = [np.zeros(o) for _, o in DIMS]
        self.w = [torch.tensor(np.asarray(x, np.float32), device=device) for x in wt]
        self.b = [torch.tensor(np.asarray(x, np.float32), device=device) for x in b]
        self.m_w = [torch.zeros_like(x) for x in self.w]
        self.v_w = [torch.zeros_like(x) for x in self.w]
        self.m_b = [torch.zeros_like(x) for x in self.b]
        self.v_b = [torch.zeros_like(x) for x in self.b]
        self.g_w = [torch.zeros_like(x) for x in self.w]
        self.g_b = [torch.zeros_like(x) for x in self.b]
        self.t = 0
        self.lib = load_library()
        self._sync_bf16()
        self._ws = None

    def _sync_bf16(self):
        # bfloat16 copies of the binary32 master in fragment order, written by
        # the optimizer kernel with a zero step (w - 0 * update == w): wt_bf
        # with rows = in, features = out (forward), w_bf with rows = out
        # (zero-padded to 32) and features = in (backward)
        torch = self.torch
        self.wt_bf = [torch.zeros(_pad32(i) * o, dtype=torch.bfloat16, device=self.device) for i, o in DIMS]
        self.w_bf = [torch.zeros(_pad32(o) * i, dtype=torch.bfloat16, device=self.device) for i, o in DIMS]
        f = ctypes.c_float
        for l, (i, o) in enumerate(DIMS):
            m = torch.zeros_like(self.w[l])
            _check(self.lib.lpsim_mlp_adam(
                ctypes.c_void_p(self.w[l].data_ptr()), ctypes.c_void_p(self.wt_bf[l].data_ptr()),
                ctypes.c_void_p(self.w_bf[l].data_ptr()), ctypes.c_void_p(m.data_ptr()),
                ctypes.c_void_p(m.data_ptr()), ctypes.c_void_p(m.data_ptr()), o, i, f(0.0), f(0.9),
                f(0.999), f(1e-8), 1, _stream()), "mlp bf16 copy")

    # -- layout of the kept activations ---------------------------------------
    # Fragment order over the rows padded to a multiple of 64.
    @staticmethod
    def padded_rows(n):
        return (n + 63) // 64 * 64

    @staticmethod
    def hidden_rows(hs, n):
        """The kept activations as [n][256] tensors."""
        return [to_matrix(h, EdgeMLP.padded_rows(n), HID)[:n] for h in hs]

    def pack_hidden(self, h):
        """[n][256] activations -> the kept layout (padding rows zero), as the
        backward takes them."""
        n = h.shape[0]
        full = self.torch.zeros((self.padded_rows(n), HID), dtype=h.dtype, device=h.device)
        full[:n] = h
        return from_matrix(full)

    def weight_matrices(self, l):
        """Layer l's bfloat16 copies as matrices: (wt_bf as [in][out], w_bf as
        [out][in])."""
        i, o = DIMS[l]
        return to_matrix(self.wt_bf[l], _pad32(i), o)[:i], to_matrix(self.w_bf[l], _pad32(o), i)[:o]

    # -- inference ----------------------------------------------------------
    def forward(self, x, keep=False):
        """x: [n][32] bfloat16 tensor -> y [n][16] float32; with keep, also the
        hidden activations (fragment order, padded_rows(n) x 256 each)."""
        torch = self.torch
        assert x.dtype == torch.bfloat16 and x.shape[1] == IN and x.is_contiguous()
        n = x.shape[0]
        y = torch.empty((n, OUT), dtype=torch.float32, device=self.device)
        hs = [torch.empty(self.padded_rows(n) * HID, dtype=torch.bfloat16, device=self.device)
              for _ in range(3)] if keep else None
        h_arr = _ptrs(hs) if keep else None
        _check(self.lib.lpsim_mlp_forward(ctypes.c_void_p(x.data_ptr()), _ptrs(self.wt_bf), _ptrs(self.b),
                                          ctypes.c_void_p(y.data_ptr()), h_arr, n, _stream()), "mlp forward")
        return (y, hs) if keep else y

    # -- training ------------------------------------------------------------
    def gradients(self, x, target, mask=None, count=None):
        """Loss (masked MSE) and gradients into self.g_w / self.g_b.  `count`
        (the number of set mask entries) may be given to spare a device sync."""
        torch = self.torch
        n = x.shape[0]
        y, hs = self.forward(x, keep=True)
        dz = torch.empty((n, OUT), dtype=torch.bfloat16, device=self.device)
        loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        if count is None:
            count = int(mask.sum().item()) if mask is not None else n * OUT
        inv = 1.0 / max(count, 1)
        mptr = ctypes.c_void_p(mask.data_ptr()) if mask is not None else None
        _check(self.lib.lpsim_mlp_loss_grad(ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(target.data_ptr()),
                                            mptr, n, ctypes.c_float(inv), ctypes.c_void_p(dz.data_ptr()),
                                            ctypes.c_void_p(loss.data_ptr()), _stream()), "mlp loss")
        self.backward(x, hs, dz)
        return loss, y

    def splits(self, n):
        # 8 slices (one per XCD) up to 16k rows, then one per 2,048 rows up to 64
        return self.n_split if self.n_split else max(8, min(64, n // 2048))

    def backward(self, x, hs, dz):
        """hs: the forward's kept activations (fragment order)."""
        torch = self.torch
        n = x.shape[0]
        n_split = self.splits(n)
        nbytes = self.lib.lpsim_mlp_workspace_bytes(n, n_split)
        if self._ws is None or self._ws.numel() * 4 < nbytes:
            self._ws = torch.empty((nbytes + 3) // 4, dtype=torch.float32, device=self.device)
        _check(self.lib.lpsim_mlp_backward(ctypes.c_void_p(x.data_ptr()), _ptrs(hs), ctypes.c_void_p(dz.data_ptr()),
                                           _ptrs(self.w_bf), _ptrs(self.g_w), _ptrs(self.g_b),
                                           ctypes.c_void_p(self._ws.data_ptr()), n_split, n, _stream()),
               "mlp backward")

    def adam_step(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.t += 1
        f = ctypes.c_float
        for l, (i, o) in enumerate(DIMS):
            _check(self.lib.lpsim_mlp_adam(
                ctypes.c_void_p(self.w[l].data_ptr()), ctypes.c_void_p(self.wt_bf[l].data_ptr()),
                ctypes.c_void_p(self.w_bf[l].data_ptr()), ctypes.c_void_p(self.g_w[l].data_ptr()),
                ctypes.c_void_p(self.m_w[l].data_ptr()), ctypes.c_void_p(self.v_w[l].data_ptr()),
                o, i, f(lr), f(beta1), f(beta2), f(eps), self.t, _stream()), "mlp adam")
            _check(self.lib.lpsim_mlp_adam(
                ctypes.c_void_p(self.b[l].data_ptr()), None, None, ctypes.c_void_p(self.g_b[l].data_ptr()),
                ctypes.c_void_p(self.m_b[l].data_ptr()), ctypes.c_void_p(self.v_b[l].data_ptr()),
                1, o, f(lr), f(beta1), f(beta2), f(eps), self.t, _stream()), "mlp adam")

    def train_step(self, x, target, mask=None, lr=1e-3, count=None):
        loss, _ = self.gradients(x, target, mask, count)
        self.adam_step(lr=lr)
        return loss
