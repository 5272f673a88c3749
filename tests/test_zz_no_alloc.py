"""The allocation-free perceptron backward (lpsim_mlp_backward_noalloc)
against the backward with caller-owned buffers (lpsim_mlp_backward), through
the C ABI: the same kernels with the same slices give the same bits.  Two
calls in a row, the second smaller than the first, so the second runs on the
scratch array as the first left it; the size limits are checked on the host."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HID, IN, OUT = 256, 32, 16
DIMS = ((IN, HID), (HID, HID), (HID, HID), (HID, OUT))


def case(*a):
    print("CASE:", *a, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_08496_amd.lpsim import load_library
    from paper_2406_08496_amd.surrogate import EdgeMLP

    return torch, load_library(), EdgeMLP


def _ptrs(ts):
    arr = (ctypes.c_void_p * len(ts))(*[t.data_ptr() for t in ts])
    return arr


def _inputs(torch, lib, net, n, seed):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    x = torch.randn((n, IN), generator=g, device="cuda").to(torch.bfloat16)
    tgt = torch.randn((n, OUT), generator=g, device="cuda")
    y, hs = net.forward(x, keep=True)
    dz = torch.empty((n, OUT), dtype=torch.bfloat16, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.lpsim_mlp_loss_grad(ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(tgt.data_ptr()), None, n,
                                 ctypes.c_float(1.0 / (n * OUT)), ctypes.c_void_p(dz.data_ptr()), None, s)
    assert rc == 0
    return x, hs, dz


def _grads(torch):
    dwt = [torch.full((o, i), float("nan"), device="cuda") for i, o in DIMS]
    db = [torch.full((o,), float("nan"), device="cuda") for _, o in DIMS]
    return dwt, db


def _reference(torch, lib, net, x, hs, dz, n_split, n):
    dwt, db = _grads(torch)
    ws = torch.empty((lib.lpsim_mlp_workspace_bytes(n, n_split) + 3) // 4, dtype=torch.float32, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.lpsim_mlp_backward(ctypes.c_void_p(x.data_ptr()), _ptrs(hs), ctypes.c_void_p(dz.data_ptr()),
                                _ptrs(net.w_bf), _ptrs(dwt), _ptrs(db), ctypes.c_void_p(ws.data_ptr()),
                                n_split, n, s)
    assert rc == 0
    return dwt, db


def _noalloc(torch, lib, net, x, hs, dz, n_split, n):
    dwt, db = _grads(torch)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.lpsim_mlp_backward_noalloc(ctypes.c_void_p(x.data_ptr()), _ptrs(hs), ctypes.c_void_p(dz.data_ptr()),
                                        _ptrs(net.w_bf), _ptrs(dwt), _ptrs(db), n_split, n, s)
    assert rc == 0, rc
    return dwt, db


def _same(a, b, what):
    for l, (u, v) in enumerate(zip(a, b)):
        ua = u.cpu().numpy().view(np.uint32)
        ub = v.cpu().numpy().view(np.uint32)
        assert np.array_equal(ua, ub), f"{what}: layer {l} differs at {np.argwhere(ua != ub)[:4].tolist()}"


def test_noalloc_backward_matches(env):
    torch, lib, EdgeMLP = env
    net = EdgeMLP(seed=3)
    # the largest call first, then a smaller one on the scratch it left
    for n, n_split, seed in ((8192, 32, 1), (3001, 12, 2)):
        case("noalloc backward, rows", n, "slices", n_split)
        x, hs, dz = _inputs(torch, lib, net, n, seed)
        rw, rb = _reference(torch, lib, net, x, hs, dz, n_split, n)
        nw, nb = _noalloc(torch, lib, net, x, hs, dz, n_split, n)
        torch.cuda.synchronize()
        _same(nw, rw, f"dwt n={n}")
        _same(nb, rb, f"db n={n}")


def test_noalloc_backward_empty_and_limits(env):
    torch, lib, EdgeMLP = env
    net = EdgeMLP(seed=4)
    case("noalloc backward, no rows and the size limits")
    dwt, db = _grads(torch)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    hs = [torch.empty((1, HID), dtype=torch.bfloat16, device="cuda") for _ in range(3)]
    x = torch.empty((1, IN), dtype=torch.bfloat16, device="cuda")
    dz = torch.empty((1, OUT), dtype=torch.bfloat16, device="cuda")
    args = (ctypes.c_void_p(x.data_ptr()), _ptrs(hs), ctypes.c_void_p(dz.data_ptr()), _ptrs(net.w_bf),
            _ptrs(dwt), _ptrs(db))
    assert lib.lpsim_mlp_backward_noalloc(*args, 8, 0, s) == 0
    torch.cuda.synchronize()
    for t in dwt + db:
        assert torch.count_nonzero(t).item() == 0
    # beyond the limits: rejected on the host before any launch
    assert lib.lpsim_mlp_backward_noalloc(*args, 8, 8193, s) == -5
    assert lib.lpsim_mlp_backward_noalloc(*args, 33, 100, s) == -5
    assert lib.lpsim_mlp_backward_noalloc(*args, 0, 100, s) == -1
