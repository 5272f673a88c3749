"""Host-side logic that needs no GPU: the benchmark's command-line contract,
its byte model and traffic bookkeeping, and argument checks of the
surrogate entry points (they validate before touching the device)."""
import ctypes
import hashlib
import json
import os
import subprocess
import sys

import pytest

from paper_2406_08496_amd import lpsim

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in out["error"]


def test_bench_byte_model_and_traffic_key():
    import bench

    # the method's 18 bytes of state read and 8 written per vehicle-step
    assert bench.MOVE_FIXED_BYTES == 26
    src = os.path.join(ROOT, "paper_2406_08496_amd", "csrc", "lpsim_kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    for key, m in bench.MOVE_TRAFFIC.items():
        t = bench.move_traffic_bytes(*key)
        if m["kernels_sha256"] == sha:
            assert t == pytest.approx((m["fetch_kib"] * m["fetch_scale"] + m["write_kib"] * m["write_scale"]) * 1024)
        else:
            assert t is None  # counters were taken on another kernel source
    # only for the workload and window the counters were taken on
    assert bench.move_traffic_bytes("large-x1.0", 0, 20) is None
    assert bench.move_traffic_bytes("regional-225k-2.82M", 1, 20) is None


def test_bench_step_byte_model():
    import bench

    d = {"vehicle_steps": 10, "scan_bytes": 7, "transfers": 2, "arrived": 1, "departures": 3,
         "lc_attempts": 4, "claims_lost": 0, "lc_accepts": 0}
    # 28 per vehicle-step, the scan counter, 16 per exit, 20 per departure,
    # two look-ahead windows per lane-change attempt
    assert bench.step_bytes(d, 41) == 28 * 10 + 7 + 16 * 3 + 20 * 3 + 2 * 41 * 4
    assert bench.delta({k: 5 for k in bench.CNT_DELTA}, {k: 2 for k in bench.CNT_DELTA}) == \
        {k: 3 for k in bench.CNT_DELTA}


def test_bench_workload_names():
    import bench

    assert bench.make_workload("tiny")[0].n_trips == 2000
    inst, nb = bench.make_workload("regional:0.002")
    assert nb == 48 and inst.n_trips > 0
    inst, _ = bench.make_workload("regional-demand:0.5")
    assert inst.n_edges == 550_000 and inst.n_trips == 1_410_000
    with pytest.raises(SystemExit):
        bench.make_workload("nonsense")


def test_surrogate_entry_points_validate_arguments():
    lib = lpsim.load_library()
    v = ctypes.c_void_p(0x1000)  # never dereferenced: the checks fail first
    f = ctypes.c_float
    assert lib.lpsim_surrogate_features(10, 13, 600, f(7.0), v, v, v, v, v, v, None) == lpsim.EINVAL  # bins % 12
    assert lib.lpsim_surrogate_features(0, 12, 600, f(7.0), v, v, v, v, v, v, None) == lpsim.EINVAL
    assert lib.lpsim_surrogate_targets(10, 24, None, v, v, v, v, None) == lpsim.EINVAL
    assert lib.lpsim_surrogate_tt(10, 24, v, v, f(1.5), f(100.0), v, None) == lpsim.EINVAL  # damping > 1
    assert lib.lpsim_surrogate_shift(10, 24, v, v, v, f(-1.0), f(100.0), v, None) == lpsim.EINVAL
    assert lib.lpsim_surrogate_shift(10, 24, v, v, v, f(1.0), f(0.5), v, None) == lpsim.EINVAL
    assert lib.lpsim_surrogate_edge_tt(10, 24, v, v, v, f(0.0), v, None) == lpsim.EINVAL
    assert lib.lpsim_surrogate_load(None, None, None, 5, v, 10, 12, 50, 100, v, v, None) == lpsim.EINVAL


def test_mlp_entry_points_validate_arguments():
    lib = lpsim.load_library()
    i, h, o = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    assert lib.lpsim_mlp_shape(ctypes.byref(i), ctypes.byref(h), ctypes.byref(o)) == 0
    assert (i.value, h.value, o.value) == (32, 256, 16)
    # data gradients and input in fragment order (16 + 3*256 + 32 features,
    # rows padded to 64, bfloat16), then the slice partials (144,144 binary32
    # parameters each)
    assert lib.lpsim_mlp_workspace_bytes(8192, 8) == 816 * 8192 * 2 + 8 * 144_144 * 4
    assert lib.lpsim_mlp_workspace_bytes(1001, 3) == 816 * 1024 * 2 + 3 * 144_144 * 4
    assert lib.lpsim_mlp_workspace_bytes(0, 1) == 144_144 * 4
    assert lib.lpsim_mlp_workspace_bytes(10, 0) == 0
    assert lib.lpsim_mlp_workspace_bytes(10, 1025) == 0
    assert lib.lpsim_mlp_workspace_bytes(-1, 4) == 0
    # argument checks run on the host, before any launch
    assert lib.lpsim_mlp_backward(None, None, None, None, None, None, None, 1, 10, None) == -1
    assert lib.lpsim_mlp_backward_noalloc(None, None, None, None, None, None, 1, 10, None) == -1


def test_fragment_order_layout():
    """to_matrix / from_matrix invert each other and place element (r, f) of
    a [rows][feats] matrix where the MFMA 16x16x32 operand of lane
    L = f%16 + 16*((r%32)//8) reads it: block (r//32, f//16), slot r%8."""
    import torch

    from paper_2406_08496_amd.surrogate import from_matrix, to_matrix

    rows, feats = 64, 48
    m = torch.arange(rows * feats, dtype=torch.int64).reshape(rows, feats)
    flat = from_matrix(m)
    for r, f in [(0, 0), (7, 15), (8, 0), (31, 47), (32, 16), (45, 33), (63, 47)]:
        lane = f % 16 + 16 * ((r % 32) // 8)
        off = ((r // 32) * (feats // 16) + f // 16) * 512 + lane * 8 + r % 8
        assert flat[off].item() == m[r, f].item()
    assert torch.equal(to_matrix(flat, rows, feats), m)


def test_bench_mlp_flop_model():
    import bench

    # 2 * (32*256 + 256*256 + 256*256 + 256*16) forward; backward adds the
    # data gradients of layers 2..4
    assert bench.MLP_FWD_FLOP == 286_720
    assert bench.MLP_BWD_FLOP == 286_720 + 2 * (256 * 256 + 256 * 256 + 256 * 16)


def test_signal_plan_generator():
    """The synthetic plan is a valid input: signals only at nodes with 3+
    approaches on both axes, every approach of such a node served in the
    phase of its axis, offsets inside the cycle, nothing elsewhere."""
    import numpy as np

    from paper_2406_08496_amd import synth

    inst = synth.grid_instance(seed=3, side=6, n_trips=10)
    p = synth.signal_plan(inst, seed=1, green_s=40.0, allred_s=5.0)
    indeg = np.bincount(inst.dst, minlength=inst.n_nodes)
    sig = p.n_phases > 0
    assert sig.any() and np.all(indeg[sig] >= 3)
    assert np.all(p.n_phases[sig] == 2) and np.all(p.green[sig] == 80) and np.all(p.allred[sig] == 10)
    cycle = 2 * (p.green + p.allred)
    assert np.all((p.offset[sig] >= 0) & (p.offset[sig] < cycle[sig]))
    served = p.edge_phase >= 0
    assert np.array_equal(served, sig[inst.dst])
    d = inst.node_xy[inst.dst] - inst.node_xy[inst.src]
    axis = np.where(np.abs(d[:, 0]) >= np.abs(d[:, 1]), 0, 1)
    assert np.array_equal(p.edge_phase[served], axis[served])
    # both phases present at every signalised node
    for n in np.nonzero(sig)[0]:
        assert set(p.edge_phase[inst.dst == n]) == {0, 1}
