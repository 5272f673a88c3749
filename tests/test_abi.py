"""The C-ABI library loads and exports every entry point that include/lpsim.h
declares (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_2406_08496_amd import lpsim

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "lpsim.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lpsim_[a-z_]+)\s*\(", text)))


def test_header_parses():
    names = declared_functions()
    for required in ("lpsim_load_network", "lpsim_load_trips", "lpsim_step", "lpsim_edge_stats"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = lpsim.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert name in lpsim.SIGNATURES, f"binding has no signature for {name}"


def test_binding_covers_only_declared_symbols():
    assert set(lpsim.SIGNATURES) == set(declared_functions())


def test_params_struct_matches_header_layout():
    # float x12, double, int32 x2, uint64, int32 x2, float x2
    assert ctypes.sizeof(lpsim.Params) == 12 * 4 + 8 + 2 * 4 + 8 + 2 * 4 + 2 * 4
    assert lpsim.Params.eps_b.offset == 84
    assert ctypes.sizeof(lpsim.Counters) == 12 * 8


def test_invalid_params_rejected_without_gpu():
    lib = lpsim.load_library()
    bad = lpsim.Params(**dict(lpsim.DEFAULT_PARAMS, delta=2))
    h = ctypes.c_void_p()
    assert lib.lpsim_create(ctypes.byref(bad), ctypes.byref(h)) == lpsim.EINVAL
    bad = lpsim.Params(**dict(lpsim.DEFAULT_PARAMS, bin_seconds=0.7))
    assert lib.lpsim_create(ctypes.byref(bad), ctypes.byref(h)) == lpsim.EINVAL
    for eps in (dict(eps_a=-1.0), dict(eps_b=101.0), dict(eps_a=float("nan"))):
        bad = lpsim.Params(**dict(lpsim.DEFAULT_PARAMS, **eps))
        assert lib.lpsim_create(ctypes.byref(bad), ctypes.byref(h)) == lpsim.EINVAL
    assert lib.lpsim_last_error(None) == b""


def test_no_gpu_means_device_error():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(lpsim.LpsimError) as ei:
        lpsim.Simulator()
    assert ei.value.code == lpsim.EDEVICE
