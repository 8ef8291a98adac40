"""CPU-side checks of the C ABI: the library loads, exports every entry point
the header declares, and fails cleanly (no crash) where no GPU is present."""
import ctypes
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def P():
    from paper_2110_00085_amd import prt
    if not os.path.exists(prt.LIB_PATH):
        pytest.skip("libprt.so not built (run __graft_entry__.build())")
    return prt


def test_header_entry_points_are_exported(P):
    names = P.header_entry_points()
    assert len(names) >= 18
    out = subprocess.run(["nm", "-D", "--defined-only", P.LIB_PATH], capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    lib = P.lib()
    for n in names:
        assert hasattr(lib, n)


def test_binding_names_match_header(P):
    for n in P.header_entry_points():
        assert callable(getattr(P, n, None)), f"binding lacks {n}"


def test_kernel_names_and_last_error(P):
    assert P.prt_kernel_name(4) == "render"
    assert P.prt_kernel_name(999) == "unknown"
    assert isinstance(P.lib().prt_last_error(), bytes)


def test_null_arguments_are_rejected_before_any_device_work(P):
    L = P.lib()
    assert L.prt_render(None, None, None, None, 0, None) == P.PRT_E_INVALID
    assert L.prt_grad(None, None, None, None, None, None) == P.PRT_E_INVALID
    assert L.prt_loss(None, 0, None, None, None, None) == P.PRT_E_INVALID
    assert L.prt_paths_info(None, None) == P.PRT_E_INVALID
    L.prt_paths_destroy(None)
    L.prt_destroy(None)
    # reflectometry calls (prt_surface.h)
    assert L.prt_surface_render(None, None, None, None) == P.PRT_E_INVALID
    assert L.prt_surface_grad(None, None, None, None, None) == P.PRT_E_INVALID
    assert L.prt_surface_reweight(None, None, None, None) == P.PRT_E_INVALID
    assert L.prt_surface_adam(None, None, None, None, None, 1, 0.1, 0.1, 0.9, 0.999, 1e-8) == P.PRT_E_INVALID
    assert L.prt_surface_info(None, None, None) == P.PRT_E_INVALID
    assert L.prt_surface_sample(None, None, None, None, 0, 1, None) == P.PRT_E_INVALID
    assert L.prt_surface_resample(None, None, None, None, None, 0, 1) == P.PRT_E_INVALID
    assert L.prt_surface_resample_device(None, None, None, None, None, 0, 1) == P.PRT_E_INVALID
    L.prt_surface_destroy(None)


def test_create_without_gpu_fails_cleanly(P):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    rc = P.lib().prt_create(0, None, 0, ctypes.byref(h))
    assert rc == P.PRT_E_HIP and h.value is None
    assert b"device" in P.lib().prt_last_error()
