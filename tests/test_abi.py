"""Host-side checks of the C ABI: the library loads and exports every entry point
include/gpe.h declares (no compute calls; CPU only)."""
import ctypes
import os
import re

from paper_2404_14401_amd import gpe

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "gpe.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gpe_[a-z_]+)\s*\(", src)))


def test_header_declarations_match_binding():
    assert declared() == sorted(gpe.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(gpe.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_error_message_is_empty_string_initially():
    assert isinstance(gpe.lib().gpe_last_error(), bytes)


def _desc(nx=64, ny=64, lx=8.0, ly=8.0, dt=0.01, g=1.0):
    return gpe.PlanDesc(nx, ny, lx, ly, dt, g, None, 0)


def test_invalid_plans_are_rejected_before_any_device_call():
    lib = gpe.lib()
    h = ctypes.c_void_p()
    for d in (_desc(nx=15), _desc(ny=16384), _desc(nx=96), _desc(dt=0.0), _desc(dt=-1e-3), _desc(g=-1.0),
              _desc(lx=0.0), _desc(dt=float("nan"))):
        rc = lib.gpe_plan_create(ctypes.byref(h), ctypes.byref(d))
        assert rc == gpe.ERR_INVALID
        assert lib.gpe_last_error()  # a message is left for the caller
    assert lib.gpe_plan_create(None, ctypes.byref(_desc())) == gpe.ERR_INVALID


def test_null_handles_are_rejected():
    lib = gpe.lib()
    assert lib.gpe_step_real(None, None, 1, 0.0, None) == gpe.ERR_INVALID
    assert lib.gpe_step_imag(None, None, 1, 0.0, None) == gpe.ERR_INVALID
    assert lib.gpe_sync(None) == gpe.ERR_INVALID
    assert lib.gpe_plan_destroy(None) == gpe.OK
    assert lib.gpe_batch_destroy(None) == gpe.OK
    assert lib.gpe_step_batched(None, None, 1, 0.0) == gpe.ERR_INVALID
    assert lib.gpe_batch_create(None, 0, None, None) == gpe.ERR_INVALID
