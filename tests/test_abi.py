"""The C ABI without a GPU: the library loads, exports every declared symbol,
and rejects invalid arguments on the host before touching the device."""
import ctypes
import os
import re

import pytest

from paper_1312_0195_amd import lbm as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    lib = L.lib()
    declared = _declared()
    assert declared, "no declarations found"
    missing = [n for n in sorted(declared) if not hasattr(lib, n)]
    assert not missing, missing
    assert set(L.EXPORTS) == declared


def test_status_strings():
    for s in (L.LBM_OK, L.LBM_EINVAL, L.LBM_EDEVICE, L.LBM_ENOTCONV, L.LBM_ENONFINITE,
              L.LBM_EWORKSPACE):
        assert L.lbm_status_str(s).startswith("LBM_")


def test_workspace_bytes_host_only():
    p = L.make_params(2048, 2048, 0.8, 0.4, 0.1, 1.0, 1e-6, 0.0, 1)
    n = L.lbm_workspace_bytes(p)
    # two FP32 population sets plus the coefficient plane, at least
    assert n >= 2 * 9 * 4 * 2048 * 2048 + 4 * 2048 * 2048
    p64 = L.make_params(64, 64, 0.8, 0.4, 0.1, 1.0, 1e-6, 0.0, 1, L.LBM_F64)
    assert L.lbm_workspace_bytes(p64) >= 2 * 9 * 8 * 64 * 64
    bad = L.make_params(64, 64, 0.49, 0.4, 0.1)
    assert L.lbm_workspace_bytes(bad) == 0


@pytest.mark.parametrize("field,value", [("tau", 0.4), ("eps", 0.0), ("eps", 1.5), ("nu", 0.0),
                                         ("nx", 0), ("rho0", -1.0), ("walls_y", 2),
                                         ("pop_dtype", 7), ("perm_kind", 2)])
def test_init_rejects_invalid_parameters_on_host(field, value):
    p = L.make_params(16, 16, 0.8, 0.4, 0.1, 1.0, 1e-6, 0.0, 1)
    setattr(p, field, value)
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(256 * 1024)  # never dereferenced: validation fails first
    st = L.lib().lbm_init(ctypes.byref(h), ctypes.byref(p), fake, None, fake, 1 << 30, None)
    assert st == L.LBM_EINVAL
    assert L.lbm_last_error()


def test_init_rejects_small_workspace_on_host():
    p = L.make_params(16, 16, 0.8, 0.4, 0.1, 1.0, 1e-6, 0.0, 1)
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(256 * 1024)
    st = L.lib().lbm_init(ctypes.byref(h), ctypes.byref(p), fake, None, fake, 16, None)
    assert st == L.LBM_EWORKSPACE


def test_step_rejects_null_handle():
    st = L.lib().lbm_step(None, 10, 0.0, 0, None, None)
    assert st == L.LBM_EINVAL
