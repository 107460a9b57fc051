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
            names |= set(re.findall(r"\b(lbm(?:3d)?_[a-z0-9_]+)\s*\(", txt))
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
                                         ("pop_dtype", 7), ("perm_kind", 2), ("scheme", 2)])
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


def test_guo_form_requires_scalar_permeability():
    p = L.make_params(16, 16, 0.8, 0.4, 0.1, 1.0, 1e-6, 0.0, 1, L.LBM_F32_SHIFTED,
                      L.LBM_PERM_TENSOR, L.LBM_SCHEME_GUO)
    assert L.lbm_workspace_bytes(p) == 0
    p.perm_kind = L.LBM_PERM_SCALAR
    assert L.lbm_workspace_bytes(p) > 0


def test_local_rejects_unknown_pop_dtype_on_host():
    lp = L.lbm_local_params(0.8, 0.4, 0.1, 1e-6, 1e-6, 100, 1000, 5)
    one = (ctypes.c_int32 * 1)(0)
    side = (ctypes.c_int32 * 1)(8)
    mask = (ctypes.c_int32 * 1)(3)
    fake = ctypes.c_void_p(256 * 1024)  # never dereferenced: validation fails first
    st = L.lib().lbm_local_keff(ctypes.byref(lp), 1, one, one, side, mask, fake, 8, 8, fake,
                                None, None, None, 0, 0, fake, 1 << 20, None)
    assert st == L.LBM_EINVAL


def test_local_rejects_bad_avg_margin_on_host():
    one = (ctypes.c_int32 * 1)(0)
    side = (ctypes.c_int32 * 1)(8)
    mask = (ctypes.c_int32 * 1)(3)
    fake = ctypes.c_void_p(256 * 1024)  # never dereferenced: validation fails first
    for margin in (-1, 4, 9):          # side 8 leaves no inner window from m = 4 on
        lp = L.lbm_local_params(0.8, 0.4, 0.1, 1e-6, 1e-6, 100, 1000, L.LBM_F32_SHIFTED, margin)
        st = L.lib().lbm_local_keff(ctypes.byref(lp), 1, one, one, side, mask, fake, 8, 8, fake,
                                    None, None, None, 0, 0, fake, 1 << 20, None)
        assert st == L.LBM_EINVAL, margin
        assert b"avg_margin" in L.lib().lbm_last_error()


def test_local_rejects_unknown_schedule_on_host():
    one = (ctypes.c_int32 * 1)(0)
    side = (ctypes.c_int32 * 1)(8)
    mask = (ctypes.c_int32 * 1)(3)
    fake = ctypes.c_void_p(256 * 1024)  # never dereferenced: validation fails first
    for sched in (-1, 2):
        lp = L.lbm_local_params(0.8, 0.4, 0.1, 1e-6, 1e-6, 100, 1000, L.LBM_F32_SHIFTED, 0, sched)
        st = L.lib().lbm_local_keff(ctypes.byref(lp), 1, one, one, side, mask, fake, 8, 8, fake,
                                    None, None, None, 0, 0, fake, 1 << 20, None)
        assert st == L.LBM_EINVAL, sched
        assert b"schedule" in L.lib().lbm_last_error()


def test_local_workspace_grows_with_patches():
    a, b = L.lbm_local_workspace_bytes(1), L.lbm_local_workspace_bytes(1000)
    # per patch: two items and their reordered copy (16 B each), two sort keys, the drive mask
    assert b - a >= 999 * (2 * 16 + 2 * 16 + 2 * 4 + 4) - 4096


def test_d3q19_params_validated_on_host():
    ok = L.make_params3(64, 8, 8, 0.8, 0.4, 0.1)
    assert L.lbm3d_workspace_bytes(ok) > 2 * 19 * 64 * 8 * 8 * 4
    f64 = L.make_params3(64, 8, 8, 0.8, 0.4, 0.1, pop_dtype=L.LBM_F64)
    assert L.lbm3d_workspace_bytes(f64) > L.lbm3d_workspace_bytes(ok)
    for field, bad in (("nz", 0), ("tau", 0.49), ("eps", 0.0), ("nu", -1.0), ("walls_z", 2),
                       ("pop_dtype", 7), ("gz", float("nan")), ("nx", 1 << 20)):
        p = L.make_params3(64, 8, 8, 0.8, 0.4, 0.1)
        setattr(p, field, bad)
        if field == "nx":
            p.ny, p.nz = 1 << 10, 1 << 10
        assert L.lbm3d_workspace_bytes(p) == 0, field
        h = ctypes.c_void_p()
        fake = ctypes.c_void_p(256 * 1024)  # never dereferenced: validation fails first
        st = L.lib().lbm3d_init(ctypes.byref(h), ctypes.byref(p), fake, fake, 1 << 40, None)
        assert st == L.LBM_EINVAL and not h.value, field


def test_size_limits_on_host():
    """The largest grids each solver accepts: 9 (nx ny + 8192) < 2^31 for the
    D2Q9 grid; (nx ny nz + 65536) x 4 B (FP32) or 8 B (FP64) below 4 GiB for
    D3Q19 (32-bit byte offsets within a population plane)."""
    assert L.lbm_workspace_bytes(L.make_params(16384, 14336, 0.8, 0.4, 0.1)) > 0
    assert L.lbm_workspace_bytes(L.make_params(16384, 14592, 0.8, 0.4, 0.1)) == 0
    assert L.lbm3d_workspace_bytes(L.make_params3(1024, 1024, 1023, 0.8, 0.4, 0.1)) > 0
    assert L.lbm3d_workspace_bytes(L.make_params3(1024, 1024, 1024, 0.8, 0.4, 0.1)) == 0
    f64 = L.make_params3(1024, 1024, 511, 0.8, 0.4, 0.1, pop_dtype=L.LBM_F64)
    assert L.lbm3d_workspace_bytes(f64) > 0
    f64.nz = 512
    assert L.lbm3d_workspace_bytes(f64) == 0


def test_empty_and_degenerate_inputs_on_host():
    """Empty batches: zero local problems is a no-op (no pointer is read);
    an empty CNN batch, a block size that does not divide the grid and a
    zero-sized workspace request are rejected before any device work."""
    lp = L.lbm_local_params(0.8, 0.4, 0.1, 1e-6, 1e-6, 100, 1000, L.LBM_F32_SHIFTED, 0)
    st = L.lib().lbm_local_keff(ctypes.byref(lp), 0, None, None, None, None, None, 1, 1, None,
                                None, None, None, 0, 0, None, 0, None)
    assert st == L.LBM_OK
    fake = ctypes.c_void_p(256 * 1024)
    assert L.lib().lbm_cnn_forward(fake, 0, fake, 1, fake, None, fake, 1 << 20, None) == L.LBM_EINVAL
    assert L.lib().lbm_patch_stats(0, fake, fake, None) == L.LBM_EINVAL
    assert L.lbm_cnn_workspace_bytes(0, 0) == 0
    assert L.lib().lbm_block_average(fake, 10, 10, 1, 3, fake, None) == L.LBM_EINVAL
    assert L.lib().lbm_block_average(fake, 0, 10, 1, 1, fake, None) == L.LBM_EINVAL
    assert L.lbm_workspace_bytes(L.make_params(0, 8, 0.8, 0.4, 0.1)) == 0
    assert L.lbm_local_workspace_bytes(0) >= 0


def test_cnn_forward_rejects_bad_n_sym_on_host():
    fake = ctypes.c_void_p(256 * 1024)
    for n_sym in (0, 9):
        st = L.lib().lbm_cnn_forward(fake, 4, fake, n_sym, fake, None, fake, 1 << 30, None)
        assert st == L.LBM_EINVAL


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_cnn_forward_limited_rejects_negative_cap_on_host():
    fake = ctypes.c_void_p(256 * 1024)  # never dereferenced: validation fails first
    st = L.lib().lbm_cnn_forward_limited(fake, 4, fake, 1, fake, None, -1, fake, 1 << 20, None)
    assert st == L.LBM_EINVAL
    assert b"max_workgroups" in L.lib().lbm_last_error()
