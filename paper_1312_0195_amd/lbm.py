"""Python binding of liblbm (ctypes).

Thin marshalling layer over the C ABI declared in include/lbm.h: the functions
keep the C names and only convert arguments. Device memory and streams come
from PyTorch (tensors are passed as raw pointers). Every step of the method
runs in the HIP library; if liblbm.so is missing this module raises instead of
falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_EDEVICE, LBM_ENOTCONV, LBM_ENONFINITE, LBM_EWORKSPACE = 0, -1, -2, -3, -4, -5
LBM_F32_SHIFTED, LBM_F64, LBM_F32_FAST = 0, 1, 2
LBM_PERM_SCALAR, LBM_PERM_TENSOR = 1, 4
LBM_SCHEME_SHAN_CHEN, LBM_SCHEME_GUO = 0, 1
LBM_SCHEDULE_GIVEN, LBM_SCHEDULE_COST = 0, 1
LBM_KEFF_SCALAR, LBM_KEFF_TENSOR = 0, 1

#: default FP32 step budget of the local problems (0: none). The FP32 state
#: is stored rebased on each item's mean momentum, which keeps every tensor
#: within 1e-4 of the fixed point relative to its largest diagonal entry; a
#: nearly blocked direction of a very heterogeneous patch (kappa spanning ten
#: e-folds) can still be short by a few 1e-4 of its own small value, and a
#: budget such as 10 000 steps re-runs those slow items with FP64 state.
FP32_STEP_BUDGET = 0

#: every symbol the header declares (checked against include/lbm.h by the tests)
EXPORTS = (
    "lbm_workspace_bytes", "lbm_init", "lbm_step", "lbm_fields", "lbm_get_populations",
    "lbm_set_populations", "lbm_steps_total", "lbm_destroy", "lbm_local_max_side",
    "lbm_local_workspace_bytes", "lbm_local_keff", "lbm_coarse_params",
    "lbm_coarse_workspace_bytes", "lbm_coarse_solve", "lbm_block_average", "lbm_status_str",
    "lbm_last_error",
    "lbm_cnn_param_count", "lbm_cnn_workspace_bytes", "lbm_cnn_forward", "lbm_cnn_forward_limited",
    "lbm_cnn_forward_noalloc", "lbm_cnn_forward_spread",
    "lbm_cnn_gradients",
    "lbm_cnn_train_step", "lbm_patch_stats",
    "lbm3d_workspace_bytes", "lbm3d_init", "lbm3d_step", "lbm3d_fields", "lbm3d_get_populations",
    "lbm3d_set_populations", "lbm3d_steps_total", "lbm3d_destroy",
)


class LbmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class lbm_params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("tau", ctypes.c_double),
                ("eps", ctypes.c_double), ("nu", ctypes.c_double), ("rho0", ctypes.c_double),
                ("gx", ctypes.c_double), ("gy", ctypes.c_double), ("walls_y", ctypes.c_int32),
                ("pop_dtype", ctypes.c_int32), ("perm_kind", ctypes.c_int32),
                ("scheme", ctypes.c_int32)]


class lbm3d_params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("tau", ctypes.c_double), ("eps", ctypes.c_double), ("nu", ctypes.c_double),
                ("rho0", ctypes.c_double), ("gx", ctypes.c_double), ("gy", ctypes.c_double),
                ("gz", ctypes.c_double), ("walls_z", ctypes.c_int32), ("pop_dtype", ctypes.c_int32)]


class lbm_local_params(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("eps", ctypes.c_double), ("nu", ctypes.c_double),
                ("g", ctypes.c_double), ("tol", ctypes.c_double),
                ("check_every", ctypes.c_int32), ("max_steps", ctypes.c_int64),
                ("pop_dtype", ctypes.c_int32), ("avg_margin", ctypes.c_int32),
                ("schedule", ctypes.c_int32), ("fp32_step_budget", ctypes.c_int32)]


class lbm_local_tile(ctypes.Structure):
    _fields_ = [("side", ctypes.c_int32), ("slot_threads", ctypes.c_int32)]


_lib = None
_vp = ctypes.c_void_p
_i32p = ctypes.POINTER(ctypes.c_int32)
_dp = ctypes.POINTER(ctypes.c_double)


def lib():
    """Load liblbm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LbmError(LBM_EDEVICE, f"{LIB_PATH} is missing: build it with "
                                    "`python -m paper_1312_0195_amd.build`")
    # torch ships its own HIP runtime; load it first so that liblbm binds to
    # the same one (two runtimes in one process do not share devices).
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    pp = ctypes.POINTER(lbm_params)
    L.lbm_workspace_bytes.argtypes = [pp]
    L.lbm_workspace_bytes.restype = ctypes.c_size_t
    L.lbm_init.argtypes = [ctypes.POINTER(_vp), pp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
    L.lbm_init.restype = ctypes.c_int
    L.lbm_step.argtypes = [_vp, ctypes.c_int64, ctypes.c_double, ctypes.c_int32,
                           ctypes.POINTER(ctypes.c_int64), _dp]
    L.lbm_step.restype = ctypes.c_int
    L.lbm_fields.argtypes = [_vp, _vp, _vp]
    L.lbm_fields.restype = ctypes.c_int
    L.lbm_get_populations.argtypes = [_vp, _vp]
    L.lbm_get_populations.restype = ctypes.c_int
    L.lbm_set_populations.argtypes = [_vp, _vp]
    L.lbm_set_populations.restype = ctypes.c_int
    L.lbm_steps_total.argtypes = [_vp]
    L.lbm_steps_total.restype = ctypes.c_int64
    L.lbm_destroy.argtypes = [_vp]
    L.lbm_destroy.restype = None
    p3 = ctypes.POINTER(lbm3d_params)
    L.lbm3d_workspace_bytes.argtypes = [p3]
    L.lbm3d_workspace_bytes.restype = ctypes.c_size_t
    L.lbm3d_init.argtypes = [ctypes.POINTER(_vp), p3, _vp, _vp, ctypes.c_size_t, _vp]
    L.lbm3d_init.restype = ctypes.c_int
    L.lbm3d_step.argtypes = [_vp, ctypes.c_int64, ctypes.c_double, ctypes.c_int32,
                             ctypes.POINTER(ctypes.c_int64), _dp]
    L.lbm3d_step.restype = ctypes.c_int
    for name in ("lbm3d_fields",):
        getattr(L, name).argtypes = [_vp, _vp, _vp]
        getattr(L, name).restype = ctypes.c_int
    for name in ("lbm3d_get_populations", "lbm3d_set_populations"):
        getattr(L, name).argtypes = [_vp, _vp]
        getattr(L, name).restype = ctypes.c_int
    L.lbm3d_steps_total.argtypes = [_vp]
    L.lbm3d_steps_total.restype = ctypes.c_int64
    L.lbm3d_destroy.argtypes = [_vp]
    L.lbm3d_destroy.restype = None
    L.lbm_local_max_side.argtypes = []
    L.lbm_local_max_side.restype = ctypes.c_int32
    L.lbm_local_workspace_bytes.argtypes = [ctypes.c_int32]
    L.lbm_local_workspace_bytes.restype = ctypes.c_size_t
    L.lbm_local_keff.argtypes = [ctypes.POINTER(lbm_local_params), ctypes.c_int32, _i32p, _i32p,
                                 _i32p, _i32p, _vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp,
                                 ctypes.POINTER(lbm_local_tile), ctypes.c_int32, ctypes.c_int32,
                                 _vp, ctypes.c_size_t, _vp]
    L.lbm_local_keff.restype = ctypes.c_int
    L.lbm_coarse_params.argtypes = [pp, ctypes.c_int32, pp]
    L.lbm_coarse_params.restype = ctypes.c_int
    L.lbm_coarse_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32]
    L.lbm_coarse_workspace_bytes.restype = ctypes.c_size_t
    L.lbm_coarse_solve.argtypes = [pp, ctypes.c_int32, _vp, ctypes.c_int32, _vp, ctypes.c_int64,
                                   ctypes.c_double, ctypes.c_int32, _vp, _vp,
                                   ctypes.POINTER(ctypes.c_int64), _vp, ctypes.c_size_t, _vp]
    L.lbm_coarse_solve.restype = ctypes.c_int
    L.lbm_block_average.argtypes = [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_int32, _vp, _vp]
    L.lbm_block_average.restype = ctypes.c_int
    L.lbm_cnn_param_count.argtypes = []
    L.lbm_cnn_param_count.restype = ctypes.c_int32
    L.lbm_cnn_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32]
    L.lbm_cnn_workspace_bytes.restype = ctypes.c_size_t
    L.lbm_patch_stats.argtypes = [ctypes.c_int32, _vp, _vp, _vp]
    L.lbm_patch_stats.restype = ctypes.c_int
    L.lbm_cnn_forward.argtypes = [_vp, ctypes.c_int32, _vp, ctypes.c_int32, _vp, _vp, _vp,
                                  ctypes.c_size_t, _vp]
    L.lbm_cnn_forward.restype = ctypes.c_int
    L.lbm_cnn_forward_limited.argtypes = [_vp, ctypes.c_int32, _vp, ctypes.c_int32, _vp, _vp, ctypes.c_int32,
                                          _vp, ctypes.c_size_t, _vp]
    L.lbm_cnn_forward_limited.restype = ctypes.c_int
    L.lbm_cnn_forward_noalloc.argtypes = [_vp, ctypes.c_int32, _vp, ctypes.c_int32, _vp, _vp, ctypes.c_int32,
                                          _vp]
    L.lbm_cnn_forward_noalloc.restype = ctypes.c_int
    L.lbm_cnn_forward_spread.argtypes = [_vp, ctypes.c_int32, _vp, ctypes.c_int32, _vp, _vp, ctypes.c_int32,
                                         _vp, ctypes.c_size_t, _vp]
    L.lbm_cnn_forward_spread.restype = ctypes.c_int
    L.lbm_cnn_gradients.argtypes = [_vp, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                    ctypes.c_size_t, _vp]
    L.lbm_cnn_gradients.restype = ctypes.c_int
    L.lbm_cnn_train_step.argtypes = [_vp, _vp, _vp, ctypes.c_int32, ctypes.c_float, ctypes.c_int32,
                                     _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
    L.lbm_cnn_train_step.restype = ctypes.c_int
    L.lbm_status_str.argtypes = [ctypes.c_int]
    L.lbm_status_str.restype = ctypes.c_char_p
    L.lbm_last_error.argtypes = []
    L.lbm_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _raise(status: int, where: str):
    if status != LBM_OK:
        raise LbmError(status, f"{where}: {lbm_last_error()}")


def _ptr(t) -> int | None:
    """Device pointer of a tensor (or None)."""
    return None if t is None else int(t.data_ptr())


def _stream(stream) -> int | None:
    if stream is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream)
    return int(stream)


# ---------------------------------------------------------------------------
# The C entry points, same names
# ---------------------------------------------------------------------------


def lbm_status_str(status: int) -> str:
    return lib().lbm_status_str(status).decode()


def lbm_last_error() -> str:
    return lib().lbm_last_error().decode()


def lbm_workspace_bytes(p: lbm_params) -> int:
    return int(lib().lbm_workspace_bytes(ctypes.byref(p)))


def lbm_init(p: lbm_params, d_perm, d_force, d_ws, ws_bytes: int, stream=None) -> ctypes.c_void_p:
    h = _vp()
    st = lib().lbm_init(ctypes.byref(h), ctypes.byref(p), _ptr(d_perm), _ptr(d_force),
                        _ptr(d_ws), ws_bytes, _stream(stream))
    _raise(st, "lbm_init")
    return h


def lbm_step(h, max_steps: int, tol: float = 0.0, check_every: int = 0, mean: bool = True):
    """Returns (status, steps_done, mean_u); raises on errors other than
    LBM_ENOTCONV and LBM_ENONFINITE, which are returned. With mean=False no
    mean velocity is asked for (mean_u NULL): the call then waits for the
    device only at the checks that fall within it, and mean_u is NaN."""
    steps = ctypes.c_int64(0)
    mu = (ctypes.c_double * 2)(np.nan, np.nan)
    st = lib().lbm_step(h, int(max_steps), float(tol), int(check_every), ctypes.byref(steps),
                        mu if mean else None)
    if st not in (LBM_OK, LBM_ENOTCONV, LBM_ENONFINITE):
        _raise(st, "lbm_step")
    return st, steps.value, np.array([mu[0], mu[1]])


def lbm_fields(h, d_u, d_rho=None) -> None:
    _raise(lib().lbm_fields(h, _ptr(d_u), _ptr(d_rho)), "lbm_fields")


def lbm_get_populations(h, d_f) -> None:
    _raise(lib().lbm_get_populations(h, _ptr(d_f)), "lbm_get_populations")


def lbm_set_populations(h, d_f) -> None:
    _raise(lib().lbm_set_populations(h, _ptr(d_f)), "lbm_set_populations")


def lbm_steps_total(h) -> int:
    return int(lib().lbm_steps_total(h))


def lbm_destroy(h) -> None:
    lib().lbm_destroy(h)


def lbm3d_workspace_bytes(p: lbm3d_params) -> int:
    return int(lib().lbm3d_workspace_bytes(ctypes.byref(p)))


def lbm3d_init(p: lbm3d_params, d_kappa, d_ws, ws_bytes: int, stream=None) -> ctypes.c_void_p:
    h = _vp()
    st = lib().lbm3d_init(ctypes.byref(h), ctypes.byref(p), _ptr(d_kappa), _ptr(d_ws), ws_bytes,
                          _stream(stream))
    _raise(st, "lbm3d_init")
    return h


def lbm3d_step(h, max_steps: int, tol: float = 0.0, check_every: int = 0):
    """Returns (status, steps_done, mean_u[3]), as lbm_step."""
    steps = ctypes.c_int64(0)
    mu = (ctypes.c_double * 3)()
    st = lib().lbm3d_step(h, int(max_steps), float(tol), int(check_every), ctypes.byref(steps), mu)
    if st not in (LBM_OK, LBM_ENOTCONV, LBM_ENONFINITE):
        _raise(st, "lbm3d_step")
    return st, steps.value, np.array([mu[0], mu[1], mu[2]])


def lbm3d_fields(h, d_u, d_rho=None) -> None:
    _raise(lib().lbm3d_fields(h, _ptr(d_u), _ptr(d_rho)), "lbm3d_fields")


def lbm3d_get_populations(h, d_f) -> None:
    _raise(lib().lbm3d_get_populations(h, _ptr(d_f)), "lbm3d_get_populations")


def lbm3d_set_populations(h, d_f) -> None:
    _raise(lib().lbm3d_set_populations(h, _ptr(d_f)), "lbm3d_set_populations")


def lbm3d_steps_total(h) -> int:
    return int(lib().lbm3d_steps_total(h))


def lbm3d_destroy(h) -> None:
    lib().lbm3d_destroy(h)


def lbm_local_max_side() -> int:
    return int(lib().lbm_local_max_side())


def lbm_local_workspace_bytes(n_patches: int) -> int:
    return int(lib().lbm_local_workspace_bytes(int(n_patches)))


def _host_i32(a, n):
    a = np.ascontiguousarray(a, dtype=np.int32)
    assert a.shape == (n,)
    return a, a.ctypes.data_as(_i32p)


def lbm_local_keff(lp: lbm_local_params, x0, y0, side, drive_mask, d_kappa_field, d_keff,
                   d_steps=None, d_flags=None, tiles=None, block_threads: int = 0, d_ws=None,
                   ws_bytes: int = 0, stream=None) -> None:
    n = len(x0)
    fny, fnx = d_kappa_field.shape
    hx, px = _host_i32(x0, n)
    hy, py = _host_i32(y0, n)
    hs, ps = _host_i32(side, n)
    hm, pm = _host_i32(drive_mask, n)
    if tiles:
        arr = (lbm_local_tile * len(tiles))(*[lbm_local_tile(int(s), int(t)) for s, t in tiles])
        ntiles = len(tiles)
    else:
        arr, ntiles = None, 0
    st = lib().lbm_local_keff(ctypes.byref(lp), n, px, py, ps, pm, _ptr(d_kappa_field), fnx, fny,
                              _ptr(d_keff), _ptr(d_steps), _ptr(d_flags), arr, ntiles,
                              int(block_threads), _ptr(d_ws), int(ws_bytes), _stream(stream))
    _raise(st, "lbm_local_keff")


def lbm_coarse_params(fine: lbm_params, r: int) -> lbm_params:
    out = lbm_params()
    _raise(lib().lbm_coarse_params(ctypes.byref(fine), int(r), ctypes.byref(out)),
           "lbm_coarse_params")
    return out


def lbm_coarse_workspace_bytes(ncx: int, ncy: int) -> int:
    return int(lib().lbm_coarse_workspace_bytes(int(ncx), int(ncy)))


def lbm_coarse_solve(fine: lbm_params, r: int, d_keff, keff_mode: int, d_force, max_steps: int,
                     tol: float, check_every: int, d_u, d_rho, d_ws, ws_bytes: int, stream=None):
    """Returns (status, steps_done); raises on errors other than LBM_ENOTCONV."""
    steps = ctypes.c_int64(0)
    st = lib().lbm_coarse_solve(ctypes.byref(fine), int(r), _ptr(d_keff), int(keff_mode),
                                _ptr(d_force), int(max_steps), float(tol), int(check_every),
                                _ptr(d_u), _ptr(d_rho), ctypes.byref(steps), _ptr(d_ws),
                                int(ws_bytes), _stream(stream))
    if st not in (LBM_OK, LBM_ENOTCONV):
        _raise(st, "lbm_coarse_solve")
    return st, steps.value


def lbm_block_average(d_in, nx, ny, nplanes, r, d_out, stream=None) -> None:
    _raise(lib().lbm_block_average(_ptr(d_in), int(nx), int(ny), int(nplanes), int(r), _ptr(d_out),
                                   _stream(stream)), "lbm_block_average")


def lbm_cnn_param_count() -> int:
    return int(lib().lbm_cnn_param_count())


def lbm_cnn_workspace_bytes(batch: int, training: bool) -> int:
    return int(lib().lbm_cnn_workspace_bytes(int(batch), int(bool(training))))


def lbm_patch_stats(batch, d_logk, d_stats, stream=None) -> None:
    _raise(lib().lbm_patch_stats(int(batch), _ptr(d_logk), _ptr(d_stats), _stream(stream)),
           "lbm_patch_stats")


def lbm_cnn_forward(d_params, batch, d_logk, n_sym, d_pred, d_stats, d_ws, ws_bytes,
                    stream=None) -> None:
    _raise(lib().lbm_cnn_forward(_ptr(d_params), int(batch), _ptr(d_logk), int(n_sym), _ptr(d_pred),
                                 _ptr(d_stats), _ptr(d_ws), int(ws_bytes), _stream(stream)),
           "lbm_cnn_forward")


def lbm_cnn_forward_limited(d_params, batch, d_logk, n_sym, d_pred, d_stats, max_workgroups, d_ws,
                            ws_bytes, stream=None) -> None:
    _raise(lib().lbm_cnn_forward_limited(_ptr(d_params), int(batch), _ptr(d_logk), int(n_sym),
                                         _ptr(d_pred), _ptr(d_stats), int(max_workgroups), _ptr(d_ws),
                                         int(ws_bytes), _stream(stream)), "lbm_cnn_forward_limited")


def lbm_cnn_forward_spread(d_params, batch, d_logk, n_sym, d_pred, d_spread, max_workgroups, d_ws,
                           ws_bytes, stream=None) -> None:
    _raise(lib().lbm_cnn_forward_spread(_ptr(d_params), int(batch), _ptr(d_logk), int(n_sym),
                                        _ptr(d_pred), _ptr(d_spread), int(max_workgroups), _ptr(d_ws),
                                        int(ws_bytes), _stream(stream)), "lbm_cnn_forward_spread")


def lbm_cnn_forward_noalloc(d_params, batch, d_logk, n_sym, d_pred, d_stats, max_workgroups=0,
                            stream=None) -> None:
    _raise(lib().lbm_cnn_forward_noalloc(_ptr(d_params), int(batch), _ptr(d_logk), int(n_sym),
                                         _ptr(d_pred), _ptr(d_stats), int(max_workgroups),
                                         _stream(stream)), "lbm_cnn_forward_noalloc")


def lbm_cnn_gradients(d_params, batch, d_logk, d_sym, d_target, d_grad, d_loss, d_pred, d_ws,
                      ws_bytes, stream=None) -> None:
    _raise(lib().lbm_cnn_gradients(_ptr(d_params), int(batch), _ptr(d_logk), _ptr(d_sym),
                                   _ptr(d_target), _ptr(d_grad), _ptr(d_loss), _ptr(d_pred),
                                   _ptr(d_ws), int(ws_bytes), _stream(stream)), "lbm_cnn_gradients")


def lbm_cnn_train_step(d_params, d_m, d_v, step, lr, batch, d_logk, d_sym, d_target, d_loss, d_ws,
                       ws_bytes, stream=None) -> None:
    _raise(lib().lbm_cnn_train_step(_ptr(d_params), _ptr(d_m), _ptr(d_v), int(step), float(lr),
                                    int(batch), _ptr(d_logk), _ptr(d_sym), _ptr(d_target),
                                    _ptr(d_loss), _ptr(d_ws), int(ws_bytes), _stream(stream)),
           "lbm_cnn_train_step")


# ---------------------------------------------------------------------------
# Convenience wrappers (device memory from torch; no arithmetic of the method)
# ---------------------------------------------------------------------------


def make_params(nx, ny, tau, eps, nu, rho0=1.0, gx=0.0, gy=0.0, walls_y=0,
                pop_dtype=LBM_F32_SHIFTED, perm_kind=LBM_PERM_SCALAR,
                scheme=LBM_SCHEME_SHAN_CHEN) -> lbm_params:
    return lbm_params(int(nx), int(ny), float(tau), float(eps), float(nu), float(rho0), float(gx),
                      float(gy), int(walls_y), int(pop_dtype), int(perm_kind), int(scheme))


def _workspace(nbytes: int, device):
    import torch
    # torch's caching allocator hands out 512-byte aligned blocks
    ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
    assert ws.data_ptr() % 256 == 0
    return ws


class FineSolver:
    """Owns the torch buffers of one lbm_handle."""

    def __init__(self, p: lbm_params, kappa, force=None, device="cuda"):
        import torch
        self.p = p
        self.device = torch.device(device)
        kappa = torch.as_tensor(np.ascontiguousarray(kappa), dtype=torch.float64)
        self.kappa = kappa.to(self.device).contiguous()
        self.force = None
        if force is not None:
            self.force = torch.as_tensor(np.ascontiguousarray(force), dtype=torch.float64).to(
                self.device).contiguous()
        nbytes = lbm_workspace_bytes(p)
        if nbytes == 0:
            raise LbmError(LBM_EINVAL, "invalid parameters")
        self.ws = _workspace(nbytes, self.device)
        self.h = lbm_init(p, self.kappa, self.force, self.ws, nbytes)

    def step(self, max_steps, tol=0.0, check_every=0, mean=True):
        return lbm_step(self.h, max_steps, tol, check_every, mean)

    def fields(self):
        import torch
        u = torch.empty((2, self.p.ny, self.p.nx), dtype=torch.float64, device=self.device)
        rho = torch.empty((self.p.ny, self.p.nx), dtype=torch.float64, device=self.device)
        lbm_fields(self.h, u, rho)
        torch.cuda.synchronize(self.device)
        return u, rho

    def populations(self):
        import torch
        f = torch.empty((9, self.p.ny, self.p.nx), dtype=torch.float64, device=self.device)
        lbm_get_populations(self.h, f)
        torch.cuda.synchronize(self.device)
        return f

    def set_populations(self, f):
        import torch
        f = torch.as_tensor(f, dtype=torch.float64).to(self.device).contiguous()
        lbm_set_populations(self.h, f)
        torch.cuda.synchronize(self.device)

    @property
    def steps_total(self):
        return lbm_steps_total(self.h)

    def close(self):
        if getattr(self, "h", None) is not None:
            lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solver3D:
    """Owns the torch buffers of one lbm3d_handle (D3Q19 fine grid)."""

    def __init__(self, p: lbm3d_params, kappa, device="cuda"):
        import torch
        self.p = p
        self.device = torch.device(device)
        k = torch.as_tensor(np.ascontiguousarray(kappa) if isinstance(kappa, np.ndarray) else kappa,
                            dtype=torch.float64)
        self.kappa = k.to(self.device).contiguous()
        nbytes = lbm3d_workspace_bytes(p)
        if nbytes == 0:
            raise LbmError(LBM_EINVAL, "invalid parameters")
        self.ws = _workspace(nbytes, self.device)
        self.h = lbm3d_init(p, self.kappa, self.ws, nbytes)

    def step(self, max_steps, tol=0.0, check_every=0):
        return lbm3d_step(self.h, max_steps, tol, check_every)

    def fields(self):
        import torch
        shape = (self.p.nz, self.p.ny, self.p.nx)
        u = torch.empty((3,) + shape, dtype=torch.float64, device=self.device)
        rho = torch.empty(shape, dtype=torch.float64, device=self.device)
        lbm3d_fields(self.h, u, rho)
        torch.cuda.synchronize(self.device)
        return u, rho

    def populations(self):
        import torch
        f = torch.empty((19, self.p.nz, self.p.ny, self.p.nx), dtype=torch.float64,
                        device=self.device)
        lbm3d_get_populations(self.h, f)
        torch.cuda.synchronize(self.device)
        return f

    def set_populations(self, f):
        import torch
        f = torch.as_tensor(f, dtype=torch.float64).to(self.device).contiguous()
        lbm3d_set_populations(self.h, f)
        torch.cuda.synchronize(self.device)

    @property
    def steps_total(self):
        return lbm3d_steps_total(self.h)

    def close(self):
        if getattr(self, "h", None) is not None:
            lbm3d_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_params3(nx, ny, nz, tau, eps, nu, rho0=1.0, g=(0.0, 0.0, 0.0), walls_z=0,
                 pop_dtype=LBM_F32_SHIFTED) -> lbm3d_params:
    return lbm3d_params(int(nx), int(ny), int(nz), float(tau), float(eps), float(nu), float(rho0),
                        float(g[0]), float(g[1]), float(g[2]), int(walls_z), int(pop_dtype))


@dataclass
class LocalResult:
    keff: np.ndarray   # [n, 4] kxx, kxy, kyx, kyy
    steps: np.ndarray  # [n, 2]
    flags: np.ndarray  # [n, 2]


def local_keff(kappa_field, x0, y0, side, tau, eps, nu, g=1e-6, tol=1e-6, check_every=100,
               max_steps=200000, drive_mask=None, tiles=None, block_threads=0, device="cuda",
               kappa_dev=None, use_tuned=True, pop_dtype=LBM_F32_SHIFTED,
               avg_margin=0, schedule=None, fp32_step_budget=None) -> LocalResult:
    """Run lbm_local_keff on a field (host array or device tensor) and return
    host results. Without explicit tiles, the autotuned table is used when
    one exists (see paper_1312_0195_amd.autotune); without an explicit
    schedule, the table's, else LBM_SCHEDULE_COST. fp32_step_budget: FP32
    items still running after this many steps are re-run with FP64 state
    (default FP32_STEP_BUDGET; 0 = never)."""
    import torch
    if tiles is None and block_threads == 0 and use_tuned:
        from .autotune import load_table
        block_threads, tiles = load_table()
    if schedule is None:
        from .autotune import load_schedule
        schedule = load_schedule() if use_tuned else None
        schedule = LBM_SCHEDULE_COST if schedule is None else schedule
    n = len(x0)
    dev = torch.device(device)
    kd = kappa_dev if kappa_dev is not None else torch.as_tensor(
        np.ascontiguousarray(kappa_field), dtype=torch.float64).to(dev)
    keff = torch.empty((n, 4), dtype=torch.float64, device=dev)
    steps = torch.empty((n, 2), dtype=torch.int32, device=dev)
    flags = torch.empty((n, 2), dtype=torch.int32, device=dev)
    nbytes = lbm_local_workspace_bytes(n)
    ws = _workspace(nbytes, dev)
    budget = FP32_STEP_BUDGET if fp32_step_budget is None else fp32_step_budget
    lp = lbm_local_params(float(tau), float(eps), float(nu), float(g), float(tol),
                          int(check_every), int(max_steps), int(pop_dtype), int(avg_margin),
                          int(schedule), int(budget))
    dm = np.full(n, 3, np.int32) if drive_mask is None else drive_mask
    lbm_local_keff(lp, x0, y0, side, dm, kd, keff, steps, flags, tiles, block_threads, ws,
                   nbytes)
    torch.cuda.synchronize(dev)
    return LocalResult(keff.cpu().numpy(), steps.cpu().numpy(), flags.cpu().numpy())
