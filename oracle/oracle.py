"""Python face of the FP64 CPU oracle (ctypes over liblbm_oracle.so).

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the benchmark's
CPU-baseline leg import this module. The product path never does.

The C library implements the scheme of Sec. 2 (Shan-Chen and Guo forms) and
the local problems of Sec. 3 (Eq. tensor-kappa). This module adds the plain
Python pieces that sit around it: parameter records, the coarse-grid
parameter mapping of Sec. 3 / Sec. 4.3, and block averages.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, replace

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")

OK, EINVAL, ENOTCONV, ENONFINITE = 0, -1, -3, -4


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP). Returns the library path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", _SRC,
                        "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("tau", ctypes.c_double),
                ("eps", ctypes.c_double), ("nu", ctypes.c_double), ("rho0", ctypes.c_double),
                ("walls_y", ctypes.c_int32), ("perm_kind", ctypes.c_int32),
                ("scheme", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(_Params)
        L.orc_step.argtypes = [pp, dp, dp, ctypes.c_double, ctypes.c_double, dp, dp]
        L.orc_moments.argtypes = [pp, dp, dp, ctypes.c_double, ctypes.c_double, dp, dp, dp, dp]
        L.orc_mean_velocity.argtypes = [pp, dp, dp, ctypes.c_double, ctypes.c_double, dp, dp]
        L.orc_init_rest.argtypes = [pp, dp]
        L.orc_run.argtypes = [pp, dp, dp, ctypes.c_double, ctypes.c_double, dp, ctypes.c_int64,
                              ctypes.c_int32, ctypes.c_double, ctypes.POINTER(ctypes.c_int64), dp]
        L.orc_run.restype = ctypes.c_int
        L.orc_local_keff.argtypes = [dp, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                     ctypes.c_double, ctypes.c_int64, ctypes.c_int32, dp,
                                     ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)]
        L.orc_local_keff.restype = ctypes.c_int
        L.orc_block_average.argtypes = [dp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, dp]
        L.orc_lattice.argtypes = [ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                  dp, ctypes.POINTER(ctypes.c_int32)]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass(frozen=True)
class Params:
    """Lattice-unit parameters of one run (Sec. 2)."""
    nx: int
    ny: int
    tau: float
    eps: float
    nu: float
    rho0: float = 1.0
    walls_y: int = 0
    perm_kind: int = 1   # 1 scalar kappa, 4 tensor [kxx, kxy, kyx, kyy]
    scheme: int = 0      # 0 Shan-Chen form (the method), 1 Guo form

    def c(self) -> _Params:
        return _Params(self.nx, self.ny, self.tau, self.eps, self.nu, self.rho0,
                       self.walls_y, self.perm_kind, self.scheme)


def lattice():
    """(ex, ey, w, opp) as the oracle holds them."""
    ex = (ctypes.c_int32 * 9)(); ey = (ctypes.c_int32 * 9)()
    w = (ctypes.c_double * 9)(); opp = (ctypes.c_int32 * 9)()
    lib().orc_lattice(ex, ey, w, opp)
    return np.array(ex), np.array(ey), np.array(w), np.array(opp)


def _perm(p: Params, perm) -> np.ndarray:
    perm = np.ascontiguousarray(perm, dtype=np.float64)
    assert perm.size == p.nx * p.ny * p.perm_kind, "permeability has the wrong size"
    return perm


def _force(p: Params, force):
    if force is None:
        return None
    force = np.ascontiguousarray(force, dtype=np.float64)
    assert force.shape == (p.ny, p.nx, 2)
    return force


def rest_state(p: Params) -> np.ndarray:
    f = np.empty((p.ny, p.nx, 9))
    lib().orc_init_rest(ctypes.byref(p.c()), _dp(f))
    return f


def step(p: Params, perm, f, g=(0.0, 0.0), force=None) -> np.ndarray:
    """One time step; returns the new populations [ny, nx, 9]."""
    perm = _perm(p, perm)
    force = _force(p, force)
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.empty_like(f)
    lib().orc_step(ctypes.byref(p.c()), _dp(perm), _dp(force), g[0], g[1], _dp(f), _dp(out))
    return out


def moments(p: Params, perm, f, g=(0.0, 0.0), force=None):
    """(rho, ux, uy), each [ny, nx]: density and flow velocity (Eq. u-of-S-C)."""
    perm = _perm(p, perm)
    force = _force(p, force)
    f = np.ascontiguousarray(f, dtype=np.float64)
    rho = np.empty((p.ny, p.nx)); ux = np.empty_like(rho); uy = np.empty_like(rho)
    lib().orc_moments(ctypes.byref(p.c()), _dp(perm), _dp(force), g[0], g[1], _dp(f), _dp(rho),
                      _dp(ux), _dp(uy))
    return rho, ux, uy


def mean_velocity(p: Params, perm, f, g=(0.0, 0.0), force=None) -> np.ndarray:
    perm = _perm(p, perm)
    force = _force(p, force)
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.empty(2)
    lib().orc_mean_velocity(ctypes.byref(p.c()), _dp(perm), _dp(force), g[0], g[1], _dp(f),
                            _dp(out))
    return out


@dataclass
class RunResult:
    f: np.ndarray
    steps: int
    status: int
    mean_u: np.ndarray


def run(p: Params, perm, g=(0.0, 0.0), f=None, max_steps: int = 1000, check_every: int = 0,
        tol: float = 0.0, force=None) -> RunResult:
    """Run from ``f`` (rest state if None) for at most ``max_steps`` steps,
    stopping once the mean velocity changes by <= tol (relative) between
    checks taken every ``check_every`` steps."""
    perm = _perm(p, perm)
    force = _force(p, force)
    f = rest_state(p) if f is None else np.array(f, dtype=np.float64, order="C", copy=True)
    steps = ctypes.c_int64(0)
    mu = np.empty(2)
    st = lib().orc_run(ctypes.byref(p.c()), _dp(perm), _dp(force), g[0], g[1], _dp(f),
                       max_steps, check_every, tol, ctypes.byref(steps), _dp(mu))
    if st == EINVAL:
        raise ValueError("oracle rejected the parameters")
    return RunResult(f, steps.value, st, mu)


@dataclass
class KeffResult:
    keff: np.ndarray      # [kxx, kxy, kyx, kyy]
    steps: np.ndarray     # per drive
    status: np.ndarray    # per drive


def local_keff(kappa_patch, tau: float, eps: float, nu: float, g: float = 1e-6,
               check_every: int = 100, tol: float = 1e-10, max_steps: int = 2_000_000,
               drive_mask: int = 3) -> KeffResult:
    """Effective permeability tensor of one periodic patch (Sec. 3, Eq. tensor-kappa)."""
    k = np.ascontiguousarray(kappa_patch, dtype=np.float64)
    side = k.shape[0]
    assert k.shape == (side, side)
    keff = np.empty(4)
    steps = (ctypes.c_int64 * 2)(); status = (ctypes.c_int32 * 2)()
    st = lib().orc_local_keff(_dp(k), side, tau, eps, nu, g, check_every, tol, max_steps,
                              drive_mask, _dp(keff), steps, status)
    if st == EINVAL:
        raise ValueError("oracle rejected the parameters")
    return KeffResult(keff, np.array(steps), np.array(status))


def block_average(field, r: int) -> np.ndarray:
    field = np.ascontiguousarray(field, dtype=np.float64)
    ny, nx = field.shape
    out = np.empty((ny // r, nx // r))
    lib().orc_block_average(_dp(field), nx, ny, r, _dp(out))
    return out


def coarse_params(fine: Params, r: int) -> tuple[Params, dict]:
    """Coarse-grid parameters (Sec. 3 and Sec. 4.3): the physical rho0, nu_eff,
    eps, nu and G are kept while dx and dt both grow by r (c fixed). In lattice
    units this gives tau_c = 1/2 + (tau_f - 1/2)/r, nu_c = nu_f / r,
    kappa_c = kappa_f / r^2, G_c = r G_f and u_c = u_f.
    Returns the coarse Params and the scale factors."""
    pc = replace(fine, nx=fine.nx // r, ny=fine.ny // r, tau=0.5 + (fine.tau - 0.5) / r,
                 nu=fine.nu / r)
    return pc, dict(kappa=1.0 / (r * r), force=float(r), velocity=1.0)


def set_threads(n: int) -> None:
    lib().orc_set_num_threads(int(n))


def num_threads() -> int:
    return int(lib().orc_num_threads())
