"""The upscaled method end to end (Sec. 3, Sec. 4.3), on the GPU.

    fine permeability field (periodic)
      -> batched local problems on the r x r subdomains (lbm_local_keff)
      -> effective permeability tensor per coarse cell (Eq. tensor-kappa)
      -> coarse-grid solve (lbm_coarse_solve, scalar or tensor drag)
    compared with
      fine-grid solve to steady state (lbm_step) -> velocity (lbm_fields)
      -> r x r block averages (lbm_block_average)

The comparison metric is the relative L2 difference of the velocity fields on
the coarse grid. Every step runs in the HIP library; torch holds the buffers.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np

from . import lbm as L


@dataclass
class UpscaleResult:
    keff: np.ndarray          # [ncy, ncx, 4] fine lattice units
    u_coarse: np.ndarray      # [2, ncy, ncx]
    u_fine_avg: np.ndarray    # [2, ncy, ncx]
    rel_l2: float
    rel_l2_scalar: float
    t_local: float
    t_coarse: float
    t_fine: float
    fine_steps: int
    fine_status: int
    coarse_steps: int
    local_flags_ok: bool


def _rel_l2(a, b):
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))


def local_tensor(kappa_dev, r, tau, eps, nu, g, tol=1e-7):
    """K_eff per r x r subdomain of a periodic field: [ncy, ncx, 4]."""
    ny, nx = kappa_dev.shape
    ncy, ncx = ny // r, nx // r
    J, I = np.meshgrid(np.arange(ncy), np.arange(ncx), indexing="ij")
    x0 = (I.ravel() * r).astype(np.int32)
    y0 = (J.ravel() * r).astype(np.int32)
    side = np.full(x0.shape, r, np.int32)
    res = L.local_keff(None, x0, y0, side, tau, eps, nu, g, tol=tol, check_every=100,
                       max_steps=2_000_000, kappa_dev=kappa_dev)
    return res.keff.reshape(ncy, ncx, 4), bool((res.flags == 0).all())


def coarse_solve(kappa_shape, keff, r, tau, eps, nu, g, mode, tol=1e-7, max_steps=4_000_000,
                 pop_dtype=None):
    import torch
    ny, nx = kappa_shape
    ncy, ncx = keff.shape[:2]
    fine = L.make_params(nx, ny, tau, eps, nu, 1.0, g, 0.0, 0,
                         L.LBM_F32_SHIFTED if pop_dtype is None else pop_dtype)
    kd = torch.as_tensor(np.ascontiguousarray(keff)).cuda()
    u = torch.empty((2, ncy, ncx), dtype=torch.float64, device="cuda")
    nb = L.lbm_coarse_workspace_bytes(ncx, ncy)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    st, steps = L.lbm_coarse_solve(fine, r, kd, mode, None, max_steps, tol, 100, u, None, ws, nb)
    return u.cpu().numpy(), steps, st


def fine_solve(kappa, tau, eps, nu, g, tol=1e-7, max_steps=2_000_000, check_every=1000):
    """Fine-grid velocity at steady state (periodic), [2, ny, nx] on device."""
    import torch
    ny, nx = kappa.shape
    p = L.make_params(nx, ny, tau, eps, nu, 1.0, g, 0.0, 0, L.LBM_F32_SHIFTED)
    s = L.FineSolver(p, kappa)
    st, steps, _ = s.step(max_steps, tol, check_every)
    u = torch.empty((2, ny, nx), dtype=torch.float64, device="cuda")
    L.lbm_fields(s.h, u, None)
    return u, steps, st, s


def block_average(u_dev, r):
    import torch
    planes, ny, nx = u_dev.shape
    out = torch.empty((planes, ny // r, nx // r), dtype=torch.float64, device=u_dev.device)
    L.lbm_block_average(u_dev, nx, ny, planes, r, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def run(kappa, r, tau=0.8, eps=0.4, nu=0.1, g=1e-6, fine_tol=1e-7, fine_max_steps=2_000_000,
        fine_check=1000, coarse_tol=1e-7) -> UpscaleResult:
    import torch
    kd = torch.as_tensor(np.ascontiguousarray(kappa)).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    keff, ok = local_tensor(kd, r, tau, eps, nu, g)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    u_c, c_steps, _ = coarse_solve(kappa.shape, keff, r, tau, eps, nu, g, L.LBM_KEFF_TENSOR,
                                   coarse_tol)
    t2 = time.perf_counter()
    u_cs, _, _ = coarse_solve(kappa.shape, keff, r, tau, eps, nu, g, L.LBM_KEFF_SCALAR, coarse_tol)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    u_f, f_steps, f_st, solver = fine_solve(kappa, tau, eps, nu, g, fine_tol, fine_max_steps,
                                            fine_check)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    u_avg = block_average(u_f, r)
    solver.close()
    return UpscaleResult(keff, u_c, u_avg, _rel_l2(u_c, u_avg), _rel_l2(u_cs, u_avg),
                         t1 - t0, t2 - t1, t4 - t3, f_steps, f_st, c_steps, ok)
