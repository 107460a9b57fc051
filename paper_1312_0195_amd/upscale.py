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

Oversampling (the paper names it as a remedy for high contrast and channels,
without details): the local problem of a coarse cell runs on a periodic
window of side r + 2m centred on the cell, and only the cell's own r x r
block enters the mean velocity (lbm_local_keff's avg_margin), so the
artificial periodic boundary sits m cells away from the cells averaged.

    python -m paper_1312_0195_amd.upscale [--n 4096] [--r 64] [--channels] [--margins 0,8,16]

runs the upscaling workload (log-normal K, sigma 2, correlation length
64 n / 4096, periodic; optionally with high-permeability streaks) and prints
the timings and errors as one JSON line.
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
    rel_l2_geomean: float     # coarse run with the block geometric mean of kappa instead of K*
    by_margin: dict           # oversampling margin -> rel. L2 of u (tensor, scalar), local seconds
    mean_err: float           # relative error of the domain-mean velocity, tensor K*
    t_local: float
    t_coarse: float
    t_fine: float
    fine_steps: int
    fine_status: int
    coarse_steps: int
    local_flags_ok: bool


def _rel_l2(a, b):
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))


def local_tensor(kappa_dev, r, tau, eps, nu, g, tol=1e-7, margin=0):
    """K_eff per r x r subdomain of a periodic field: [ncy, ncx, 4]. With
    margin m > 0 each local problem runs on the (r + 2m)-sided window centred
    on its subdomain (wrapping around the field) and averages over the
    subdomain only."""
    ny, nx = kappa_dev.shape
    ncy, ncx = ny // r, nx // r
    J, I = np.meshgrid(np.arange(ncy), np.arange(ncx), indexing="ij")
    x0 = ((I.ravel() * r - margin) % nx).astype(np.int32)
    y0 = ((J.ravel() * r - margin) % ny).astype(np.int32)
    side = np.full(x0.shape, r + 2 * margin, np.int32)
    res = L.local_keff(None, x0, y0, side, tau, eps, nu, g, tol=tol, check_every=100,
                       max_steps=2_000_000, kappa_dev=kappa_dev, avg_margin=margin)
    # flag 3: converged in FP32 state past the FP32 step budget (a side too
    # large for the FP64 re-run); converged, with the FP32 state's accuracy
    return res.keff.reshape(ncy, ncx, 4), bool(np.isin(res.flags, (0, 3)).all())


def coarse_solve(kappa_shape, keff, r, tau, eps, nu, g, mode, tol=1e-7, max_steps=4_000_000,
                 pop_dtype=None, check_every=100):
    import torch
    ny, nx = kappa_shape
    ncy, ncx = keff.shape[:2]
    fine = L.make_params(nx, ny, tau, eps, nu, 1.0, g, 0.0, 0,
                         L.LBM_F32_SHIFTED if pop_dtype is None else pop_dtype)
    kd = torch.as_tensor(np.ascontiguousarray(keff)).cuda()
    u = torch.empty((2, ncy, ncx), dtype=torch.float64, device="cuda")
    nb = L.lbm_coarse_workspace_bytes(ncx, ncy)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    st, steps = L.lbm_coarse_solve(fine, r, kd, mode, None, max_steps, tol, check_every, u, None,
                                   ws, nb)
    return u.cpu().numpy(), steps, st


def fine_solve(kappa, tau, eps, nu, g, tol=1e-7, max_steps=2_000_000, check_every=1000,
               chunk=None, verbose=False):
    """Fine-grid velocity at steady state (periodic), [2, ny, nx] on device.
    With chunk set, runs in calls of that many steps (a multiple of
    check_every; the solver keeps its last check across calls) and prints
    progress after each."""
    import torch
    ny, nx = kappa.shape
    p = L.make_params(nx, ny, tau, eps, nu, 1.0, g, 0.0, 0, L.LBM_F32_SHIFTED)
    s = L.FineSolver(p, kappa)
    chunk = max_steps if chunk is None else chunk
    steps, st = 0, L.LBM_ENOTCONV
    t0 = time.perf_counter()
    while steps < max_steps:
        st, done, mu = s.step(min(chunk, max_steps - steps), tol, check_every)
        steps += done
        if verbose:
            print(f"fine: {steps} steps, mean u {mu[0]:.9e} {mu[1]:.9e}, "
                  f"{time.perf_counter() - t0:.1f} s", flush=True)
        if st != L.LBM_ENOTCONV:
            break
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
        fine_check=1000, coarse_tol=1e-7, verbose=False, coarse_check=100,
        coarse_max_steps=4_000_000, margins=(0,)) -> UpscaleResult:
    import torch
    kd = torch.as_tensor(np.ascontiguousarray(kappa)).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    keff, ok = local_tensor(kd, r, tau, eps, nu, g)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    u_c, c_steps, _ = coarse_solve(kappa.shape, keff, r, tau, eps, nu, g, L.LBM_KEFF_TENSOR,
                                   coarse_tol, coarse_max_steps, check_every=coarse_check)
    t2 = time.perf_counter()
    u_cs, _, _ = coarse_solve(kappa.shape, keff, r, tau, eps, nu, g, L.LBM_KEFF_SCALAR, coarse_tol,
                              coarse_max_steps, check_every=coarse_check)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    # the method without local problems: each coarse cell takes the geometric
    # mean of kappa over its block
    ny, nx = kappa.shape
    gm = np.exp(np.log(kappa).reshape(ny // r, r, nx // r, r).mean(axis=(1, 3)))
    kg = np.stack([gm, 0 * gm, 0 * gm, gm], axis=-1)
    u_cg, _, _ = coarse_solve(kappa.shape, kg, r, tau, eps, nu, g, L.LBM_KEFF_SCALAR, coarse_tol,
                              coarse_max_steps, check_every=coarse_check)
    over = {}
    for m in margins:
        if m == 0:
            continue
        torch.cuda.synchronize()
        ta = time.perf_counter()
        km, okm = local_tensor(kd, r, tau, eps, nu, g, margin=m)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        ut, _, _ = coarse_solve(kappa.shape, km, r, tau, eps, nu, g, L.LBM_KEFF_TENSOR, coarse_tol,
                                coarse_max_steps, check_every=coarse_check)
        us, _, _ = coarse_solve(kappa.shape, km, r, tau, eps, nu, g, L.LBM_KEFF_SCALAR, coarse_tol,
                                coarse_max_steps, check_every=coarse_check)
        over[m] = (ut, us, tb - ta, okm)
    if verbose:
        print(f"local problems {t1 - t0:.2f} s, coarse solves {t3 - t1:.2f} s", flush=True)
    u_f, f_steps, f_st, solver = fine_solve(kappa, tau, eps, nu, g, fine_tol, fine_max_steps,
                                            fine_check,
                                            chunk=fine_check * max(1, 20000 // fine_check)
                                            if verbose else None, verbose=verbose)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    u_avg = block_average(u_f, r)
    solver.close()
    mc, mf = u_c.mean(axis=(1, 2)), u_avg.mean(axis=(1, 2))
    by_margin = {0: dict(rel_l2_tensor=_rel_l2(u_c, u_avg), rel_l2_scalar=_rel_l2(u_cs, u_avg),
                         t_local_s=t1 - t0, local_flags_ok=ok)}
    for m, (ut, us, tl, okm) in over.items():
        by_margin[m] = dict(rel_l2_tensor=_rel_l2(ut, u_avg), rel_l2_scalar=_rel_l2(us, u_avg),
                            t_local_s=tl, local_flags_ok=okm)
    return UpscaleResult(keff, u_c, u_avg, _rel_l2(u_c, u_avg), _rel_l2(u_cs, u_avg),
                         _rel_l2(u_cg, u_avg), by_margin,
                         float(np.linalg.norm(mc - mf) / np.linalg.norm(mf)),
                         t1 - t0, t2 - t1, t4 - t3, f_steps, f_st, c_steps, ok)


def main():
    import argparse
    import json
    from . import inputs as I
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--r", type=int, default=64)
    ap.add_argument("--channels", action="store_true")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--tol", type=float, default=1e-6,
                    help="relative change allowed per check on both grids")
    ap.add_argument("--coarse-check", type=int, default=100,
                    help="coarse steps between checks; the fine grid checks every r times "
                         "as many steps, the same physical time")
    ap.add_argument("--fine-max-steps", type=int, default=2_000_000)
    ap.add_argument("--margins", default="0",
                    help="comma-separated oversampling margins m (r + 2m <= 64)")
    args = ap.parse_args()
    margins = tuple(int(v) for v in args.margins.split(","))
    L.lib()
    w = I.workload_upscale(seed=args.seed, n=args.n, channels=args.channels)
    res = run(w["kappa"], args.r, fine_tol=args.tol, fine_check=args.coarse_check * args.r,
              fine_max_steps=args.fine_max_steps, coarse_tol=args.tol,
              coarse_check=args.coarse_check, verbose=True, margins=margins)
    print(json.dumps(dict(
        n=args.n, r=args.r, channels=args.channels, seed=args.seed,
        rel_l2_tensor=res.rel_l2, rel_l2_scalar=res.rel_l2_scalar,
        rel_l2_geometric_mean_blocks=res.rel_l2_geomean, mean_velocity_rel_err=res.mean_err,
        t_local_s=res.t_local, t_coarse_s=res.t_coarse, t_fine_s=res.t_fine,
        speedup_upscaled_vs_fine=res.t_fine / (res.t_local + res.t_coarse),
        fine_steps=res.fine_steps, fine_status=res.fine_status, coarse_steps=res.coarse_steps,
        tol=args.tol, coarse_check=args.coarse_check, fine_check=args.coarse_check * args.r,
        local_flags_ok=res.local_flags_ok,
        oversampling={str(m): v for m, v in res.by_margin.items()},
        max_abs_kxy_over_kxx=float(np.max(np.abs(res.keff[..., 1]) / res.keff[..., 0])))),
        flush=True)


if __name__ == "__main__":
    main()
