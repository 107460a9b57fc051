"""The two-grid experiments of Sec. 4.3 on the GPU.

Setting shared by Sec. 4.3.1 and 4.3.2: a 1 m x 1 m periodic domain, eps 0.8,
nu 2e-6 m^2/s, body force G = (sin pi x, sin pi y) m/s^2, the permeability of
Eq. finekappa-fiveblock on a 400 x 400 fine grid (dx 0.0025 m, dt 2.5e-5 s)
split into 40 x 40 subdomains of 10 x 10 points, and a 40 x 40 coarse grid
(dx and dt ten times larger).

* Sec. 4.3.1 (Darcy): k_const 1e-13 m^2, nu_eff = 0 (tau 1/2 on both grids
  and in the local problems).
* Sec. 4.3.2 (Brinkman): k_const 1e-7 m^2, nu_eff 1e-5 m^2/s (tau 0.50012 on
  the fine grid and in the local problems, 0.500012 on the coarse grid); the
  ablation runs the local problems with nu_eff = 0 instead (kappa*,err).

Pipeline, every step in the HIP library:
 1. lbm_local_keff on the 1600 subdomains, both drives -> K* per subdomain;
 2. lbm_coarse_solve with the scalar kappa* = (kxx + kyy) / 2 per coarse
    point (the paper's choice for these fields) and with the full tensor;
 3. the fine solve to steady state with the per-cell force (FP64
    populations: the drag is strong enough in the Darcy case that density
    deviations exceed the velocity by about 1e4);
 4. 10 x 10 block averages of the fine u, v and p, compared with the coarse
    fields (relative L2 over the coarse grid).
The paper shows these comparisons as figures only; the numbers reported here
(K* of each kind of subdomain, errors of each coarse run) are ours.

    python -m paper_1312_0195_amd.two_grid --case darcy|brinkman [--out FILE]
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import inputs as I
from . import lbm as L

DX_F, DT_F = 0.0025, 2.5e-5
R = 10
EPS, NU_PHYS = 0.8, 2e-6
CASES = {
    "darcy": dict(k_const=1e-13, nu_eff=0.0),
    "brinkman": dict(k_const=1e-7, nu_eff=1e-5),
}


def setting(case: str, n: int = 400):
    """Lattice-unit inputs of one case: kappa [n, n], force [n, n, 2] (fine
    lattice units), tau_f, nu_f, and the unit conversion."""
    c = CASES[case]
    U = I.LatticeUnits(DX_F, DT_F)
    kappa = U.kappa(I.five_block_field(n, DX_F, c["k_const"]))
    x = I.cell_coords(n, DX_F, 0.5)
    X, Y = np.meshgrid(x, x, indexing="xy")
    force = np.stack([U.force(np.sin(np.pi * X)), U.force(np.sin(np.pi * Y))], axis=-1)
    return dict(kappa=kappa, force=np.ascontiguousarray(force), tau=U.tau(c["nu_eff"]),
                nu=U.nu(NU_PHYS), units=U, k_const_lat=float(U.kappa(c["k_const"])))


def local_keff(kappa_dev, tau, nu, tol=1e-10, max_steps=8_000_000):
    """K* tensor of every R x R subdomain (fine lattice units) [nc, nc, 4].
    FP64 state: with tau near 1/2 and weak drag (the Brinkman case) a step
    changes the state by less than half an FP32 ulp long before the fixed
    point, and an FP32 state stalls short of it."""
    n = kappa_dev.shape[0]
    x0, y0, side = I.tile_patches(n, n, R)
    res = L.local_keff(None, x0, y0, side, tau, EPS, nu, 1e-6, tol=tol, check_every=200,
                       max_steps=max_steps, kappa_dev=kappa_dev, pop_dtype=L.LBM_F64)
    nc = n // R
    return res.keff.reshape(nc, nc, 4), res.flags.reshape(nc, nc, 2), res.steps.reshape(nc, nc, 2)


def coarse(n, tau_f, nu_f, keff, force_c, mode, tol=1e-11, max_steps=40_000_000):
    """Coarse solve; force_c is G per coarse point in fine lattice units."""
    import torch
    fine = L.make_params(n, n, tau_f, EPS, nu_f, 1.0, 0.0, 0.0, 0, L.LBM_F64)
    nc = n // R
    kd = torch.as_tensor(np.ascontiguousarray(keff)).cuda()
    fd = torch.as_tensor(np.ascontiguousarray(force_c)).cuda()
    u = torch.empty((2, nc, nc), dtype=torch.float64, device="cuda")
    rho = torch.empty((nc, nc), dtype=torch.float64, device="cuda")
    nb = L.lbm_coarse_workspace_bytes(nc, nc)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    st, steps = L.lbm_coarse_solve(fine, R, kd, mode, fd, max_steps, tol, 1000, u, rho, ws, nb)
    return u.cpu().numpy(), rho.cpu().numpy(), int(steps), int(st)


def fine(kappa, force, tau, nu, tol=1e-12, max_steps=40_000_000, check_every=20_000,
         chunk=1_000_000, verbose=True):
    """Fine steady state: u [2, n, n] and rho [n, n] on the device. Runs in
    chunks of whole check intervals (the solver keeps the last check across
    calls) and prints progress after each."""
    import torch
    n = kappa.shape[0]
    p = L.make_params(n, n, tau, EPS, nu, 1.0, 0.0, 0.0, 0, L.LBM_F64)
    s = L.FineSolver(p, kappa, force)
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
    u, rho = s.fields()
    torch.cuda.synchronize()
    s.close()
    return u, rho, int(steps), int(st)


def _block(dev, r=R):
    import torch
    planes = dev.shape[0] if dev.dim() == 3 else 1
    d = dev.reshape(planes, dev.shape[-2], dev.shape[-1]).contiguous()
    out = torch.empty((planes, d.shape[1] // r, d.shape[2] // r), dtype=torch.float64,
                      device=d.device)
    L.lbm_block_average(d, d.shape[2], d.shape[1], planes, r, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def rel_l2(a, b):
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))


def run(case: str, n: int = 400, fine_max_steps=40_000_000, fine_tol=1e-12,
        coarse_tol=1e-11) -> dict:
    import torch
    L.lib()
    S = setting(case, n)
    kd = torch.as_tensor(S["kappa"]).cuda()
    out = dict(case=case, n_fine=n, n_coarse=n // R, tau_fine=S["tau"],
               tau_coarse=0.5 + (S["tau"] - 0.5) / R, nu_fine=S["nu"])
    # 1. local problems (and, for the Brinkman case, the nu_eff = 0 ablation)
    t0 = time.perf_counter()
    keff, flags, steps = local_keff(kd, S["tau"], S["nu"])
    out["t_local_s"] = time.perf_counter() - t0
    print(f"local problems: {out['t_local_s']:.2f} s", flush=True)
    kinds = {}
    const = np.isclose(S["kappa"].reshape(n // R, R, n // R, R).std(axis=(1, 3)), 0.0)
    for name, mask in (("constant", const), ("sinusoid", ~const)):
        k = keff[mask] / S["k_const_lat"]
        kinds[name] = dict(count=int(mask.sum()), kxx=float(np.median(k[:, 0])),
                           kyy=float(np.median(k[:, 3])),
                           scalar=float(np.median(0.5 * (k[:, 0] + k[:, 3]))),
                           max_abs_offdiag=float(np.abs(k[:, [1, 2]]).max()),
                           spread_scalar=float(np.ptp(0.5 * (k[:, 0] + k[:, 3]))))
    out["keff_over_k_const"] = kinds
    out["local_flags_ok"] = bool((flags == 0).all())
    out["local_max_steps"] = int(steps.max())
    variants = {"kappa_star": keff}
    if S["tau"] > 0.5:
        keff_err, flags_err, _ = local_keff(kd, 0.5, S["nu"])
        k = keff_err[~const] / S["k_const_lat"]
        out["keff_err_over_k_const_sinusoid"] = float(np.median(0.5 * (k[:, 0] + k[:, 3])))
        out["local_err_flags_ok"] = bool((flags_err == 0).all())
        variants["kappa_star_err"] = keff_err
    # 3. fine grid
    t0 = time.perf_counter()
    u_f, rho_f, f_steps, f_st = fine(S["kappa"], S["force"], S["tau"], S["nu"], fine_tol,
                                     fine_max_steps)
    out["t_fine_s"] = time.perf_counter() - t0
    out["fine_steps"], out["fine_status"] = f_steps, f_st
    uf = _block(u_f)
    pf = _block(rho_f)[0] / 3.0
    # 2. coarse runs (G at the coarse points), compared with the block-averaged
    # fine fields
    xc = I.cell_coords(n // R, DX_F * R, 0.5)
    Xc, Yc = np.meshgrid(xc, xc, indexing="xy")
    U = S["units"]
    fc = np.stack([U.force(np.sin(np.pi * Xc)), U.force(np.sin(np.pi * Yc))], axis=-1)
    runs = {}
    for vname, kv in variants.items():
        for mname, mode in (("scalar", L.LBM_KEFF_SCALAR), ("tensor", L.LBM_KEFF_TENSOR)):
            t0 = time.perf_counter()
            uc, rc, c_steps, c_st = coarse(n, S["tau"], S["nu"], kv, fc, mode, coarse_tol)
            dt = time.perf_counter() - t0
            pc = rc / 3.0
            runs[f"{vname}_{mname}"] = dict(
                rel_l2_u=rel_l2(uc[0], uf[0]), rel_l2_v=rel_l2(uc[1], uf[1]),
                rel_l2_p=rel_l2(pc - pc.mean(), pf - pf.mean()), steps=c_steps, status=c_st,
                seconds=dt)
    out["coarse_vs_fine_avg"] = runs
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--case", choices=sorted(CASES), default="brinkman")
    ap.add_argument("--n", type=int, default=400)
    ap.add_argument("--fine-max-steps", type=int, default=40_000_000)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    res = run(args.case, args.n, args.fine_max_steps)
    print(json.dumps(res), flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(res, fh, indent=1)


if __name__ == "__main__":
    main()
