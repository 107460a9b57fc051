"""Benchmark of the upscaled Brinkman LBM hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload (the fine-grid configuration the throughput metric is quoted on):
D2Q9 BGK Brinkman LBM with the Shan-Chen velocity-shift force on a 2048 x 2048
grid, log-normal permeability K = exp(Z) (Z a seeded periodic Gaussian random
field, sigma 1.5, correlation length 32 cells), porosity 0.4, tau 0.8,
nu = nu_eff = 0.1, g = 1e-6 along x, bounce-back walls in y, FP32 deviation
populations. Steps run six per launch (temporal blocking through LDS); the
volume-averaged velocity (FP64 reduction) is taken every 100 steps inside the
timed region.

Printed: one JSON line with MLUPS (value), the HBM roofline of the step kernel
measured live with HIP events, the batched local K_eff throughput (patches/s)
on the 4096 32 x 32 tiles of the same field plus 4096 mixed-size patches, the
learned K_eff path (network + LBM fallback vs LBM alone, with its error), the
same step on the D3Q19 lattice (256^3) against the HBM roofline and a plain
device copy, and the CPU oracle timed on a bounded sample of the same
workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS (D2Q9 Brinkman, % HBM roofline); K_eff patches/s surrogate vs LBM @2%"
HBM_PEAK_GBS = 8000.0
VALU_ISSUE_PER_S = 256 * 4 * 2.4e9 / 4  # wave64 VALU instructions per second (one per 4 cycles per SIMD)
BYTES_PER_LU = 76  # per cell and launch: 9 x 4 B read + 9 x 4 B written + 4 B drag coefficient
# operations of one collision (FMA = 2), counted on the FP64 formulation; the
# FP32 one issues a few more (its exactly summing weights), not counted
FLOPS_PER_LU = 65
# the local solver's collision in FP32: the same 65 operations (FMA = 2)
FP32_FLOPS_PER_LU_LOCAL = 65
FP32_PEAK_TFLOPS = 157.3      # MI355X FP32 vector (published; counts packed FP32 issue)
FP32_UNPACKED_TFLOPS = 78.6   # 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz x 2: packed FP32 is not used
DEPTH = 7          # time steps per launch of the fine-step kernel (FP32 state, FP32 arithmetic)
# The fine step as benchmarked: FP32 state and FP32 collision arithmetic
# (LBM_F32_FAST), within 2.6e-6 of the FP64-state solver in relative L2 of
# the velocity after the workload's 20 000 steps (the target is 1e-5);
# LBM_F32_SHIFTED (FP64 arithmetic, 2.0e-7) is the high-accuracy mode.
FINE_DTYPE_NAME = "LBM_F32_FAST"
STEP_KERNEL_SRC = os.path.join(ROOT, "paper_1312_0195_amd", "csrc", "lbm_fine.hip")
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "fine_step_2048_hbm_counters.md")
VALU_SUMMARY = os.path.join(ROOT, "profiles", "fine_step_2048_valu_counters.md")
LOCAL_KERNEL_SRC = os.path.join(ROOT, "paper_1312_0195_amd", "csrc", "lbm_local.hip")
LOCAL_VALU_SUMMARY = os.path.join(ROOT, "profiles", "local_keff_valu_counters.md")
# one forward pass of the surrogate network per patch and symmetry: four 3x3
# convolutions on 32 x 32 (1 -> 32, then 32 -> 32 channels) and the head MLP
CNN_FLOPS_PER_PATCH = 2 * 1024 * 9 * (32 + 3 * 32 * 32) + 2 * (32 * 37 + 2 * 32)
BF16_MFMA_PEAK_TFLOPS = 2500.0


def _src_hash(path):
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def _summary_value(path, pattern, src=STEP_KERNEL_SRC):
    """A number from a committed counter summary, or None when the summary is
    missing or was taken on a different kernel source."""
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_src = re.search(r"kernel source sha256\[:16\]:\s*([0-9a-f]{16})", txt)
    m_b = re.search(pattern, txt)
    if not m_src or not m_b or m_src.group(1) != _src_hash(src):
        return None
    return float(m_b.group(1))


def _traffic_per_launch():
    """HBM bytes per step-kernel launch (scaled FETCH_SIZE + WRITE_SIZE)."""
    return _summary_value(TRAFFIC_SUMMARY, r"HBM bytes per launch \(scaled\):\s*([0-9.eE+]+)")


def _valu_per_launch():
    """Wave64 VALU instructions per step-kernel launch (SQ_INSTS_VALU)."""
    return _summary_value(VALU_SUMMARY, r"SQ_INSTS_VALU per launch:\s*([0-9.eE+]+)")


KERNEL_WARMUP_LAUNCHES = 900  # ~0.1 s of back-to-back step launches before the kernel-alone timing
KERNEL_LAUNCHES = 360         # launches timed for the kernel-alone roofline (fixed, whatever --steps)


def bench_fine(L, torch, kappa, steps, warmup, check_every=100, repeats=5):
    n = kappa.shape[0]
    p = L.make_params(n, n, 0.8, 0.4, 0.1, 1.0, 1e-6, 0.0, 1, getattr(L, FINE_DTYPE_NAME))
    stream = torch.cuda.current_stream()
    # step kernel alone, first (so the device is also warm for the timed
    # region): a fixed number of back-to-back launches of the multi-step
    # kernel (no reductions, same stream) after a fixed warm-up, independent
    # of --steps / --warmup, on a solver of its own
    s = L.FineSolver(p, kappa)
    s.step(KERNEL_WARMUP_LAUNCHES * DEPTH, 0.0, 0)
    e2, e3 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e2.record(stream)
    s.step(KERNEL_LAUNCHES * DEPTH, 0.0, 0)
    e3.record(stream)
    torch.cuda.synchronize()
    step_ms = e2.elapsed_time(e3) / KERNEL_LAUNCHES  # per launch (DEPTH time steps)
    s.close()
    # the workload from rest: W warm-up steps, then the timed K steps with the
    # FP64 mean-velocity reduction every 100 steps (no extra reduction at the
    # end of the window: the mean velocity is read after it, for the check)
    s = L.FineSolver(p, kappa)
    s.step(warmup, 0.0, check_every)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    st, done, _ = s.step(steps, 0.0, check_every, mean=False)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    _, _, mu = s.step(0, 0.0, check_every)
    assert st == L.LBM_OK and done == steps and np.isfinite(mu).all()
    # the same K steps again, for the spread over runs (median of `repeats`)
    runs = [ev_ms]
    for _ in range(repeats - 1):
        e0.record(stream)
        s.step(steps, 0.0, check_every, mean=False)
        e1.record(stream)
        torch.cuda.synchronize()
        runs.append(e0.elapsed_time(e1))
    s.close()
    return dict(wall_s=wall, event_ms=ev_ms, run_ms=runs, step_kernel_ms=step_ms,
                mean_u=mu.tolist())


def bench_forms(L, torch, kappa, steps=2000):
    """Time per step of the two forms of the step on the same workload (Sec.
    2.1 Guo form vs Sec. 2.2 Shan-Chen form; the paper reports 23 vs 21 min
    on its CPU code): back-to-back two-step launches, no reductions."""
    n = kappa.shape[0]
    out = {}
    stream = torch.cuda.current_stream()
    for name, scheme in (("shan_chen", L.LBM_SCHEME_SHAN_CHEN), ("guo", L.LBM_SCHEME_GUO)):
        p = L.make_params(n, n, 0.8, 0.4, 0.1, 1.0, 1e-6, 0.0, 1, L.LBM_F32_SHIFTED,
                          L.LBM_PERM_SCALAR, scheme)
        s = L.FineSolver(p, kappa)
        s.step(200, 0.0, 0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        s.step(steps, 0.0, 0)
        e1.record(stream)
        torch.cuda.synchronize()
        out[name + "_us_per_step"] = round(e0.elapsed_time(e1) * 1e3 / steps, 3)
        s.close()
    out["guo_over_shan_chen"] = round(out["guo_us_per_step"] / out["shan_chen_us_per_step"], 4)
    return out


def bench_paper_sec41(L, torch):
    """The paper's only timing (Sec. 4.1): 100 x 100 periodic, tau 0.53, the
    block field of Eq. kappa-forcemodel, 200 000 steps, Guo form about 23 min
    and Shan-Chen form about 21 min on the paper's (unstated) CPU. Here: both
    forms with FP64 populations (the paper's precision is not stated; its
    7-digit K_eff values imply FP64) and the Shan-Chen form with FP32
    deviations, each the full 200 000 steps on one MI355X."""
    from paper_1312_0195_amd import inputs as I
    w = I.workload_sec41()
    stream = torch.cuda.current_stream()
    out = {"workload": "Sec. 4.1: 100x100 periodic, tau 0.53, eps 0.8, block field, 200000 steps",
           "paper_minutes": {"shan_chen": 21, "guo": 23, "hardware": "not stated (CPU)"}}
    for name, scheme, dtype in (("shan_chen_f64", L.LBM_SCHEME_SHAN_CHEN, L.LBM_F64),
                                ("guo_f64", L.LBM_SCHEME_GUO, L.LBM_F64),
                                ("shan_chen_f32", L.LBM_SCHEME_SHAN_CHEN, L.LBM_F32_SHIFTED)):
        p = L.make_params(w["nx"], w["ny"], w["tau"], w["eps"], w["nu"], 1.0, w["g"][0], w["g"][1],
                          0, dtype, L.LBM_PERM_SCALAR, scheme)
        s = L.FineSolver(p, w["kappa"])
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        st, done, _ = s.step(w["steps"], 0.0, 0)
        e1.record(stream)
        torch.cuda.synchronize()
        assert st == L.LBM_OK and done == w["steps"]
        sec = e0.elapsed_time(e1) * 1e-3
        out[name + "_seconds"] = round(sec, 3)
        s.close()
    return out


def bench_local(L, torch, kappa_dev, reps=5, sets=None):
    """Batched local problems (Sec. 3, Eq. tensor-kappa) on the fine field's
    4096 tiles of 32 x 32 and on 4096 patches of mixed sides: `reps` calls
    each, median and best wall time around the whole call (inputs resident)."""
    from paper_1312_0195_amd import inputs as I
    n = kappa_dev.shape[0]
    out = {}
    if sets is None:
        sets = {"tiles32": I.tile_patches(n, n, 32), "mixed": I.mixed_patches(4096, n, n, seed=1)}
    keff_tiles = None
    for name, (x0, y0, side) in sets.items():
        times = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = L.local_keff(None, x0, y0, side, 0.8, 0.4, 0.1, 1e-6, tol=1e-7, check_every=100,
                             max_steps=400000, kappa_dev=kappa_dev)
            times.append(time.perf_counter() - t0)
        med, best = float(np.median(times)), min(times)
        lu = float(np.sum(r.steps.astype(np.float64) * (side.astype(np.float64) ** 2)[:, None]))
        flops = FP32_FLOPS_PER_LU_LOCAL * lu / med / 1e12
        out[name] = dict(patches=int(len(x0)), seconds_median=round(med, 5),
                         seconds_best=round(best, 5), runs=len(times),
                         patches_per_s=len(x0) / med, patches_per_s_best=len(x0) / best,
                         lattice_updates=lu, mlups=lu / med / 1e6,
                         # what a step streamed through HBM would need for the same
                         # updates (76 B each): an on-chip design passes 8 TB/s
                         hbm_equivalent_gbs=round(lu / med * BYTES_PER_LU / 1e9, 1),
                         converged=int((r.flags == 0).sum()), items=int(r.flags.size),
                         mean_steps=float(r.steps.mean()),
                         # the collisions' FP32 arithmetic against the vector FP32 peak
                         roofline={"bound": "alu", "achieved": round(flops, 2),
                                   "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                                   "frac": round(flops / FP32_PEAK_TFLOPS, 4),
                                   "frac_of_unpacked_fp32": round(flops / FP32_UNPACKED_TFLOPS, 4),
                                   "flops_per_lu": FP32_FLOPS_PER_LU_LOCAL})
        # VALU issue: the kernel's measured VALU lane instructions per lattice
        # update (committed counter summary) at the achieved update rate
        ipl = _summary_value(LOCAL_VALU_SUMMARY,
                             name + r" VALU lane instructions per lattice update:\s*([0-9.]+)",
                             LOCAL_KERNEL_SRC)
        if ipl is not None:
            out[name]["roofline"].update(
                valu_lane_instructions_per_lu=ipl,
                valu_issue_frac=round(lu / med * ipl / 64 / VALU_ISSUE_PER_S, 4))
        if name == "tiles32":
            keff_tiles = r.keff.reshape(n // 32, n // 32, 4)
    return out, keff_tiles


def cpu_baseline_local(kappa, sample_every_tile=16, sample_every_mixed=32, single=8):
    """The oracle's local problems (Sec. 3, Eq. tensor-kappa: both drives to
    a relative change of 1e-7 per 100 steps, as the GPU runs them) on a
    bounded sample of the same two sets: every `sample_every_tile`-th tile and
    every `sample_every_mixed`-th mixed patch, items spread over host threads
    (one oracle call per thread at a time, each single-threaded), plus the
    first `single` tiles on one thread."""
    import concurrent.futures as cf
    from oracle import oracle as O
    from paper_1312_0195_amd import inputs as I
    n = kappa.shape[0]
    sets = {"tiles32": I.tile_patches(n, n, 32), "mixed": I.mixed_patches(4096, n, n, seed=1)}
    threads = min(os.cpu_count() or 1, 16)

    def solve(args):
        O.set_threads(1)
        x0, y0, sd = args
        return O.local_keff(I.cut_patch(kappa, x0, y0, sd), 0.8, 0.4, 0.1, 1e-6,
                            check_every=100, tol=1e-7, max_steps=400000)

    out = {"cores": threads, "kind": "oracle", "cpu_model": _cpu_model()}
    O.lib()
    for name, (x0, y0, side) in sets.items():
        every = sample_every_tile if name == "tiles32" else sample_every_mixed
        idx = np.arange(0, len(x0), every)
        work = [(int(x0[i]), int(y0[i]), int(side[i])) for i in idx]
        t0 = time.perf_counter()
        with cf.ThreadPoolExecutor(threads) as ex:
            res = list(ex.map(solve, work))
        dt = time.perf_counter() - t0
        lu = sum(float(r.steps.sum()) * w[2] ** 2 for r, w in zip(res, work))
        out[name] = dict(value=round(len(work) / dt, 2), unit="patches/s",
                         sample=f"{len(work)} of {len(x0)} patches (every {every}-th), {dt:.1f} s",
                         mlups=round(lu / dt / 1e6, 1))
    x0, y0, side = sets["tiles32"]
    main_threads = O.num_threads()
    t0 = time.perf_counter()
    res = [solve((int(x0[i]), int(y0[i]), int(side[i]))) for i in range(single)]
    dt = time.perf_counter() - t0
    O.set_threads(main_threads)  # solve() set this thread's OpenMP team to one
    out["tiles32_single_thread"] = dict(value=round(single / dt, 2), unit="patches/s",
                                        sample=f"the first {single} tiles, one thread, {dt:.1f} s")
    return out


def bench_coarse(L, torch, keff, r=32, reps=3):
    """Time to steady state of the coarse grid built from the local K_eff of
    the fine field's 32 x 32 tiles (64 x 64 coarse cells, tensor drag; Sec. 3
    mapping of tau, nu, kappa and G): one persistent on-chip solve."""
    ncy, ncx = keff.shape[:2]
    fine = L.make_params(ncx * r, ncy * r, 0.8, 0.4, 0.1, 1.0, 1e-6, 0.0, 0)
    kd = torch.as_tensor(np.ascontiguousarray(keff)).cuda()
    u = torch.empty((2, ncy, ncx), dtype=torch.float64, device="cuda")
    nb = L.lbm_coarse_workspace_bytes(ncx, ncy)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    best, steps = None, 0
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, steps = L.lbm_coarse_solve(fine, r, kd, L.LBM_KEFF_TENSOR, None, 4_000_000, 1e-6, 100,
                                       u, None, ws, nb)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        assert st == L.LBM_OK
        best = dt if best is None else min(best, dt)
    return dict(grid=f"{ncx}x{ncy} coarse cells (r {r}), tensor K_eff, rel. change 1e-6 per 100 steps",
                steps=int(steps), seconds_to_steady_state=round(best, 5),
                mlups=round(ncx * ncy * steps / best / 1e6, 1))


def cpu_baseline_surrogate(big, x0, y0, every=512):
    """The oracle's local problems on a bounded sample of the surrogate's test
    patches (every `every`-th 32 x 32 patch, both drives, the labels'
    tolerance of 1e-7 per 100 steps), items spread over host threads as in
    cpu_baseline_local: the LBM-only rate the surrogate path replaces."""
    import concurrent.futures as cf
    from oracle import oracle as O
    from paper_1312_0195_amd import inputs as I
    from paper_1312_0195_amd import surrogate as S
    threads = min(os.cpu_count() or 1, 16)
    ph = S.PHYS

    def solve(args):
        O.set_threads(1)
        a, b = args
        return O.local_keff(I.cut_patch(big, a, b, S.SIDE), ph["tau"], ph["eps"], ph["nu"], ph["g"],
                            check_every=100, tol=1e-7, max_steps=400000)

    O.lib()
    main_threads = O.num_threads()
    idx = np.arange(0, len(x0), every)
    work = [(int(x0[i]), int(y0[i])) for i in idx]
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(threads) as ex:
        res = list(ex.map(solve, work))
    dt = time.perf_counter() - t0
    O.set_threads(main_threads)
    lu = sum(float(r.steps.sum()) * S.SIDE ** 2 for r in res)
    return dict(value=round(len(work) / dt, 2), unit="patches/s", cores=threads, kind="oracle",
                cpu_model=_cpu_model(),
                sample=f"{len(work)} of {len(x0)} test patches (every {every}-th), {dt:.1f} s",
                mlups=round(lu / dt / 1e6, 1))


def bench_surrogate(n_test=65536, cpu=False):
    """The learned K_eff path on a test set of 32 x 32 patches (about 90% from
    the training distribution, 10% outside it): network, network + batched
    LBM fallback for flagged patches, and batched LBM alone; K_eff error of
    the network against the LBM; with cpu, the oracle on a sample beside it."""
    from paper_1312_0195_amd import surrogate as S
    from paper_1312_0195_amd import train_surrogate as T
    if not os.path.exists(T.DEFAULT_MODEL):
        return None
    model = S.Surrogate.load(T.DEFAULT_MODEL)
    big, x0, y0, is_oor = T.test_set(n_test)
    r = T.evaluate(model, big, x0, y0, is_oor)
    e = r["keff_error_network_in_range"]
    net_tflops = r["patches_per_s_network"] * r["n_sym"] * CNN_FLOPS_PER_PATCH / 1e12
    return dict(patches=r["n_patches"], flagged_to_lbm=r["flagged"],
                network_roofline={"bound": "mfma", "achieved": round(net_tflops, 1),
                                  "peak": BF16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                                  "frac": round(net_tflops / BF16_MFMA_PEAK_TFLOPS, 4),
                                  "flops_per_patch_and_symmetry": CNN_FLOPS_PER_PATCH},
                patches_per_s_network=r["patches_per_s_network"],
                patches_per_s_network_plus_fallback=r["patches_per_s_network_plus_fallback"],
                patches_per_s_lbm_only=r["patches_per_s_lbm_only"],
                speedup_vs_lbm=r["patches_per_s_network_plus_fallback"] / r["patches_per_s_lbm_only"],
                n_sym=r["n_sym"],
                keff_rel_error_in_range_p50=e["p50"], keff_rel_error_in_range_p95=e["p95"],
                by_n_sym={k: dict(p50=v["p50"], p95=v["p95"], patches_per_s_network=v["patches_per_s"])
                          for k, v in r["keff_error_in_range_by_n_sym"].items()},
                keff_rel_error_all_with_fallback=r["keff_error_combined_all"],
                keff_rel_error_geometric_mean_p50=r["keff_error_geometric_mean_in_range"]["p50"],
                **({"cpu_baseline": cpu_baseline_surrogate(big, x0, y0)} if cpu else {}))


D3Q19_BYTES_PER_LU = 156  # 19 x 4 B read + 19 x 4 B written + 4 B drag coefficient


def bench_d3q19(L, torch, n=256, steps=200, warmup=20):
    """The step on the D3Q19 lattice: n^3 log-normal field (sigma 1.5), walls
    in z, FP32 deviation populations, two steps per launch; the kernel time
    from HIP events over back-to-back launches, and a plain device copy of
    the same byte count (one pass of the state) as the HBM reference."""
    from paper_1312_0195_amd import inputs as I
    w = I.workload_d3q19(n=n)
    p = L.make_params3(n, n, n, w["tau"], w["eps"], w["nu"], 1.0, w["g"], w["walls_z"],
                       L.LBM_F32_SHIFTED)
    s = L.Solver3D(p, w["kappa"])
    stream = torch.cuda.current_stream()
    s.step(warmup, 0.0, 0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    s.step(steps, 0.0, 0)
    e1.record(stream)
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / steps
    st, _, mu = s.step(2, 0.0, 1)
    assert st == L.LBM_OK and np.isfinite(mu).all()
    s.close()
    cells = n ** 3
    launch_us = 2 * us                       # two time steps per launch
    gbs = D3Q19_BYTES_PER_LU * cells / (launch_us * 1e-6) / 1e9
    # plain copy moving the same bytes (half read, half written)
    src = torch.empty(D3Q19_BYTES_PER_LU * cells // 8, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0.record(stream)
    for _ in range(10):
        dst.copy_(src)
    e1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2 * src.numel() * 4 * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    return dict(workload=f"{n}^3 D3Q19 Brinkman LBM, log-normal K (sigma 1.5, corr {16 * n // 256}), "
                         f"tau 0.8, g 1e-6 along x, walls in z, FP32 deviation populations",
                us_per_step=round(us, 2), mlups=round(cells / us, 1),
                roofline={"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                          "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                          "kernel": "k3_step2<walls> (2 time steps per launch)",
                          "avg_launch_us": round(launch_us, 2),
                          "hbm_bytes_per_launch_algorithmic": D3Q19_BYTES_PER_LU * cells,
                          "single_step_hbm_equivalent_gbs":
                              round(D3Q19_BYTES_PER_LU * cells / (us * 1e-6) / 1e9, 1)},
                device_copy_gbs=round(copy_gbs, 1),
                single_step_equivalent_over_device_copy=round(
                    D3Q19_BYTES_PER_LU * cells / (us * 1e-6) / 1e9 / copy_gbs, 4))


def bench_upscale_reduced(L, torch, n=512, r=64):
    """The upscaling workload (log-normal K, sigma 2, correlation length
    64 n / 4096, fully periodic) at the reduced size n = 512 with r = 64:
    local problems, coarse solve (tensor K_eff) and the fine grid to steady
    state (relative change 1e-6 per check, the coarse check every 100 steps
    and the fine one every 100 r: the same physical time), with the oracle
    timed beside it."""
    from paper_1312_0195_amd import inputs as I
    from paper_1312_0195_amd import upscale as U
    kappa = I.workload_upscale(seed=1, n=n)["kappa"]
    res = U.run(kappa, r, fine_tol=1e-6, fine_check=100 * r, coarse_tol=1e-6, coarse_check=100)
    out = dict(workload=f"{n}x{n}, sigma 2, corr {64 * n // 4096}, periodic, r {r}",
               rel_l2_tensor=round(res.rel_l2, 5), rel_l2_scalar=round(res.rel_l2_scalar, 5),
               t_local_s=round(res.t_local, 5), t_coarse_s=round(res.t_coarse, 5),
               t_fine_s=round(res.t_fine, 4), fine_steps=int(res.fine_steps),
               coarse_steps=int(res.coarse_steps),
               speedup_upscaled_vs_fine=round(res.t_fine / (res.t_local + res.t_coarse), 2))
    return out, kappa, res


def cpu_baseline_upscale(kappa, res, r=64, fine_sample_steps=200):
    """The oracle on the reduced upscaling workload: all local problems (items
    over host threads, each single-threaded; Sec. 3, Eq. tensor-kappa), the
    coarse solve with the tensor drag on the coarse lattice (Sec. 3 mapping),
    and the fine step timed on a bounded sample of steps, its time to the
    GPU run's steady-state step count projected from that rate."""
    import concurrent.futures as cf
    from oracle import oracle as O
    from paper_1312_0195_amd import inputs as I
    n = kappa.shape[0]
    nc = n // r
    threads = min(os.cpu_count() or 1, 16)
    main_threads = O.num_threads()

    def solve(ij):
        O.set_threads(1)
        J, Ii = ij
        return O.local_keff(kappa[J * r:(J + 1) * r, Ii * r:(Ii + 1) * r], 0.8, 0.4, 0.1, 1e-6,
                            check_every=100, tol=1e-7, max_steps=2_000_000).keff

    O.lib()
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(threads) as ex:
        keff = np.array(list(ex.map(solve, [(J, Ii) for J in range(nc) for Ii in range(nc)])))
    t_local = time.perf_counter() - t0
    O.set_threads(main_threads)
    # coarse lattice: dx, dt x r; kappa / r^2, G x r, nu / r, tau_c = 1/2 + (tau - 1/2) / r
    pf = O.Params(nx=n, ny=n, tau=0.8, eps=0.4, nu=0.1)
    pc, sc = O.coarse_params(pf, r)
    pc = O.Params(nx=pc.nx, ny=pc.ny, tau=pc.tau, eps=pc.eps, nu=pc.nu, perm_kind=4)
    kt = (keff * sc["kappa"]).reshape(nc, nc, 4)
    t0 = time.perf_counter()
    rc = O.run(pc, kt, (1e-6 * sc["force"], 0.0), max_steps=4_000_000, check_every=100, tol=1e-6)
    t_coarse = time.perf_counter() - t0
    pfine = O.Params(nx=n, ny=n, tau=0.8, eps=0.4, nu=0.1)
    t0 = time.perf_counter()
    O.run(pfine, kappa, (1e-6, 0.0), max_steps=fine_sample_steps)
    dt = time.perf_counter() - t0
    mlups = n * n * fine_sample_steps / dt / 1e6
    return dict(kind="oracle", cores=threads, cpu_model=_cpu_model(),
                t_local_s=round(t_local, 3), local_items=int(nc * nc * 2),
                t_coarse_s=round(t_coarse, 4), coarse_steps=int(rc.steps),
                fine_mlups=round(mlups, 1),
                fine_sample=f"{fine_sample_steps} steps of {n}x{n}, {dt:.1f} s, {O.num_threads()} threads",
                t_fine_projected_s=round(res.fine_steps * n * n / (mlups * 1e6), 1),
                keff_max_rel_diff_vs_gpu=float(np.max(np.abs(keff - res.keff.reshape(-1, 4))) /
                                               np.max(np.abs(keff[:, [0, 3]]))))


def bench_seeds(L, torch, steps, no_local, seeds=(2, 3)):
    """The fine step and the local problems on the same workloads drawn with
    other seeds (the headline numbers use seed 1): fine MLUPS over `steps`
    steps (median of 3) and local patches/s (median of 3 calls)."""
    from paper_1312_0195_amd import inputs as I
    out = {}
    for seed in seeds:
        kappa = I.workload_fine(seed=seed)["kappa"]
        n = kappa.shape[0]
        f = bench_fine(L, torch, kappa, steps, 200, repeats=3)
        o = dict(fine_mlups_median=round(float(np.median(
            [n * n * steps / (ms * 1e-3) / 1e6 for ms in f["run_ms"]])), 1),
            fine_steps=steps, fine_step_kernel_us=round(f["step_kernel_ms"] * 1e3, 2))
        if not no_local:
            kd = torch.as_tensor(kappa).cuda()
            sets = {"tiles32": I.tile_patches(n, n, 32),
                    "mixed": I.mixed_patches(4096, n, n, seed=seed)}
            loc, _ = bench_local(L, torch, kd, reps=3, sets=sets)
            for k, v in loc.items():
                o[k + "_patches_per_s_median"] = round(v["patches_per_s"], 1)
                o[k + "_mean_steps"] = round(v["mean_steps"], 1)
            del kd
        out[f"seed{seed}"] = o
    return out


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(kappa, steps, single_steps=40):
    from oracle import oracle as O
    n = kappa.shape[0]
    p = O.Params(nx=n, ny=n, tau=0.8, eps=0.4, nu=0.1, walls_y=1)
    f = O.rest_state(p)
    t0 = time.perf_counter()
    O.run(p, kappa, (1e-6, 0.0), f=f, max_steps=steps)
    dt = time.perf_counter() - t0
    lu = steps * n * n
    threads = O.num_threads()
    # the same oracle on one thread (its results do not depend on the count)
    O.set_threads(1)
    t1 = time.perf_counter()
    O.run(p, kappa, (1e-6, 0.0), f=O.rest_state(p), max_steps=single_steps)
    dt1 = time.perf_counter() - t1
    O.set_threads(threads)
    return dict(value=lu / dt / 1e6, unit="MLUPS", cores=threads, kind="oracle",
                sample=f"{steps} steps of the {n}x{n} workload (FP64 C oracle, OpenMP over rows), "
                       f"{dt:.1f} s",
                single_thread_mlups=round(single_steps * n * n / dt1 / 1e6, 2),
                single_thread_sample=f"{single_steps} steps, {dt1:.1f} s", cpu_model=_cpu_model())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--cpu-steps", type=int, default=600)
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-local", action="store_true")
    ap.add_argument("--no-d3q19", action="store_true")
    ap.add_argument("--no-seeds", action="store_true", help="skip the seed 2 and 3 workloads")
    ap.add_argument("--no-upscale", action="store_true", help="skip the reduced upscaling leg")
    ap.add_argument("--no-paper-timing", action="store_true",
                    help="skip the 100 x 100 Sec. 4.1 leg (its 200000 steps swamp a profile)")
    ap.add_argument("--only-d3q19", action="store_true",
                    help="run the D3Q19 leg alone (for profiling) and print its object")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 302 MB device copy, the reference for HBM counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1312_0195_amd import inputs as I
    from paper_1312_0195_amd import lbm as L

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    L.lib()
    w = I.workload_fine(seed=1)
    kappa = w["kappa"]
    n = kappa.shape[0]
    cells = n * n
    if args.copy_calibration:
        # a plain copy kernel of known size: 9 planes of 2048 x 2048 FP32
        src = torch.ones(9 * cells, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_each_way": src.numel() * 4}), flush=True)
        del src, dst
    if args.only_d3q19:
        print(json.dumps({"d3q19": bench_d3q19(L, torch)}), flush=True)
        return
    fine = bench_fine(L, torch, kappa, args.steps, args.warmup)
    ms_per_step = fine["event_ms"] / args.steps
    mlups = cells * args.steps / (fine["event_ms"] * 1e-3) / 1e6
    step_ms = fine["step_kernel_ms"]  # one launch = DEPTH time steps
    # The multi-step kernel moves the state through HBM once per DEPTH steps;
    # its bound is the VALU. achieved: the collisions' FP32 arithmetic per
    # launch (DEPTH x cells lattice updates x FLOPS_PER_LU) over the launch,
    # against the published FP32 vector peak (which counts packed FP32; with
    # packed FP32 off the instruction rate allows half of it, reported too).
    t_launch = step_ms * 1e-3
    achieved = FLOPS_PER_LU * DEPTH * cells / t_launch / 1e12
    hbm_gbs = BYTES_PER_LU * cells / t_launch / 1e9
    traffic = _traffic_per_launch()
    valu = _valu_per_launch()
    result = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "fine 2048x2048 D2Q9 Brinkman LBM, log-normal K (sigma 1.5, "
                               "corr 32), tau 0.8, g 1e-6, walls in y, FP32 deviation "
                               "populations and FP32 collision arithmetic, FP64 mean-velocity "
                               "reduction every 100 steps",
                   "nx": n, "ny": n, "check_every": 100},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
                     "frac_of_unpacked_fp32": round(achieved / FP32_UNPACKED_TFLOPS, 4),
                     "peak_note": "the published FP32 vector rate counts packed FP32 FMAs; the "
                                  "kernels are built without packed FP32, whose instruction-rate "
                                  "ceiling is half that (frac_of_unpacked_fp32)",
                     "traffic": traffic,
                     "kernel": f"k_stepd<float, walls, scalar, no force field, {DEPTH}, float, no y drive> ({DEPTH} time steps per launch, FP32 arithmetic)",
                     "avg_launch_us": round(step_ms * 1e3, 3),
                     "launches_timed": KERNEL_LAUNCHES,
                     "warmup_launches": KERNEL_WARMUP_LAUNCHES,
                     "flops_per_launch": FLOPS_PER_LU * DEPTH * cells,
                     "lattice_updates_per_launch": DEPTH * cells,
                     "hbm_bytes_per_launch_algorithmic": BYTES_PER_LU * cells,
                     "hbm_achieved_gbs": round(hbm_gbs, 1),
                     "hbm_frac": round(hbm_gbs / HBM_PEAK_GBS, 4),
                     "valu_issue_frac": None if valu is None else
                     round(valu / (t_launch * VALU_ISSUE_PER_S), 4),
                     "single_step_hbm_equivalent_gbs": round(mlups * 1e6 * BYTES_PER_LU / 1e9, 1)},
        "wall_s": round(fine["wall_s"], 3),
        "mlups_runs": [round(cells * args.steps / (ms * 1e-3) / 1e6, 1) for ms in fine["run_ms"]],
    }
    result["mlups_median"] = float(np.median(result["mlups_runs"]))
    result["step_forms"] = bench_forms(L, torch, kappa)
    if not args.no_paper_timing:
        result["paper_sec41_timing"] = bench_paper_sec41(L, torch)
    if not args.no_local:
        kd = torch.as_tensor(kappa).cuda()
        result["local_keff"], keff_tiles = bench_local(L, torch, kd)
        result["coarse"] = bench_coarse(L, torch, keff_tiles)
        del kd
        if not args.no_cpu:
            result["local_keff"]["cpu_baseline"] = cpu_baseline_local(kappa)
    if not args.no_local and not args.no_upscale:
        result["upscale_reduced"], kap_u, res_u = bench_upscale_reduced(L, torch)
        if not args.no_cpu:
            result["upscale_reduced"]["cpu_baseline"] = cpu_baseline_upscale(kap_u, res_u)
    if not args.no_seeds:
        result["seeds"] = bench_seeds(L, torch, min(args.steps, 6000), args.no_local)
    if not args.no_surrogate and not args.no_local:
        result["keff_surrogate"] = bench_surrogate(cpu=not args.no_cpu)
    if not args.no_d3q19:
        result["d3q19"] = bench_d3q19(L, torch)
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(kappa, args.cpu_steps)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
