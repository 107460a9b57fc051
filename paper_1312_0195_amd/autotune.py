"""Autotuner for the tile table of the batched local solver.

    python -m paper_1312_0195_amd.autotune [--out PATH] [--patches N]

For every patch side it times lbm_local_keff on a batch of that side under
every legal (block_threads, slot_threads) pair: slot_threads a multiple of 64
dividing block_threads, at most 4 cells per thread, the slots of a workgroup
fitting in LDS. It then keeps, per block size, the fastest slot size of each
side, times the mixed-size workload (4096 patches, sides 16..64) with each
block size, and keeps the winner. Last it times the start orders
(LBM_SCHEDULE_GIVEN, LBM_SCHEDULE_COST) with that table on two batches, 4096
patches of side 32 and the mixed workload, and keeps the faster one. The
result is written as JSON:

    {"block_threads": T, "tiles": [[side, slot_threads], ...], "schedule": S, ...}

    python -m paper_1312_0195_amd.autotune --schedule-only

re-times only the start order for the tile table already in the file.
lbm.local_keff() uses the table at DEFAULT_TABLE when it exists and no
explicit tiles (or schedule) are passed. Timings use the same synthetic
log-normal field (sigma 1.5, correlation length 32) as the benchmark.
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

from . import inputs as I
from . import lbm as L

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(HERE, "tuning", "local_tiles_gfx950.json")
SIDES = (16, 24, 32, 48, 64)
BLOCKS = (256, 512, 1024)
LDS_BYTES = 160 * 1024 - 2048


def legal_slots(side: int, block: int):
    out = []
    g = 64
    while g <= block:
        cells_per_thread = -(-side * side // g)
        if block % g == 0 and cells_per_thread <= 4 and 32 * side * side <= LDS_BYTES:
            out.append(g)
        g *= 2
    return out


def _time(fn, reps=2):
    import torch
    best = None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
    return best


def tune(n_patches: int = 1024, seed: int = 1, verbose: bool = True) -> dict:
    import torch
    field = I.lognormal_kappa(2048, 2048, 1.5, 32.0, seed)
    kd = torch.as_tensor(field).cuda()
    rng = np.random.default_rng(seed)
    per_side = {}
    for side in SIDES:
        x0 = rng.integers(0, 2048, n_patches).astype(np.int32)
        y0 = rng.integers(0, 2048, n_patches).astype(np.int32)
        s = np.full(n_patches, side, np.int32)
        for block in BLOCKS:
            for g in legal_slots(side, block):
                def run():
                    L.local_keff(None, x0, y0, s, 0.8, 0.4, 0.1, 1e-6, tol=1e-7, kappa_dev=kd,
                                 tiles=[(side, g)], block_threads=block)
                run()  # warm-up, and compile-time effects out of the timing
                dt = _time(run)
                per_side.setdefault(block, {}).setdefault(side, []).append((dt, g))
                if verbose:
                    print(f"side {side:3d} block {block:5d} slot {g:5d}: {n_patches / dt:10.0f} patches/s",
                          flush=True)
    xm, ym, sm = I.mixed_patches(4096, 2048, 2048, seed=seed)
    results = {}
    for block, sides in per_side.items():
        tiles = [(side, min(v)[1]) for side, v in sorted(sides.items())]
        if len(tiles) != len(SIDES):
            continue

        def run_mixed():
            L.local_keff(None, xm, ym, sm, 0.8, 0.4, 0.1, 1e-6, tol=1e-7, kappa_dev=kd,
                         tiles=tiles, block_threads=block)
        run_mixed()
        dt = _time(run_mixed)
        results[block] = (dt, tiles)
        if verbose:
            print(f"mixed block {block}: {4096 / dt:.0f} patches/s with {tiles}", flush=True)
    best_block = min(results, key=lambda b: results[b][0])
    dt, tiles = results[best_block]
    sched = tune_schedule(kd, best_block, tiles, seed, verbose)
    return {
        "block_threads": int(best_block),
        "tiles": [[int(a), int(b)] for a, b in tiles],
        **sched,
        "mixed_patches_per_s": 4096 / dt,
        "per_side": {str(b): {str(s): [[float(t), int(g)] for t, g in v] for s, v in d.items()}
                     for b, d in per_side.items()},
        "device": torch.cuda.get_device_name(0),
        "workload": "log-normal K sigma 1.5, corr 32 on 2048^2; tau 0.8, eps 0.4, nu 0.1, "
                    f"g 1e-6, tol 1e-7 per 100 steps; {n_patches} patches per side",
    }


def tune_schedule(kd, block: int, tiles, seed: int = 1, verbose: bool = True) -> dict:
    """{"schedule": the faster start order, "schedule_seconds": {...}} for the
    tile table (block, tiles), timed on 4096 patches of side 32 at random
    origins plus the mixed workload, on the device field kd."""
    n = kd.shape[1]
    rng = np.random.default_rng(seed + 7)
    batches = {
        "side32": (rng.integers(0, n, 4096).astype(np.int32), rng.integers(0, n, 4096).astype(np.int32),
                   np.full(4096, 32, np.int32)),
        "mixed": I.mixed_patches(4096, n, kd.shape[0], seed=seed),
    }
    secs = {}
    for sched, name in ((L.LBM_SCHEDULE_GIVEN, "given"), (L.LBM_SCHEDULE_COST, "cost")):
        secs[name] = {}
        for bname, (x0, y0, s) in batches.items():
            def run():
                L.local_keff(None, x0, y0, s, 0.8, 0.4, 0.1, 1e-6, tol=1e-7, kappa_dev=kd, tiles=tiles,
                             block_threads=block, schedule=sched)
            run()
            secs[name][bname] = _time(run)
        if verbose:
            print(f"schedule {name}: " + ", ".join(f"{b} {4096 / t:.0f} patches/s" for b, t in secs[name].items()),
                  flush=True)
    best = min(secs, key=lambda k: sum(secs[k].values()))
    return {"schedule": L.LBM_SCHEDULE_GIVEN if best == "given" else L.LBM_SCHEDULE_COST,
            "schedule_seconds": secs}


def load_schedule(path: str = DEFAULT_TABLE):
    """The tuned start order from a tuning file, or None."""
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    return int(t["schedule"]) if "schedule" in t else None


def load_table(path: str = DEFAULT_TABLE):
    """(block_threads, tiles) from a tuning file, or (0, None) if absent."""
    if not os.path.exists(path):
        return 0, None
    with open(path) as fh:
        t = json.load(fh)
    return int(t["block_threads"]), [tuple(x) for x in t["tiles"]]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--patches", type=int, default=1024)
    ap.add_argument("--schedule-only", action="store_true",
                    help="keep the tile table in --out and re-time only the start order")
    args = ap.parse_args()
    L.lib()
    if args.schedule_only:
        import torch
        with open(args.out) as fh:
            table = json.load(fh)
        kd = torch.as_tensor(I.lognormal_kappa(2048, 2048, 1.5, 32.0, 1)).cuda()
        table.update(tune_schedule(kd, int(table["block_threads"]), [tuple(x) for x in table["tiles"]]))
        with open(args.out, "w") as fh:
            json.dump(table, fh, indent=1)
        print(json.dumps({k: table[k] for k in ("block_threads", "tiles", "schedule", "schedule_seconds")}))
        return
    table = tune(args.patches)
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    with open(args.out, "w") as fh:
        json.dump(table, fh, indent=1)
    print(json.dumps({k: table[k] for k in ("block_threads", "tiles", "mixed_patches_per_s")}))


if __name__ == "__main__":
    main()
