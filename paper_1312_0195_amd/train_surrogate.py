"""Train and evaluate the K_eff surrogate on the GPU.

    python -m paper_1312_0195_amd.train_surrogate [--train N] [--epochs E] [--out DIR]

1. Training data: N 32 x 32 tiles of 256 x 256 log-normal fields with sigma
   ~ U[0.5, 2.5] and correlation length ~ U[4, 32] (new seed per field),
   labelled by the batched local LBM (lbm_local_keff, both drives).
2. Training: Adam on the library's BF16-MFMA forward/backward kernels.
3. Test set: 65536 patches, about 90% from the training distribution (fresh
   seeds) and 10% outside it (sigma 3.5 at correlation length 8; sigma 1 at
   correlation length 1.5; 8-row channels of K x 1e3 on a sigma-1 field).
   Every test patch is also labelled by the LBM, the reference for the network's
   error. Reported: K_eff error of in-range patches (p50, p95, max), the same
   for the geometric-mean estimate exp(mean log K), how many patches the
   range detector sends to the LBM, and patches/s of network + fallback vs
   the batched LBM alone.
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

from . import inputs as I
from . import lbm as L
from . import surrogate as S

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_MODEL = os.path.join(HERE, "tuning", "surrogate_gfx950.npz")


def _fields_to_patches(fields):
    big, x0, y0 = S.mosaic(fields)
    return big, x0, y0


def test_set(n_total=65536, frac_oor=0.1, seed=12345):
    """(kappa mosaic, x0, y0, is_oor) with about frac_oor of the patches from
    out-of-range fields."""
    per = 64  # 32 x 32 tiles of a 256 x 256 field
    n_oor_fields = int(round(n_total * frac_oor / per))
    n_in_fields = n_total // per - n_oor_fields
    fields = [f for _, _, f in I.surrogate_fields(n_in_fields, seed)]
    rng = np.random.default_rng(seed + 1)
    oor = []
    for i in range(n_oor_fields):
        kind = i % 3
        s = int(rng.integers(1 << 30))
        if kind == 0:
            oor.append(I.lognormal_kappa(256, 256, 3.5, 8.0, s))
        elif kind == 1:
            oor.append(I.lognormal_kappa(256, 256, 1.0, 1.5, s))
        else:
            oor.append(I.channelize(I.lognormal_kappa(256, 256, 1.0, 8.0, s), 0.25, 8, 1e3, s))
    big, x0, y0 = S.mosaic(fields + oor)
    is_oor = np.zeros(len(x0), np.int8)  # 0 in range; 1, 2, 3: the three kinds above
    for i in range(n_oor_fields):
        is_oor[(n_in_fields + i) * per:(n_in_fields + i + 1) * per] = 1 + i % 3
    return big, x0, y0, is_oor


def calibration_patches(n=65536, seed=2):
    """Unlabelled log K patches from the training distribution with seeds
    the training set does not use (the network's spread on its own training
    patches is smaller than on new ones): the range detector's calibration."""
    big, x0, y0 = S.training_patches(n, seed=seed)
    return np.stack([np.log(I.cut_patch(big, a, b, S.SIDE)) for a, b in zip(x0, y0)]).astype(np.float32)


def _forward_timed(model, X, n_sym):
    """Device-resident forward of all patches: (pred, stats, seconds)."""
    import torch
    prm = torch.as_tensor(model.params).cuda()
    n = X.shape[0]
    pred = torch.empty((n, 2), dtype=torch.float32, device="cuda")
    st = torch.empty((n, 8), dtype=torch.float32, device="cuda")
    nb = L.lbm_cnn_workspace_bytes(n, False)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    L.lbm_cnn_forward(prm, n, X, n_sym, pred, st, ws, nb)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    L.lbm_cnn_forward(prm, n, X, n_sym, pred, st, ws, nb)
    e1.record()
    torch.cuda.synchronize()
    return (pred.cpu().numpy().astype(np.float64), st.cpu().numpy().astype(np.float64),
            e0.elapsed_time(e1) * 1e-3)


def evaluate(model: S.Surrogate, big, x0, y0, is_oor, sweep_nsym=(1, 2, 4, 8)):
    import torch
    kind = np.asarray(is_oor).astype(np.int8)
    is_oor = kind > 0
    # inputs resident on the device before any timing: the permeability
    # mosaic (for the LBM) and the log patches (for the network)
    big_dev = torch.as_tensor(big).cuda()
    logk = np.stack([np.log(I.cut_patch(big, a, b, S.SIDE)) for a, b in zip(x0, y0)])
    X = torch.as_tensor(logk.astype(np.float32)).cuda()
    n = len(x0)
    # LBM labels for every test patch (the reference), timed: the LBM-only
    # path (best of two runs, like the pipelined path below)
    t_lbm = None
    for _ in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        y_lbm, flags = S.label_patches(None, x0, y0, kappa_dev=big_dev)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        t_lbm = dt if t_lbm is None else min(t_lbm, dt)
    # network alone (kernel time only)
    p, stats, t_net = _forward_timed(model, X, model.n_sym)
    _, spread = model.predict_spread(logk)
    ok1 = model.in_range(stats)
    ok = ok1 & model.confident(spread)
    # network + fallback, pipelined: statistics, then the network on a second
    # stream while the LBM solves the patches flagged by the statistics, then
    # the LBM for the patches whose symmetric predictions disagree (best of
    # two runs)
    t_pipe = None
    for _ in range(2):
        combined, used_lbm, dt = S.keff_with_fallback(model, big_dev, x0, y0, X)
        t_pipe = dt if t_pipe is None else min(t_pipe, dt)
    assert (used_lbm == ~ok).all()
    good = (flags == 0).all(axis=1)
    inr = ok & ~is_oor & good
    err = np.abs(np.expm1(p[inr] - y_lbm[inr]))  # relative K_eff error
    geo = np.abs(np.expm1(stats[inr, 0][:, None] - y_lbm[inr]))
    err_all = np.abs(np.expm1(combined[good] - y_lbm[good]))
    acc_oor = ok & is_oor & good
    err_acc_oor = np.abs(np.expm1(p[acc_oor] - y_lbm[acc_oor])) if acc_oor.any() else np.zeros(1)

    def q(a):
        return dict(p50=float(np.quantile(a, 0.5)), p95=float(np.quantile(a, 0.95)),
                    p99=float(np.quantile(a, 0.99)), max=float(a.max()))

    # accuracy and speed against the number of symmetries averaged
    sweep = {}
    for ns in sweep_nsym:
        pn, _, tn = _forward_timed(model, X, ns)
        sweep[str(ns)] = dict(q(np.abs(np.expm1(pn[inr] - y_lbm[inr]))), patches_per_s=n / tn)

    by_kind = {}
    for kk, nm in ((1, "sigma3.5_l8"), (2, "sigma1_l1.5"), (3, "streaks")):
        m = (kind == kk) & good
        if m.any():
            acc = m & ok
            e = np.abs(np.expm1(p[acc] - y_lbm[acc])) if acc.any() else np.zeros(1)
            by_kind[nm] = dict(n=int(m.sum()), flagged=int((m & ~ok).sum()),
                               accepted_err_p50=float(np.quantile(e, 0.5)),
                               accepted_err_p95=float(np.quantile(e, 0.95)))
    return dict(
        n_patches=int(n), n_true_oor=int(is_oor.sum()), n_sym=int(model.n_sym),
        out_of_range_by_kind=by_kind,
        keff_error_in_range_by_n_sym=sweep,
        flagged=int((~ok).sum()), flagged_true_oor=int((~ok & is_oor).sum()),
        flagged_in_range=int((~ok & ~is_oor).sum()),
        flagged_by_statistics=int((~ok1).sum()), flagged_by_spread=int((ok1 & ~ok).sum()),
        lbm_label_failures=int((~good).sum()),
        keff_error_network_in_range=q(err),
        keff_error_geometric_mean_in_range=q(geo),
        keff_error_combined_all=q(err_all),
        keff_error_network_accepted_out_of_range=q(err_acc_oor),
        seconds_lbm_only=t_lbm, seconds_network=t_net, seconds_network_plus_fallback=t_pipe,
        patches_per_s_lbm_only=n / t_lbm,
        patches_per_s_network=n / t_net,
        patches_per_s_network_plus_fallback=n / t_pipe,
    )


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=200_000)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--test", type=int, default=65536)
    ap.add_argument("--model", default=DEFAULT_MODEL)
    ap.add_argument("--results", default=None)
    ap.add_argument("--recalibrate", action="store_true",
                    help="keep the trained weights of --model, recompute the range detector "
                         "from unlabelled held-out in-range patches, and evaluate")
    ap.add_argument("--q-feat", type=float, default=S.Q_FEAT,
                    help="quantile of the in-range Mahalanobis distances kept by stage one")
    ap.add_argument("--q-spread", type=float, default=S.Q_SPREAD,
                    help="quantile of the in-range symmetric spreads kept by stage two")
    args = ap.parse_args()
    import torch
    L.lib()
    if args.recalibrate:
        model = S.Surrogate.load(args.model)
        model.calibrate(calibration_patches(), q_feat=args.q_feat, q_spread=args.q_spread)
        model.save(args.model)
        bt, xt, yt, is_oor = test_set(args.test)
        res = evaluate(model, bt, xt, yt, is_oor)
        print(json.dumps(res), flush=True)
        if args.results:
            with open(args.results, "w") as fh:
                json.dump(res, fh, indent=1)
        return
    t0 = time.perf_counter()
    X, Y = S.training_set(args.train, seed=1)
    t_data = time.perf_counter() - t0
    print(f"training set: {len(X)} patches labelled in {t_data:.1f} s", flush=True)
    model = S.Surrogate.new(seed=0)
    t0 = time.perf_counter()
    model.fit(X, Y, epochs=args.epochs, batch=args.batch, lr=args.lr, verbose=True, calibrate=False)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    print(f"trained in {t_train:.1f} s", flush=True)
    model.calibrate(calibration_patches(), q_feat=args.q_feat, q_spread=args.q_spread)
    os.makedirs(os.path.dirname(args.model), exist_ok=True)
    model.save(args.model)
    big, x0, y0, is_oor = test_set(args.test)
    res = evaluate(model, big, x0, y0, is_oor)
    res.update(train_patches=int(len(X)), epochs=args.epochs, batch=args.batch,
               train_seconds=t_train, label_seconds=t_data, final_loss=model.history[-1],
               loss_history=model.history)
    print(json.dumps({k: v for k, v in res.items() if k != "loss_history"}), flush=True)
    if args.results:
        with open(args.results, "w") as fh:
            json.dump(res, fh, indent=1)


if __name__ == "__main__":
    main()
