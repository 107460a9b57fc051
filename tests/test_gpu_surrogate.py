"""GPU parity of the surrogate network kernels (BF16 MFMA, FP32 accumulate)
against the FP64 numpy oracle, through the C ABI.

Tolerances follow from BF16: activations and conv2-4 weights carry 8
significant bits (relative rounding 2^-9), so predictions agree to a few
1e-3 in log K and gradients to cosine >= 0.999 and relative L2 <= 3e-2 per
parameter tensor.
"""
import numpy as np
import pytest

from oracle import cnn_oracle as C
from paper_1312_0195_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

NAMES = ["W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4", "M1", "c1", "M2", "c2"]


@pytest.fixture(scope="module")
def L():
    from paper_1312_0195_amd import lbm
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lbm.lib()
    return lbm


def _flat(p):
    return np.concatenate([p[k].reshape(-1) for k in NAMES]).astype(np.float32)


def _unflat(v, like):
    out, o = {}, 0
    for k in NAMES:
        n = like[k].size
        out[k] = v[o:o + n].reshape(like[k].shape).astype(np.float64)
        o += n
    return out


def _params(seed):
    p = C.init_params(C=32, hidden=32, seed=seed)
    rng = np.random.default_rng(seed + 100)
    for k in ("b1", "b2", "b3", "b4", "c1"):
        p[k] = 0.05 * rng.standard_normal(p[k].shape)
    p["c2"] = np.array([0.1, -0.2])
    return p


def _patches(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        f = I.lognormal_kappa(32, 32, float(rng.uniform(0.5, 2.5)), float(rng.uniform(4, 16)),
                              int(rng.integers(1 << 30)))
        out.append(np.log(f) + rng.uniform(-2, 2))
    return np.stack(out)


def test_param_count_matches_layout(L):
    p = _params(0)
    assert L.lbm_cnn_param_count() == _flat(p).size == 29346


@pytest.mark.parametrize("batch", [1, 7, 300])
def test_forward_matches_oracle(L, batch):
    p = _params(1)
    x = _patches(batch, 2)
    y_o, cache = C.forward(p, x)
    pred_o = y_o + cache["m"][:, None]
    prm = torch.tensor(_flat(p), device="cuda")
    xd = torch.tensor(x.astype(np.float32), device="cuda")
    pred = torch.empty((batch, 2), dtype=torch.float32, device="cuda")
    stats = torch.empty((batch, 8), dtype=torch.float32, device="cuda")
    nb = L.lbm_cnn_workspace_bytes(batch, False)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    L.lbm_cnn_forward(prm, batch, xd, 1, pred, stats, ws, nb)
    torch.cuda.synchronize()
    pred = pred.cpu().numpy().astype(np.float64)
    err = np.abs(pred - pred_o)
    assert err.max() < 2e-2 * (1 + np.abs(pred_o).max()), err.max()
    assert np.sqrt((err ** 2).sum() / (pred_o ** 2).sum()) < 5e-3
    st = stats.cpu().numpy()
    xc = x - x.mean(axis=(1, 2), keepdims=True)
    sd = xc.std(axis=(1, 2))
    assert np.allclose(st[:, 0], x.mean(axis=(1, 2)), rtol=1e-5, atol=1e-5)
    assert np.allclose(st[:, 1], sd, rtol=1e-4)
    rx = (xc * np.roll(xc, -1, axis=2)).mean(axis=(1, 2)) / sd ** 2
    ry = (xc * np.roll(xc, -1, axis=1)).mean(axis=(1, 2)) / sd ** 2
    assert np.allclose(st[:, 2], rx, atol=1e-4) and np.allclose(st[:, 3], ry, atol=1e-4)
    # series/parallel features (FP32 exp and sums of 32 terms)
    assert np.allclose(st[:, 4:], C.series_parallel(xc), rtol=0, atol=2e-5)


@pytest.mark.parametrize("n_sym", [2, 5, 8])
def test_symmetric_forward_matches_oracle(L, n_sym):
    p = _params(11)
    x = _patches(37, 12)
    pred_o = C.predict_symmetric(p, x, n_sym)
    prm = torch.tensor(_flat(p), device="cuda")
    xd = torch.tensor(x.astype(np.float32), device="cuda")
    pred = torch.empty((37, 2), dtype=torch.float32, device="cuda")
    nb = L.lbm_cnn_workspace_bytes(37, False)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    L.lbm_cnn_forward(prm, 37, xd, n_sym, pred, None, ws, nb)
    err = np.abs(pred.cpu().numpy() - pred_o)
    assert err.max() < 2e-2 * (1 + np.abs(pred_o).max()), err.max()
    assert np.sqrt((err ** 2).sum() / (pred_o ** 2).sum()) < 5e-3


@pytest.mark.parametrize("n_sym", [1, 2, 5])
def test_forward_spread_matches_oracle(L, n_sym):
    """lbm_cnn_forward_spread: the same mean prediction as lbm_cnn_forward
    (bit for bit), and for each output the range (largest minus smallest) of
    the n_sym symmetric predictions, against the oracle's per-symmetry
    predictions mapped back to the patch's axes."""
    p = _params(15)
    x = _patches(23, 16)
    per = []
    for sym in range(n_sym):
        y, c = C.forward(p, C.transform(x, sym))
        q = y + c["m"][:, None]
        per.append(q[:, ::-1] if sym & 1 else q)
    per = np.stack(per)
    spread_o = per.max(axis=0) - per.min(axis=0)
    prm = torch.tensor(_flat(p), device="cuda")
    xd = torch.tensor(x.astype(np.float32), device="cuda")
    pred = torch.empty((23, 2), dtype=torch.float32, device="cuda")
    ref = torch.empty_like(pred)
    spr = torch.empty_like(pred)
    nb = L.lbm_cnn_workspace_bytes(23, False)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    L.lbm_cnn_forward_spread(prm, 23, xd, n_sym, pred, spr, 7, ws, nb)
    L.lbm_cnn_forward(prm, 23, xd, n_sym, ref, None, ws, nb)
    torch.cuda.synchronize()
    assert torch.equal(pred, ref)
    spr = spr.cpu().numpy()
    if n_sym == 1:
        assert (spr == 0).all()
    else:
        assert np.abs(spr - spread_o).max() < 2e-2 * (1 + np.abs(per).max()), np.abs(spr - spread_o).max()
        assert (spr >= 0).all()
    with pytest.raises(L.LbmError):
        L.lbm_cnn_forward_spread(prm, 23, xd, n_sym, pred, None, 0, ws, nb)


def test_symmetric_forward_is_equivariant_on_gpu(L):
    """With all eight symmetries averaged, a transformed patch reads exactly the
    same eight pixel arrangements as the original, so predictions agree up to
    the FP32 order of the average, with kxx and kyy exchanged by a transpose."""
    p = _params(13)
    x = _patches(3, 14)
    prm = torch.tensor(_flat(p), device="cuda")
    allx = np.concatenate([C.transform(x, s) for s in range(8)])
    xd = torch.tensor(allx.astype(np.float32), device="cuda")
    pred = torch.empty((24, 2), dtype=torch.float32, device="cuda")
    nb = L.lbm_cnn_workspace_bytes(24, False)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    L.lbm_cnn_forward(prm, 24, xd, 8, pred, None, ws, nb)
    pr = pred.cpu().numpy().reshape(8, 3, 2)
    for s in range(8):
        want = pr[0][:, ::-1] if s & 1 else pr[0]
        assert np.allclose(pr[s], want, rtol=0, atol=1e-5), s
    with pytest.raises(L.LbmError):
        L.lbm_cnn_forward(prm, 24, xd, 9, pred, None, ws, nb)
    with pytest.raises(L.LbmError):
        L.lbm_cnn_forward(prm, 24, xd, 0, pred, None, ws, nb)


def test_forward_shift_invariance_on_gpu(L):
    p = _params(3)
    x = _patches(4, 5)
    xs = np.roll(x, (7, -11), axis=(1, 2))
    prm = torch.tensor(_flat(p), device="cuda")
    nb = L.lbm_cnn_workspace_bytes(8, False)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    both = torch.tensor(np.concatenate([x, xs]).astype(np.float32), device="cuda")
    pred = torch.empty((8, 2), dtype=torch.float32, device="cuda")
    L.lbm_cnn_forward(prm, 8, both, 1, pred, None, ws, nb)
    pr = pred.cpu().numpy()
    # Invariant in exact arithmetic. On the GPU the patch mean (and the pooled
    # sums) are added in a different pixel order after a shift, which can move
    # a BF16 rounding of an activation by one unit: differences stay ~1e-5.
    assert np.allclose(pr[:4], pr[4:], rtol=0, atol=1e-4)


@pytest.mark.parametrize("batch,with_sym", [(3, False), (64, False), (40, True)])
def test_gradients_match_oracle(L, batch, with_sym):
    """With per-patch symmetries the oracle sees the transformed patches and
    the targets exchanged for the transposed ones."""
    p = _params(4)
    x = _patches(batch, 6)
    rng = np.random.default_rng(7)
    t = x.mean(axis=(1, 2))[:, None] + rng.normal(0.3, 0.5, (batch, 2))
    sym = rng.integers(0, 8, batch).astype(np.int8) if with_sym else np.zeros(batch, np.int8)
    xo = np.stack([C.transform(x[i:i + 1], int(sym[i]))[0] for i in range(batch)])
    to = np.where((sym & 1)[:, None] == 1, t[:, ::-1], t)
    y_o, cache = C.forward(p, xo)
    g_o = C.backward(p, cache, y_o, to - cache["m"][:, None])
    loss_o = C.loss(y_o, to - cache["m"][:, None])
    prm = torch.tensor(_flat(p), device="cuda")
    xd = torch.tensor(x.astype(np.float32), device="cuda")
    sd = torch.tensor(sym, device="cuda") if with_sym else None
    td = torch.tensor(t.astype(np.float32), device="cuda")
    grad = torch.empty_like(prm)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    pred = torch.empty((batch, 2), dtype=torch.float32, device="cuda")
    nb = L.lbm_cnn_workspace_bytes(batch, True)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    L.lbm_cnn_gradients(prm, batch, xd, sd, td, grad, loss, pred, ws, nb)
    torch.cuda.synchronize()
    assert abs(float(loss.item()) - loss_o) < 2e-2 * loss_o
    po = y_o + cache["m"][:, None]
    po = np.where((sym & 1)[:, None] == 1, po[:, ::-1], po)  # back to the patch's own axes
    pe = np.abs(pred.cpu().numpy() - po)
    assert pe.max() < 2e-2 * (1 + np.abs(y_o).max())
    g = _unflat(grad.cpu().numpy(), p)
    for k in NAMES:
        a, b = g[k].ravel(), g_o[k].ravel()
        cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-300)
        rel = np.linalg.norm(a - b) / (np.linalg.norm(b) + 1e-300)
        assert cos > 0.999 and rel < 3e-2, (k, cos, rel)
    # deterministic: the same call gives the same bits
    grad2 = torch.empty_like(prm)
    L.lbm_cnn_gradients(prm, batch, xd, sd, td, grad2, loss, pred, ws, nb)
    assert torch.equal(grad, grad2)


def test_adam_step_matches_oracle(L):
    p = _params(8)
    x = _patches(16, 9)
    t = x.mean(axis=(1, 2))[:, None] + 0.5
    prm = torch.tensor(_flat(p), device="cuda")
    m = torch.zeros_like(prm)
    v = torch.zeros_like(prm)
    xd = torch.tensor(x.astype(np.float32), device="cuda")
    td = torch.tensor(t.astype(np.float32), device="cuda")
    nb = L.lbm_cnn_workspace_bytes(16, True)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    grad = torch.empty_like(prm)
    pred = torch.empty((16, 2), dtype=torch.float32, device="cuda")
    sd = torch.tensor(np.arange(16, dtype=np.int8) % 8, device="cuda")
    L.lbm_cnn_gradients(prm, 16, xd, sd, td, grad, None, pred, ws, nb)
    g = grad.cpu().numpy().astype(np.float64)
    before = prm.cpu().numpy().astype(np.float64)
    L.lbm_cnn_train_step(prm, m, v, 1, 1e-3, 16, xd, sd, td, None, ws, nb)
    torch.cuda.synchronize()
    ref = {"w": before.copy()}
    C.adam_step(ref, {"w": g}, {}, lr=1e-3)
    assert np.allclose(prm.cpu().numpy(), ref["w"], rtol=0, atol=2e-6)


def test_forward_full_batch_sampled(L):
    """The benchmark's batch: 65536 patches in one launch with n_sym = 2 and
    the statistics; 12 sampled patches (first, last, spread) against the
    oracle's symmetric prediction and statistics."""
    from paper_1312_0195_amd import surrogate as S
    from paper_1312_0195_amd import train_surrogate as T
    model = S.Surrogate.load(T.DEFAULT_MODEL)
    fields = [f for _, _, f in I.surrogate_fields(1024, 77)]
    big, x0, y0 = S.mosaic(fields)
    n = len(x0)
    assert n == 65536
    logk = np.stack([np.log(I.cut_patch(big, a, b, 32)) for a, b in zip(x0, y0)]).astype(np.float32)
    pred, stats = model.predict(logk, n_sym=2)
    pd = _unflat(model.params, _params(0))
    idx = np.concatenate([[0, n - 1], np.random.default_rng(5).choice(n, 10, replace=False)])
    po = C.predict_symmetric(pd, logk[idx].astype(np.float64), 2)
    err = np.abs(pred[idx] - po)
    assert err.max() < 2e-2 * (1 + np.abs(po).max()), err.max()
    xc = logk[idx] - logk[idx].mean(axis=(1, 2), keepdims=True)
    assert np.allclose(stats[idx, 0], logk[idx].mean(axis=(1, 2)), rtol=1e-5, atol=1e-5)
    assert np.allclose(stats[idx, 4:], C.series_parallel(xc.astype(np.float64)), atol=2e-5)


def test_patch_stats_equal_forward_stats(L):
    """lbm_patch_stats gives the forward kernel's statistics bit for bit."""
    p = _params(21)
    x = _patches(300, 22).astype(np.float32)
    prm = torch.tensor(_flat(p), device="cuda")
    xd = torch.tensor(x, device="cuda")
    pred = torch.empty((300, 2), dtype=torch.float32, device="cuda")
    st_f = torch.empty((300, 8), dtype=torch.float32, device="cuda")
    st_s = torch.full((300, 8), float("nan"), dtype=torch.float32, device="cuda")
    nb = L.lbm_cnn_workspace_bytes(300, False)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    L.lbm_cnn_forward(prm, 300, xd, 2, pred, st_f, ws, nb)
    L.lbm_patch_stats(300, xd, st_s)
    torch.cuda.synchronize()
    assert torch.equal(st_f, st_s)
    with pytest.raises(L.LbmError):
        L.lbm_patch_stats(0, xd, st_s)


def test_forward_with_fewer_workgroups_is_identical(L):
    """lbm_cnn_forward_limited: any cap on the workgroups gives the same bits
    (each workgroup claims patches one at a time; a patch's arithmetic does
    not depend on which workgroup runs it)."""
    from paper_1312_0195_amd import surrogate as S
    from paper_1312_0195_amd import train_surrogate as T
    model = S.Surrogate.load(T.DEFAULT_MODEL)
    n = 777
    x = torch.randn((n, 32, 32), generator=torch.Generator().manual_seed(3)).cuda()
    prm = torch.as_tensor(model.params).cuda()
    nb = L.lbm_cnn_workspace_bytes(n, False)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    ref = torch.empty((n, 2), dtype=torch.float32, device="cuda")
    rst = torch.empty((n, 8), dtype=torch.float32, device="cuda")
    L.lbm_cnn_forward(prm, n, x, 2, ref, rst, ws, nb)
    for cap in (1, 5, 96, 4096, 0):
        out = torch.empty_like(ref)
        st = torch.empty_like(rst)
        L.lbm_cnn_forward_limited(prm, n, x, 2, out, st, cap, ws, nb)
        torch.cuda.synchronize()
        assert torch.equal(out, ref) and torch.equal(st, rst), cap
    with pytest.raises(L.LbmError):
        L.lbm_cnn_forward_limited(prm, n, x, 2, out, st, -1, ws, nb)


def test_pipelined_fallback_matches_separate_paths(L):
    """keff_with_fallback (statistics, then the network on a second stream
    concurrent with the LBM on the patches the statistics flag, then the LBM
    on the patches whose symmetric predictions disagree) returns the
    network's prediction where both stages accept a patch and the LBM's
    elsewhere, whatever the cap on the network's workgroups."""
    from paper_1312_0195_amd import surrogate as S
    from paper_1312_0195_amd import train_surrogate as T
    model = S.Surrogate.load(T.DEFAULT_MODEL)
    big, x0, y0, kind = T.test_set(64 * 12, 0.25, seed=8)
    kd = torch.as_tensor(big).cuda()
    logk = np.stack([np.log(I.cut_patch(big, a, b, 32)) for a, b in zip(x0, y0)]).astype(np.float32)
    xd = torch.as_tensor(logk).cuda()
    pred, stats = model.predict(logk)
    pred2, spread = model.predict_spread(logk)
    assert np.array_equal(pred, pred2)
    ok1 = model.in_range(stats)
    ok = ok1 & model.confident(spread)
    assert (~ok1).any() and (ok1 & ~ok).any() and ok.any()  # both stages flag something here
    y_lbm, _ = S.label_patches(None, x0[~ok], y0[~ok], kappa_dev=kd)
    for wg in (0, 96, None):
        out, used, secs = S.keff_with_fallback(model, kd, x0, y0, xd, network_workgroups=wg)
        assert (used == ~ok).all()
        assert np.array_equal(out[ok], pred[ok])
        assert np.allclose(out[~ok], y_lbm, rtol=0, atol=1e-12)
        assert secs > 0


def test_trained_network_gains_over_the_method_without_it(L):
    """What the trained network (the committed model) adds, on 16384 fresh
    test patches (90% from in-range fields, 10% from three out-of-range
    kinds), with the batched local LBM as the reference: (1) against the
    method without the local problems (the block geometric mean of kappa as
    K_eff) it is far more accurate; (2) against the method without the
    network (the batched LBM for every patch) the network plus LBM fallback
    is faster, at the accuracy the surrogate path is specified for: K_eff
    within 2% at the 95th percentile, in range and over all patches."""
    from paper_1312_0195_amd import surrogate as S
    from paper_1312_0195_amd import train_surrogate as T
    model = S.Surrogate.load(T.DEFAULT_MODEL)
    big, x0, y0, kind = T.test_set(16384)
    r = T.evaluate(model, big, x0, y0, kind, sweep_nsym=(model.n_sym,))
    net, geo = r["keff_error_network_in_range"], r["keff_error_geometric_mean_in_range"]
    allp = r["keff_error_combined_all"]
    print({k: r[k] for k in ("flagged", "flagged_true_oor", "flagged_in_range", "flagged_by_statistics",
                              "flagged_by_spread")}, net, allp)
    assert r["lbm_label_failures"] == 0
    assert net["p50"] < 0.005 and net["p95"] <= 0.02, net
    assert net["p50"] < geo["p50"] / 10 and net["p95"] < geo["p95"] / 10, (net, geo)
    assert allp["p95"] <= 0.02 and allp["p99"] <= 0.05, allp
    speedup = r["patches_per_s_network_plus_fallback"] / r["patches_per_s_lbm_only"]
    assert speedup > 1.5, (speedup, r["patches_per_s_network_plus_fallback"], r["patches_per_s_lbm_only"])


def test_training_on_gpu_learns(L):
    """End-to-end training by the library's own kernels (forward, backward,
    Adam): 4096 patches labelled by the batched LBM, 12 epochs from a fresh
    initialisation. The loss falls by an order of magnitude and the trained
    network beats the geometric-mean estimate on held-out patches."""
    from paper_1312_0195_amd import surrogate as S
    big, x0, y0 = S.training_patches(4096 + 1024, seed=77)
    y, flags = S.label_patches(big, x0, y0)
    assert (flags == 0).all()
    logk = np.stack([np.log(I.cut_patch(big, a, b, S.SIDE)) for a, b in zip(x0, y0)])
    tr, te = slice(0, 4096), slice(4096, None)
    model = S.Surrogate(S.init_params(seed=5), n_sym=1)
    model.fit(logk[tr], y[tr], epochs=12, batch=256, lr=2e-3)
    h = model.history
    assert len(h) == 12 and np.isfinite(h).all()
    assert h[-1] < 0.1 * h[0], h
    pred, stats = model.predict(logk[te], n_sym=1)
    err = np.abs(np.expm1(pred - y[te]))
    geo = np.abs(np.expm1(stats[:, [0]] - y[te]))
    assert np.median(err) < 0.5 * np.median(geo), (np.median(err), np.median(geo))
