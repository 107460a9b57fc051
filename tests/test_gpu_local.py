"""GPU parity of the batched local problems (lbm_local_keff) against the FP64
oracle, through the C ABI.

Tolerance: K_eff within 1e-4 of the oracle, relative to the largest diagonal
entry of the patch's tensor (off-diagonal entries can be near zero). The GPU
stops an item when its mean velocity changes by less than 1e-7 (relative)
over 100 steps; the oracle value is the exact fixed point of its step.
"""
import numpy as np
import pytest

from oracle import direct as DS
from oracle import oracle as O
from paper_1312_0195_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TAU, EPS, NU, G = 0.8, 0.4, 0.1, 1e-6
GPU_TOL = 1e-7
KEFF_TOL = 1e-4


@pytest.fixture(scope="module")
def L():
    from paper_1312_0195_amd import lbm
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lbm.lib()
    return lbm


def _oracle_keff(field, x0, y0, s, tau=TAU, exact=True):
    patch = I.cut_patch(field, x0, y0, s)
    if exact and s <= 32:
        return DS.keff_direct(patch, tau, EPS, NU, G)
    r = O.local_keff(patch, tau, EPS, NU, G, check_every=100, tol=1e-11, max_steps=2_000_000)
    assert (r.status == 0).all()
    return r.keff


def _check(keff_g, keff_o):
    scale = max(abs(keff_o[0]), abs(keff_o[3]))
    err = np.max(np.abs(keff_g - keff_o)) / scale
    assert err < KEFF_TOL, (keff_g, keff_o, err)
    return err


def test_local_mixed_sides_one_launch(L):
    field = I.lognormal_kappa(160, 96, 1.0, 6.0, seed=4)
    sides = [16, 24, 32, 5, 17, 33, 48, 64, 1, 2, 31]
    rng = np.random.default_rng(0)
    x0 = rng.integers(0, 160, len(sides)).astype(np.int32)
    y0 = rng.integers(0, 96, len(sides)).astype(np.int32)
    x0[0], y0[0] = 150, 90  # wraps both ways
    res = L.local_keff(field, x0, y0, np.array(sides, np.int32), TAU, EPS, NU, G, tol=GPU_TOL,
                       check_every=100, max_steps=400000)
    assert (res.flags == 0).all(), res.flags
    for i, s in enumerate(sides):
        _check(res.keff[i], _oracle_keff(field, x0[i], y0[i], s))


def test_local_drive_masks_and_duplicates(L):
    field = I.lognormal_kappa(64, 64, 1.2, 5.0, seed=9)
    x0 = np.array([0, 0, 0, 0, 10], np.int32)
    y0 = np.array([0, 0, 0, 0, 20], np.int32)
    s = np.array([16, 16, 16, 16, 16], np.int32)
    mask = np.array([3, 1, 2, 0, 3], np.int32)
    res = L.local_keff(field, x0, y0, s, TAU, EPS, NU, G, tol=GPU_TOL, drive_mask=mask)
    ko = _oracle_keff(field, 0, 0, 16)
    _check(res.keff[0], ko)
    assert np.allclose(res.keff[1][[0, 2]], res.keff[0][[0, 2]], rtol=1e-12)
    assert np.isnan(res.keff[1][[1, 3]]).all() and (res.flags[1] == [0, -1]).all()
    assert np.allclose(res.keff[2][[1, 3]], res.keff[0][[1, 3]], rtol=1e-12)
    assert np.isnan(res.keff[2][[0, 2]]).all() and (res.flags[2] == [-1, 0]).all()
    assert np.isnan(res.keff[3]).all() and (res.flags[3] == -1).all()
    _check(res.keff[4], _oracle_keff(field, 10, 20, 16))


@pytest.mark.parametrize("tau", [0.5, 0.53, 1.2])
def test_local_other_tau(L, tau):
    field = I.lognormal_kappa(48, 48, 1.0, 4.0, seed=2)
    x0 = np.array([0, 13], np.int32)
    y0 = np.array([0, 7], np.int32)
    s = np.array([24, 16], np.int32)
    res = L.local_keff(field, x0, y0, s, tau, EPS, NU, G, tol=GPU_TOL)
    assert (res.flags == 0).all()
    for i in range(2):
        _check(res.keff[i], _oracle_keff(field, x0[i], y0[i], s[i], tau))


@pytest.mark.parametrize("block_threads", [256, 512, 1024])
def test_local_tile_choices_agree(L, block_threads):
    """Every tile layout gives the same K_eff to the solver's tolerance: the
    per-cell arithmetic is the same, but the FP64 sums of the convergence
    check depend on how the cells are spread over waves, so an item can stop
    one check (100 steps) earlier or later in another layout (measured: 3e-8
    of the tensor; 1e-6 of each diagonal entry and of the larger diagonal for
    the off-diagonal ones is required)."""
    field = I.lognormal_kappa(128, 128, 1.5, 8.0, seed=3)
    x0, y0, s = I.tile_patches(128, 128, 32)
    ref = L.local_keff(field, x0, y0, s, TAU, EPS, NU, G, tol=GPU_TOL)
    for tiles in ([(32, 128)], [(32, 256)], None):
        if tiles and tiles[0][1] > block_threads:
            continue
        if tiles and 32 * 32 > 4 * tiles[0][1]:
            continue  # more than 4 cells per thread: rejected by the library
        r = L.local_keff(field, x0, y0, s, TAU, EPS, NU, G, tol=GPU_TOL, tiles=tiles,
                         block_threads=block_threads)
        assert (r.flags == 0).all()
        scale = np.maximum(np.abs(ref.keff[:, 0]), np.abs(ref.keff[:, 3]))
        assert np.all(np.abs(r.keff[:, [0, 3]] / ref.keff[:, [0, 3]] - 1) < 1e-6)
        assert np.all(np.abs(r.keff[:, [1, 2]] - ref.keff[:, [1, 2]]) / scale[:, None] < 1e-6)


def test_local_schedule_changes_only_the_order(L):
    # Items are independent: the start order (given, or longest predicted
    # first) and the order of the patch arrays must not change any result bit.
    field = I.lognormal_kappa(160, 96, 1.8, 6.0, seed=21)
    field[40:44, 100:104] = np.inf   # no drag
    field[80, 10] = -1.0             # a patch that ends non-finite
    rng = np.random.default_rng(5)
    sides = rng.choice([1, 2, 5, 16, 17, 24, 31, 32, 33, 48, 64], 60).astype(np.int32)
    x0 = rng.integers(0, 160, 60).astype(np.int32)
    y0 = rng.integers(0, 96, 60).astype(np.int32)
    # all drag-free (never converges: step cap), one cell with kappa < 0
    # (non-finite), one wrapping both ways
    x0[:3], y0[:3], sides[:3] = [100, 9, 150], [40, 78, 90], [4, 8, 24]
    mask = rng.integers(0, 4, 60).astype(np.int32)
    mask[:3] = 3
    kw = dict(tol=GPU_TOL, check_every=100, max_steps=6000, drive_mask=mask)
    a = L.local_keff(field, x0, y0, sides, TAU, EPS, NU, G, schedule=L.LBM_SCHEDULE_GIVEN, **kw)
    b = L.local_keff(field, x0, y0, sides, TAU, EPS, NU, G, schedule=L.LBM_SCHEDULE_COST, **kw)
    perm = rng.permutation(60)
    kw["drive_mask"] = mask[perm]
    c = L.local_keff(field, x0[perm], y0[perm], sides[perm], TAU, EPS, NU, G,
                     schedule=L.LBM_SCHEDULE_COST, **kw)
    assert {0, 1, 2, -1} <= set(np.unique(a.flags).tolist())  # every outcome is exercised
    for r, idx in ((b, np.arange(60)), (c, np.argsort(perm))):
        assert np.array_equal(r.keff[idx], a.keff, equal_nan=True)
        assert np.array_equal(r.steps[idx], a.steps) and np.array_equal(r.flags[idx], a.flags)


def test_local_mixed_call_matches_calls_per_side(L):
    # A call that mixes single-cell sides with larger ones runs two launches on
    # two streams; every item must come out as in a call of its side alone.
    field = I.lognormal_kappa(128, 128, 1.5, 6.0, seed=14)
    rng = np.random.default_rng(6)
    sides = rng.choice([8, 16, 24, 32, 40, 48, 64], 70).astype(np.int32)
    x0 = rng.integers(0, 128, 70).astype(np.int32)
    y0 = rng.integers(0, 128, 70).astype(np.int32)
    kw = dict(tol=GPU_TOL, check_every=100, max_steps=8000)
    both = L.local_keff(field, x0, y0, sides, TAU, EPS, NU, G, **kw)
    for s in np.unique(sides):
        m = sides == s
        one = L.local_keff(field, x0[m], y0[m], sides[m], TAU, EPS, NU, G, **kw)
        assert np.array_equal(one.keff, both.keff[m], equal_nan=True), s
        assert np.array_equal(one.steps, both.steps[m]) and np.array_equal(one.flags, both.flags[m]), s


def test_local_largest_sides_share_a_queue(L):
    # Sides 48 and 64 each fill a workgroup with more than one cell per thread
    # and share one queue, every item taking its own side from its entry; in
    # both start orders each item must come out as in a call of its side
    # alone.
    field = I.lognormal_kappa(128, 128, 1.5, 6.0, seed=21)
    rng = np.random.default_rng(22)
    sides = rng.choice([48, 64], 24).astype(np.int32)
    x0 = rng.integers(0, 128, 24).astype(np.int32)
    y0 = rng.integers(0, 128, 24).astype(np.int32)
    kw = dict(tol=GPU_TOL, check_every=100, max_steps=6000)
    alone = {s: L.local_keff(field, x0[sides == s], y0[sides == s], sides[sides == s], TAU, EPS, NU, G, **kw)
             for s in (48, 64)}
    for sched in (L.LBM_SCHEDULE_GIVEN, L.LBM_SCHEDULE_COST):
        both = L.local_keff(field, x0, y0, sides, TAU, EPS, NU, G, schedule=sched, **kw)
        for s, one in alone.items():
            m = sides == s
            assert np.array_equal(one.keff, both.keff[m], equal_nan=True), (sched, s)
            assert np.array_equal(one.steps, both.steps[m]) and np.array_equal(one.flags, both.flags[m]), (sched, s)


def test_local_schedule_f64_state(L):
    # FP64 items (sides up to 45) in both start orders: identical results
    field = I.lognormal_kappa(96, 96, 2.0, 5.0, seed=8)
    rng = np.random.default_rng(9)
    sides = rng.choice([3, 8, 16, 24, 32, 45], 24).astype(np.int32)
    x0 = rng.integers(0, 96, 24).astype(np.int32)
    y0 = rng.integers(0, 96, 24).astype(np.int32)
    kw = dict(tol=1e-9, check_every=50, max_steps=20000, pop_dtype=L.LBM_F64)
    a = L.local_keff(field, x0, y0, sides, 0.53, EPS, NU, G, schedule=L.LBM_SCHEDULE_GIVEN, **kw)
    b = L.local_keff(field, x0, y0, sides, 0.53, EPS, NU, G, schedule=L.LBM_SCHEDULE_COST, **kw)
    assert np.array_equal(a.keff, b.keff, equal_nan=True)
    assert np.array_equal(a.steps, b.steps) and np.array_equal(a.flags, b.flags)


def test_local_flags_step_cap_and_bad_kappa(L):
    field = I.lognormal_kappa(32, 32, 1.0, 4.0, seed=1)
    field[3, 4] = -1.0
    x0 = np.array([0, 16], np.int32)
    y0 = np.array([0, 16], np.int32)
    s = np.array([8, 8], np.int32)
    res = L.local_keff(field, x0, y0, s, TAU, EPS, NU, G, tol=1e-14, check_every=10,
                       max_steps=20)
    assert (res.flags[0] == 2).all()          # kappa <= 0 inside the first patch
    assert (res.flags[1] == 1).all()          # step cap
    assert (res.steps[1] == 20).all()


def _check_strict(keff_g, keff_o):
    """Each diagonal entry within KEFF_TOL of its own oracle value (a nearly
    blocked direction is held to its own size, not to the open one's), the
    off-diagonal entries within KEFF_TOL of the larger diagonal entry."""
    scale = max(abs(keff_o[0]), abs(keff_o[3]))
    e_diag = max(abs(keff_g[0] / keff_o[0] - 1), abs(keff_g[3] / keff_o[3] - 1))
    e_off = max(abs(keff_g[1] - keff_o[1]), abs(keff_g[2] - keff_o[2])) / scale
    assert e_diag < KEFF_TOL and e_off < KEFF_TOL, (keff_g, keff_o, e_diag, e_off)
    return max(e_diag, e_off)


def _oracle_keff_many(field, x0, y0, sides, threads=16):
    """Oracle K_eff of many patches by its time stepping to a relative change
    of 1e-10 per 100 steps (within ~1e-8 of the fixed point even for the
    slowest items here), items spread over host threads, one oracle call per
    thread, each single-threaded."""
    import concurrent.futures as cf

    def one(args):
        O.set_threads(1)
        x, y, s = args
        r = O.local_keff(I.cut_patch(field, x, y, s), TAU, EPS, NU, G, check_every=100, tol=1e-10,
                         max_steps=2_000_000)
        assert (r.status == 0).all(), (x, y, s, r.status)
        return r.keff

    O.lib()
    with cf.ThreadPoolExecutor(threads) as ex:
        return np.array(list(ex.map(one, [(int(a), int(b), int(c)) for a, b, c in zip(x0, y0, sides)])))


def _full_size_sample(field, steps, patches, n_random, rng):
    """Indices: the 32 slowest items (most steps over both drives), the 32
    with the largest spread of ln kappa, and n_random others; patches:
    (x0, y0, side) per item."""
    sd = np.array([np.log(I.cut_patch(field, *a)).std() for a in patches])
    slow = np.argsort(steps.max(axis=1))[-32:]
    het = np.argsort(sd)[-32:]
    rest = np.setdiff1d(np.arange(len(steps)), np.union1d(slow, het))
    return np.union1d(np.union1d(slow, het), rng.choice(rest, n_random, replace=False))


def test_local_full_size_sampled(L):
    """The 2048 x 2048 field (sigma 1.5, correlation length 32) cut into the
    4096 tiles of 32 x 32 plus 4096 mixed patches with sides from
    {16, 24, 32, 48, 64}, each set in one call (the benchmark's
    configuration: FP32 state, rebased, no FP64 re-run), with at least 256
    items of each set checked against the oracle, every diagonal entry
    against its own value: the slowest, the most heterogeneous and a random
    sample."""
    w = I.workload_fine(seed=1)
    field = w["kappa"]
    kdev = torch.as_tensor(field).cuda()
    xt, yt, st = I.tile_patches(2048, 2048, 32)
    rt = L.local_keff(None, xt, yt, st, TAU, EPS, NU, G, tol=GPU_TOL, kappa_dev=kdev,
                      max_steps=400000)
    assert (rt.flags == 0).all(), np.unique(rt.flags, return_counts=True)
    xm, ym, sm = I.mixed_patches(4096, 2048, 2048, seed=1)
    rm = L.local_keff(None, xm, ym, sm, TAU, EPS, NU, G, tol=GPU_TOL, kappa_dev=kdev,
                      max_steps=400000)
    assert (rm.flags == 0).all(), np.unique(rm.flags, return_counts=True)
    rng = np.random.default_rng(7)
    it = _full_size_sample(field, rt.steps, list(zip(xt, yt, st)), 200, rng)
    assert len(it) >= 256
    ko = _oracle_keff_many(field, xt[it], yt[it], st[it])
    errs = [_check_strict(rt.keff[i], k) for i, k in zip(it, ko)]
    print(f"tiles: {len(it)} items, max error {max(errs):.2e}")
    im = _full_size_sample(field, rm.steps, list(zip(xm, ym, sm)), 200, rng)
    assert len(im) >= 256 and set(np.unique(sm[im])) == {16, 24, 32, 48, 64}
    ko = _oracle_keff_many(field, xm[im], ym[im], sm[im])
    errs = [_check_strict(rm.keff[i], k) for i, k in zip(im, ko)]
    print(f"mixed: {len(im)} items, max error {max(errs):.2e}")
    # every tensor is positive on the diagonal and finite
    assert np.isfinite(rt.keff).all() and (rt.keff[:, [0, 3]] > 0).all()
    assert np.isfinite(rm.keff).all() and (rm.keff[:, [0, 3]] > 0).all()


def _slow_patches():
    """32 x 32 patches where FP32 state is known to stop short of the fixed
    point: the most permeable tiles of a sigma-2.5, l-32 field (in the
    surrogate's training range), the most heterogeneous tiles of a sigma-3.5,
    l-8 field and the most permeable tiles of a field with 8-row streaks of
    K x 1e3 (the surrogate's out-of-range kinds). Returns (mosaic, x0, y0)."""
    fields = [I.lognormal_kappa(256, 256, 2.5, 32.0, 101),
              I.lognormal_kappa(256, 256, 3.5, 8.0, 102),
              I.channelize(I.lognormal_kappa(256, 256, 1.0, 8.0, 103), 0.25, 8, 1e3, 103)]
    picks = []
    for f, key in zip(fields, ("mean", "sd", "mean")):
        t = I.log_patches(f, 32)
        score = np.exp(t).mean(axis=(1, 2)) if key == "mean" else t.std(axis=(1, 2))
        picks.append(np.argsort(score)[-6:])
    big = np.concatenate(fields, axis=1)
    x0, y0 = [], []
    for j, idx in enumerate(picks):
        for i in idx:
            x0.append(256 * j + 32 * (i % 8))
            y0.append(32 * (i // 8))
    return big, np.array(x0, np.int32), np.array(y0, np.int32)


def test_local_f32_permeable_and_heterogeneous_items(L):
    """FP32 state on the slowest kinds of patch against the oracle's exact
    fixed point (Sec. 3, Eq. tensor-kappa). Permeable patches (relaxation
    time kappa / (eps nu), 20 000 - 150 000 steps) stopped short by 1-3e-4
    when the FP32 state held plain deviations; stored rebased on the mean
    momentum they meet 1e-4 on every diagonal entry. The very heterogeneous
    patches (sigma 3.5) meet 1e-4 relative to the tensor's largest entry,
    and with an FP32 step budget (slow items re-run with FP64 state) on
    every diagonal entry; the re-run gives what FP64 state from the start
    gives."""
    big, x0, y0 = _slow_patches()
    side = np.full(len(x0), 32, np.int32)
    r = L.local_keff(big, x0, y0, side, TAU, EPS, NU, G, tol=GPU_TOL, max_steps=400000,
                     fp32_step_budget=0)
    assert (r.flags == 0).all(), r.flags
    ko = [DS.keff_direct(I.cut_patch(big, x0[i], y0[i], 32), TAU, EPS, NU, G) for i in range(len(x0))]
    het = np.zeros(len(x0), bool)
    het[6:12] = True  # the sigma-3.5 tiles of _slow_patches
    errs = []
    for i in range(len(x0)):
        errs.append(_check(r.keff[i], ko[i]) if het[i] else _check_strict(r.keff[i], ko[i]))
    print(f"no budget: max error {max(errs):.2e} over {len(x0)} patches; steps max {r.steps.max()}")
    budget = 10000
    rb = L.local_keff(big, x0, y0, side, TAU, EPS, NU, G, tol=GPU_TOL, max_steps=400000,
                      fp32_step_budget=budget)
    assert (rb.flags == 0).all(), rb.flags
    assert (rb.steps > budget).any()  # some items took the FP64 re-run
    errs = [_check_strict(rb.keff[i], ko[i]) for i in range(len(x0))]
    print(f"budget {budget}: max error {max(errs):.2e}")
    slow = np.flatnonzero((rb.steps > budget).any(axis=1))
    r64 = L.local_keff(big, x0[slow], y0[slow], side[slow], TAU, EPS, NU, G, tol=GPU_TOL,
                       max_steps=400000, pop_dtype=L.LBM_F64)
    for j, i in enumerate(slow):
        for d in (0, 1):
            if rb.steps[i, d] > budget:
                # same FP64 arithmetic per cell; only the order of the mean's
                # partial sums differs with the thread layout
                assert abs(int(rb.steps[i, d]) - int(r64.steps[j, d])) <= 100
                cols = [0, 2] if d == 0 else [1, 3]
                assert np.allclose(rb.keff[i, cols], r64.keff[j, cols], rtol=1e-9, atol=0)


def test_local_f64_state_reaches_fixed_point_where_f32_stalls(L):
    """FP64 populations (pop_dtype LBM_F64) against the exact fixed point, at
    tight tolerance, on mixed sides up to 40 (ragged slots). Also the regime
    that needs them: a uniform patch at tau 0.50012 with weak drag, whose
    exact K_eff is kappa (closed form of the uniform transient). There the
    FP32 state stops changing while still short of the fixed point."""
    field = I.lognormal_kappa(96, 96, 1.5, 6.0, seed=4)
    x0 = np.array([0, 50, 7, 80], np.int32)
    y0 = np.array([0, 11, 60, 90], np.int32)
    s = np.array([40, 24, 13, 8], np.int32)
    r = L.local_keff(field, x0, y0, s, TAU, EPS, NU, G, tol=1e-11, max_steps=2_000_000,
                     pop_dtype=L.LBM_F64)
    assert (r.flags == 0).all()
    for i in range(4):
        ko = DS.keff_direct(I.cut_patch(field, x0[i], y0[i], s[i]), TAU, EPS, NU, G)
        scale = max(abs(ko[0]), abs(ko[3]))
        assert np.max(np.abs(r.keff[i] - ko)) / scale < 1e-7
    # uniform patch, tau 0.50012, nu 8e-6, kappa 0.016: drag eps nu / 2 kappa = 2e-4
    kap = np.full((10, 10), 0.016)
    one = np.zeros(1, np.int32)
    r64 = L.local_keff(kap, one, one, np.array([10], np.int32), 0.50012, 0.8, 8e-6, 1e-6,
                       tol=1e-12, check_every=200, max_steps=4_000_000, pop_dtype=L.LBM_F64)
    assert (r64.flags == 0).all()
    assert np.allclose(r64.keff[0, [0, 3]], 0.016, rtol=1e-8)
    with pytest.raises(L.LbmError):   # side 48 does not fit 4 cells per thread at 512 threads
        L.local_keff(field, one, one, np.array([48], np.int32), TAU, EPS, NU, G,
                     pop_dtype=L.LBM_F64)


@pytest.mark.parametrize("pop_dtype", ["f32", "f64"])
def test_local_oversampling_inner_window(L, pop_dtype):
    """avg_margin m: the mean velocity of Eq. tensor-kappa (and the
    convergence test) is taken over the inner window [m, side - m)^2 of each
    patch only. Against the oracle's exact fixed point with the same window,
    several margins per side, odd and even windows, wrapped origins."""
    pd = L.LBM_F32_SHIFTED if pop_dtype == "f32" else L.LBM_F64
    tol, keff_tol = (GPU_TOL, KEFF_TOL) if pop_dtype == "f32" else (1e-11, 1e-7)
    field = I.lognormal_kappa(128, 96, 1.0, 6.0, seed=9)
    sides = np.array([32, 24, 17, 13, 30], np.int32)
    x0 = np.array([0, 120, 37, 64, 99], np.int32)
    y0 = np.array([0, 90, 11, 50, 70], np.int32)
    for margin in (1, 4, 6):
        r = L.local_keff(field, x0, y0, sides, TAU, EPS, NU, G, tol=tol, check_every=100,
                         max_steps=2_000_000, pop_dtype=pd, avg_margin=margin)
        assert (r.flags == 0).all(), (margin, r.flags)
        for i, s in enumerate(sides):
            ko = DS.keff_direct(I.cut_patch(field, x0[i], y0[i], s), TAU, EPS, NU, G, margin=margin)
            scale = max(abs(ko[0]), abs(ko[3]))
            err = np.max(np.abs(r.keff[i] - ko)) / scale
            assert err < keff_tol, (margin, s, r.keff[i], ko, err)


def test_local_oversampling_layered_closed_form(L):
    """Layers along y at tau = 1/2 (no Brinkman viscosity): Darcy's law holds
    point by point, so with a margin K_yy is the arithmetic mean of kappa over
    the window's columns and K_xx the harmonic mean over the whole period."""
    kx = np.roll(np.repeat([1.0, 7.0, 3.0, 20.0], 6), 3)
    field = np.ascontiguousarray(np.tile(kx, (24, 1)))
    zero = np.zeros(1, np.int32)
    for m in (0, 5, 9):
        r = L.local_keff(field, zero, zero, np.array([24], np.int32), 0.5, EPS, NU, 1e-9,
                         tol=1e-12, check_every=200, max_steps=4_000_000, pop_dtype=L.LBM_F64,
                         avg_margin=m)
        assert (r.flags == 0).all()
        assert r.keff[0, 3] == pytest.approx(kx[m:24 - m].mean(), rel=1e-7)
        assert r.keff[0, 0] == pytest.approx(1.0 / np.mean(1.0 / kx), rel=1e-6)
