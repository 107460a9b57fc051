"""GPU parity of the fine-grid solver (lbm_init / lbm_step / lbm_fields)
against the FP64 CPU oracle, through the C ABI.

Tolerances: FP64 populations agree with the oracle to 1e-9 of the velocity
scale (only the rounding order differs; the oracle keeps full populations, so
its own FP64 floor is near 1e-11 of a velocity that is 1e-5 of f). FP32 deviation populations must stay
within 1e-5 of the velocity scale (the stated target for the velocity field).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1312_0195_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def L():
    from paper_1312_0195_amd import lbm
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lbm.lib()
    return lbm


def _gpu_run(L, nx, ny, kappa, tau, eps, nu, g, walls, steps, dtype, force=None, perm_kind=1,
             scheme=0):
    p = L.make_params(nx, ny, tau, eps, nu, 1.0, g[0], g[1], walls, dtype, perm_kind, scheme)
    s = L.FineSolver(p, kappa, force)
    st, done, mu = s.step(steps)
    assert st == L.LBM_OK and done == steps
    u, rho = s.fields()
    out = u.cpu().numpy(), rho.cpu().numpy(), mu, s
    return out


def _oracle_run(nx, ny, kappa, tau, eps, nu, g, walls, steps, force=None, perm_kind=1, scheme=0):
    p = O.Params(nx=nx, ny=ny, tau=tau, eps=eps, nu=nu, walls_y=walls, perm_kind=perm_kind,
                 scheme=scheme)
    r = O.run(p, kappa, g, max_steps=steps, force=force)
    rho, ux, uy = O.moments(p, kappa, r.f, g, force)
    return np.stack([ux, uy]), rho, r


def _rel_field_err(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


CASES = [
    # nx, ny, walls, tau
    (64, 64, 1, 0.8),    # the small workload's grid
    (37, 23, 1, 0.8),    # ragged, smaller than one block row
    (300, 7, 0, 0.53),   # two blocks per row with a ragged tail, periodic
    (257, 5, 1, 0.5),    # tau = 1/2, one cell past a block
    (1, 9, 1, 1.3),      # a single column
]


@pytest.mark.parametrize("nx,ny,walls,tau", CASES)
def test_fine_f64_matches_oracle(L, nx, ny, walls, tau):
    k = I.lognormal_kappa(nx, ny, 1.0, 4.0, seed=3)
    g = (1e-6, 2e-7)
    u_o, rho_o, r = _oracle_run(nx, ny, k, tau, 0.4, 0.1, g, walls, 150)
    u_g, rho_g, mu, s = _gpu_run(L, nx, ny, k, tau, 0.4, 0.1, g, walls, 150, L.LBM_F64)
    assert _rel_field_err(u_g, u_o) < 1e-9
    assert np.max(np.abs(rho_g - rho_o)) < 1e-13
    assert np.allclose(mu, r.mean_u, rtol=1e-9)
    f_g = s.populations().cpu().numpy()
    f_o = np.moveaxis(r.f, 2, 0)
    assert np.max(np.abs(f_g - f_o)) < 1e-14


@pytest.mark.parametrize("mode", ["LBM_F32_SHIFTED", "LBM_F32_FAST"])
@pytest.mark.parametrize("nx,ny,walls,tau", CASES)
def test_fine_f32_matches_oracle(L, nx, ny, walls, tau, mode):
    """FP32 state with FP64 (SHIFTED) or FP32 (FAST) collision arithmetic."""
    k = I.lognormal_kappa(nx, ny, 1.5, 4.0, seed=5)
    g = (1e-6, 0.0)
    u_o, rho_o, r = _oracle_run(nx, ny, k, tau, 0.4, 0.1, g, walls, 300)
    u_g, rho_g, mu, _ = _gpu_run(L, nx, ny, k, tau, 0.4, 0.1, g, walls, 300, getattr(L, mode))
    assert _rel_field_err(u_g, u_o) < 1e-5
    assert np.max(np.abs(rho_g - rho_o)) < 1e-9
    assert np.allclose(mu, r.mean_u, rtol=1e-5)


@pytest.mark.parametrize("dtype", ["f64", "f32", "f32_fast"])
def test_fine_tensor_and_force_field(L, dtype):
    nx, ny = 29, 18
    rng = np.random.default_rng(2)
    kxx = np.exp(rng.standard_normal((ny, nx)))
    kyy = np.exp(rng.standard_normal((ny, nx)))
    kxy = 0.2 * np.sqrt(kxx * kyy) * rng.uniform(-1, 1, (ny, nx))
    kt = np.stack([kxx, kxy, 0.7 * kxy, kyy], axis=-1)
    force = 1e-6 * rng.standard_normal((ny, nx, 2))
    u_o, _, _ = _oracle_run(nx, ny, kt, 0.7, 0.5, 0.1, (0, 0), 0, 200, force, 4)
    dt = {"f64": L.LBM_F64, "f32": L.LBM_F32_SHIFTED, "f32_fast": L.LBM_F32_FAST}[dtype]
    u_g, _, _, _ = _gpu_run(L, nx, ny, kt, 0.7, 0.5, 0.1, (0, 0), 0, 200, dt, force, 4)
    assert _rel_field_err(u_g, u_o) < (1e-9 if dtype == "f64" else 1e-5)


@pytest.mark.parametrize("nx,ny,walls,tau,with_force", [(64, 64, 1, 0.8, False), (300, 7, 0, 0.53, True),
                                                       (37, 23, 1, 0.5, True)])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_guo_form_matches_oracle_guo_form(L, nx, ny, walls, tau, with_force, dtype):
    """The Guo form (Sec. 2.1) on the GPU against the oracle's own Guo form."""
    k = I.lognormal_kappa(nx, ny, 1.2, 4.0, seed=13)
    force = 1e-6 * np.random.default_rng(3).standard_normal((ny, nx, 2)) if with_force else None
    g = (1e-6, 2e-7)
    u_o, rho_o, _ = _oracle_run(nx, ny, k, tau, 0.4, 0.1, g, walls, 200, force, 1, 1)
    dt = L.LBM_F64 if dtype == "f64" else L.LBM_F32_SHIFTED
    u_g, rho_g, _, _ = _gpu_run(L, nx, ny, k, tau, 0.4, 0.1, g, walls, 200, dt, force, 1, 1)
    assert _rel_field_err(u_g, u_o) < (1e-9 if dtype == "f64" else 1e-5)
    assert np.max(np.abs(rho_g - rho_o)) < (1e-13 if dtype == "f64" else 1e-9)


def test_guo_form_equals_shan_chen_form_on_gpu(L):
    """With the linear f_eq the two forms are algebraically equal (Sec. 2.1 vs
    2.2): FP64 populations agree to rounding after 300 steps."""
    nx, ny = 96, 40
    k = I.lognormal_kappa(nx, ny, 1.5, 6.0, seed=14)
    _, _, _, a = _gpu_run(L, nx, ny, k, 0.7, 0.4, 0.1, (1e-6, 3e-7), 1, 300, L.LBM_F64)
    _, _, _, b = _gpu_run(L, nx, ny, k, 0.7, 0.4, 0.1, (1e-6, 3e-7), 1, 300, L.LBM_F64, None, 1, 1)
    fa, fb = a.populations().cpu().numpy(), b.populations().cpu().numpy()
    ja = fa[1] - fa[3]
    assert np.max(np.abs(fa - fb)) < 1e-9 * np.max(np.abs(ja))
    with pytest.raises(L.LbmError):
        L.FineSolver(L.make_params(8, 8, 0.7, 0.4, 0.1, 1.0, 1e-6, 0.0, 0, L.LBM_F64,
                                   L.LBM_PERM_TENSOR, L.LBM_SCHEME_GUO),
                     np.broadcast_to([1.0, 0.0, 0.0, 1.0], (8, 8, 4)).copy())


def test_fine_converges_to_oracle_steady_state(L):
    """The small workload: 64 x 64, sigma 1, correlation length 8, walls in
    y, tau 0.8, g = 1e-6, to a relative mean-velocity change < 1e-9."""
    w = I.workload_small(seed=1)
    k, g = w["kappa"], (w["g"], 0.0)
    po = O.Params(nx=64, ny=64, tau=w["tau"], eps=w["eps"], nu=w["nu"], walls_y=1)
    ro = O.run(po, k, g, max_steps=400000, check_every=100, tol=1e-11)
    assert ro.status == O.OK
    for dtype, tol_u in [(L.LBM_F64, 1e-8), (L.LBM_F32_SHIFTED, 1e-5)]:
        p = L.make_params(64, 64, w["tau"], w["eps"], w["nu"], 1.0, g[0], 0.0, 1, dtype)
        s = L.FineSolver(p, k)
        st, done, mu = s.step(400000, tol=1e-9 if dtype == L.LBM_F64 else 1e-7, check_every=100)
        assert st == L.LBM_OK, L.lbm_last_error()
        assert np.allclose(mu, ro.mean_u, rtol=tol_u, atol=tol_u * abs(ro.mean_u[0]))
        u, _ = s.fields()
        _, uxo, uyo = O.moments(po, k, ro.f, g)
        assert _rel_field_err(u.cpu().numpy(), np.stack([uxo, uyo])) < 10 * tol_u


@pytest.mark.parametrize("nx,ny,walls", [(2048, 96, 1), (130, 70, 0), (200, 37, 1), (64, 33, 1),
                                         (5, 3, 0), (3, 40, 1)])
@pytest.mark.parametrize("dtype", ["f32", "f64", "f32_fast"])
def test_multi_step_launches_match_single_steps_bitwise(L, nx, ny, walls, dtype):
    """lbm_step advances several steps per launch (temporal blocking in LDS:
    7 (FP32 collision arithmetic only), 6, 4 or 2 steps, FP32 or FP64 state)
    whenever no check falls in between; the state must equal that of
    single-step launches bit for bit (ragged tiles, walls, periodic y, grids
    smaller than the halo)."""
    dt = {"f64": L.LBM_F64, "f32": L.LBM_F32_SHIFTED, "f32_fast": L.LBM_F32_FAST}[dtype]
    k = I.lognormal_kappa(nx, ny, 1.5, 6.0, seed=11)
    p = L.make_params(nx, ny, 0.7, 0.4, 0.1, 1.0, 1e-6, 3e-7, walls, dt)
    a = L.FineSolver(p, k)
    b = L.FineSolver(p, k)
    for n in (37, 11, 3):      # FP32: 6x6 + 1, 6 + 4 + 1, 2 + 1 steps per launch;
                               # FP32 arithmetic: 7 + 5x6, 7 + 4, 2 + 1
        a.step(n)
    for _ in range(51):
        b.step(1)              # single-step launches only
    fa = a.populations().cpu().numpy()
    fb = b.populations().cpu().numpy()
    assert np.array_equal(fa, fb)


@pytest.mark.parametrize("scheme,perm_kind,force", [(0, 4, True), (1, 1, True), (0, 1, True)])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_multi_step_launches_bitwise_all_kernel_forms(L, scheme, perm_kind, force, dtype):
    """The same on the other kernel forms: tensor permeability, the Guo form,
    a per-cell force field (periodic y, ragged tiles)."""
    nx, ny = 150, 45
    rng = np.random.default_rng(4)
    if perm_kind == 4:
        kxx = np.exp(rng.standard_normal((ny, nx)))
        kyy = np.exp(rng.standard_normal((ny, nx)))
        kxy = 0.2 * np.sqrt(kxx * kyy) * rng.uniform(-1, 1, (ny, nx))
        k = np.stack([kxx, kxy, 0.5 * kxy, kyy], axis=-1)
    else:
        k = I.lognormal_kappa(nx, ny, 1.5, 6.0, seed=12)
    f = 1e-6 * rng.standard_normal((ny, nx, 2)) if force else None
    dt = L.LBM_F64 if dtype == "f64" else L.LBM_F32_SHIFTED
    p = L.make_params(nx, ny, 0.9, 0.4, 0.1, 1.0, 1e-6, 0.0, 0, dt, perm_kind, scheme)
    a = L.FineSolver(p, k, f)
    b = L.FineSolver(p, k, f)
    a.step(24)                 # 6 x 4 steps per launch
    a.step(5)                  # 4 + 1
    for _ in range(29):
        b.step(1)
    assert np.array_equal(a.populations().cpu().numpy(), b.populations().cpu().numpy())


@pytest.mark.parametrize("perm_kind,force,gy", [(4, True, 3e-7), (1, True, 3e-7), (4, False, 3e-7),
                                                (1, False, 0.0)])
def test_seven_step_launches_bitwise_other_forms(L, perm_kind, force, gy):
    """FP32 collision arithmetic takes seven steps per launch where the plan
    allows: tensor permeability, a per-cell force field, with and without a
    drive along y (ragged tiles, periodic y), bit for bit as single steps."""
    nx, ny = 150, 45
    rng = np.random.default_rng(5)
    if perm_kind == 4:
        kxx = np.exp(rng.standard_normal((ny, nx)))
        kyy = np.exp(rng.standard_normal((ny, nx)))
        kxy = 0.2 * np.sqrt(kxx * kyy) * rng.uniform(-1, 1, (ny, nx))
        k = np.stack([kxx, kxy, 0.5 * kxy, kyy], axis=-1)
    else:
        k = I.lognormal_kappa(nx, ny, 1.5, 6.0, seed=13)
    f = 1e-6 * rng.standard_normal((ny, nx, 2)) if force else None
    p = L.make_params(nx, ny, 0.9, 0.4, 0.1, 1.0, 1e-6, gy, 0, L.LBM_F32_FAST, perm_kind)
    a = L.FineSolver(p, k, f)
    b = L.FineSolver(p, k, f)
    a.step(20)                 # 7 + 7 + 6
    a.step(14)                 # 7 + 7
    for _ in range(34):
        b.step(1)
    assert np.array_equal(a.populations().cpu().numpy(), b.populations().cpu().numpy())


def test_set_populations_resumes_oracle_state(L):
    nx, ny = 40, 24
    k = I.lognormal_kappa(nx, ny, 1.0, 4.0, seed=8)
    g = (1e-6, 3e-7)
    po = O.Params(nx=nx, ny=ny, tau=0.9, eps=0.4, nu=0.1, walls_y=1)
    r1 = O.run(po, k, g, max_steps=70)
    r2 = O.run(po, k, g, f=r1.f, max_steps=45)
    for dtype, tol in [(L.LBM_F64, 1e-14), (L.LBM_F32_SHIFTED, 1e-9)]:
        p = L.make_params(nx, ny, 0.9, 0.4, 0.1, 1.0, g[0], g[1], 1, dtype)
        s = L.FineSolver(p, k)
        s.set_populations(np.moveaxis(r1.f, 2, 0))
        s.step(45)
        f = s.populations().cpu().numpy()
        assert np.max(np.abs(f - np.moveaxis(r2.f, 2, 0))) < tol


def test_nonfinite_state_is_reported(L):
    nx, ny = 16, 16
    p = L.make_params(nx, ny, 0.8, 0.4, 0.1, 1.0, 1e-6, 0.0, 1, L.LBM_F32_SHIFTED)
    s = L.FineSolver(p, np.ones((ny, nx)))
    f = s.populations().cpu().numpy()
    f[3, 5, 7] = np.nan
    s.set_populations(f)
    st, _, _ = s.step(20, tol=1e-9, check_every=10)
    assert st == L.LBM_ENONFINITE


def test_not_converged_is_reported(L):
    p = L.make_params(32, 32, 0.8, 0.4, 0.1, 1.0, 1e-6, 0.0, 1, L.LBM_F32_SHIFTED)
    s = L.FineSolver(p, np.ones((32, 32)))
    st, done, _ = s.step(30, tol=1e-12, check_every=10)
    assert st == L.LBM_ENOTCONV and done == 30


def test_invalid_permeability_rejected(L):
    p = L.make_params(16, 8, 0.8, 0.4, 0.1, 1.0, 1e-6, 0.0, 1, L.LBM_F32_SHIFTED)
    k = np.ones((8, 16))
    k[2, 3] = -1.0
    with pytest.raises(L.LbmError) as e:
        L.FineSolver(p, k)
    assert e.value.status == L.LBM_EINVAL
    k[2, 3] = np.nan
    with pytest.raises(L.LbmError):
        L.FineSolver(p, k)
    k[2, 3] = np.inf  # no drag: allowed
    L.FineSolver(p, k)


def _window(field, x0, y0, hw, walls_ny):
    """Periodic-in-x window [x0-hw, x0+hw] and rows [y0-hw, y0+hw] clipped to
    the domain (the real walls are kept)."""
    ny, nx = field.shape[:2]
    xs = np.arange(x0 - hw, x0 + hw + 1) % nx
    ylo, yhi = max(0, y0 - hw), min(ny - 1, y0 + hw)
    ys = np.arange(ylo, yhi + 1)
    return np.ascontiguousarray(field[np.ix_(ys, xs)]), hw, y0 - ylo


def test_fine_full_size_sampled(L):
    """The 2048 x 2048 workload (sigma 1.5, correlation length 32, walls in y)
    in the benchmark's launch configuration, 100 steps from rest, compared
    cell by cell with the oracle run on windows around sampled cells. After n
    steps a cell depends only on cells within n lattice steps, so the oracle
    window's own (wrong) edges cannot reach its centre."""
    w = I.workload_fine(seed=1)
    n = 100
    k, g = w["kappa"], (w["g"], 0.0)
    p = L.make_params(2048, 2048, w["tau"], w["eps"], w["nu"], 1.0, g[0], 0.0, 1,
                      L.LBM_F32_SHIFTED)
    s = L.FineSolver(p, k)
    s.step(n)
    u, _ = s.fields()
    u = u.cpu().numpy()
    samples = [(0, 0), (2047, 2047), (5, 1024), (1024, 0), (1024, 2047), (2047, 3), (777, 1333),
               (1500, 101), (0, 100), (1023, 1023)]
    hw = n + 2
    errs = []
    for x0, y0 in samples:
        kw, cx, cy = _window(k, x0, y0, hw, 2048)
        wy, wx = kw.shape
        po = O.Params(nx=wx, ny=wy, tau=w["tau"], eps=w["eps"], nu=w["nu"], walls_y=1)
        r = O.run(po, kw, g, max_steps=n)
        _, ux, uy = O.moments(po, kw, r.f, g)
        scale = max(abs(ux[cy, cx]), 1e-30)
        errs.append(abs(u[0, y0, x0] - ux[cy, cx]) / scale)
        errs.append(abs(u[1, y0, x0] - uy[cy, cx]) / scale)
    assert max(errs) < 1e-5, errs


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_fine_near_maximum_size_sampled(L, dtype):
    """A grid just under the size limit (9 (nx ny + 8192) < 2^31): 16384 x
    14336 = 235M cells, walls in y, 12 steps (FP32: two six-step launches;
    FP64: six two-step launches), checked at sampled cells, including the
    last row and column, against the oracle on windows around them. The
    permeability is a smooth closed-form pattern so the field is cheap to
    build."""
    nx, ny = 16384, 14336
    assert 0.98 * 2 ** 31 < 9 * (nx * ny + 8192) < 2 ** 31
    xs, ys = np.arange(nx), np.arange(ny)

    def kap(yy, xx):
        return np.exp(1.2 * np.sin(2 * np.pi * xx / 97.0)[None, :] *
                      np.cos(2 * np.pi * yy / 131.0)[:, None])

    k = kap(ys, xs)
    g = (1e-6, 0.0)
    pd = L.LBM_F32_SHIFTED if dtype == "f32" else L.LBM_F64
    p = L.make_params(nx, ny, 0.8, 0.4, 0.1, 1.0, g[0], 0.0, 1, pd)
    s = L.FineSolver(p, k)
    del k
    n = 12
    st, done, _ = s.step(n)
    assert st == L.LBM_OK and done == n
    u, _ = s.fields()
    samples = [(0, 0), (nx - 1, ny - 1), (nx - 1, 0), (0, ny - 1), (nx // 2, ny // 2),
               (12345, 14000), (16000, 7)]
    hw = n + 2
    errs = []
    for x0, y0 in samples:
        wxs = np.arange(x0 - hw, x0 + hw + 1) % nx
        ylo, yhi = max(0, y0 - hw), min(ny - 1, y0 + hw)
        wys = np.arange(ylo, yhi + 1)
        kw = np.ascontiguousarray(kap(wys, wxs))
        po = O.Params(nx=len(wxs), ny=len(wys), tau=0.8, eps=0.4, nu=0.1, walls_y=1)
        r = O.run(po, kw, g, max_steps=n)
        _, ux, uy = O.moments(po, kw, r.f, g)
        cx, cy = hw, y0 - ylo
        ug = u[:, y0, x0].cpu().numpy()
        scale = max(abs(ux[cy, cx]), 1e-30)
        errs += [abs(ug[0] - ux[cy, cx]) / scale, abs(ug[1] - uy[cy, cx]) / scale]
    s.close()
    assert max(errs) < (1e-5 if dtype == "f32" else 1e-10), errs


def test_fine_f32_error_over_full_step_count(L):
    """FP32 deviation storage over the 20000 steps of the fine workload, on a
    128 x 128 field of the same statistics (sigma 1.5, correlation 32 scaled
    to 8 for the smaller grid), against the oracle at the same step."""
    nx = ny = 128
    k = I.lognormal_kappa(nx, ny, 1.5, 8.0, seed=2)
    g = (1e-6, 0.0)
    u_o, _, _ = _oracle_run(nx, ny, k, 0.8, 0.4, 0.1, g, 1, 20000)
    u_g, _, _, _ = _gpu_run(L, nx, ny, k, 0.8, 0.4, 0.1, g, 1, 20000, L.LBM_F32_SHIFTED)
    err = np.sqrt(np.sum((u_g - u_o) ** 2) / np.sum(u_o ** 2))
    assert err < 1e-5, err


@pytest.mark.parametrize("scheme", ["shan_chen", "guo"])
def test_paper_sec41_transient_matches_oracle(L, scheme):
    """The Sec. 4.1 setting (100 x 100 periodic, tau 0.53, eps 0.8, block
    field, G = (2, 0) m/s^2 in lattice units) at the paper's transient
    snapshot, step 5000, FP64 populations, both force forms, against the
    oracle's Shan-Chen run: the two forms agree (Sec. 2.1 vs 2.2) and match
    the oracle to rounding."""
    w = I.workload_sec41()
    sc = L.LBM_SCHEME_GUO if scheme == "guo" else L.LBM_SCHEME_SHAN_CHEN
    p = L.make_params(100, 100, w["tau"], w["eps"], w["nu"], 1.0, w["g"][0], w["g"][1], 0, L.LBM_F64,
                      L.LBM_PERM_SCALAR, sc)
    s = L.FineSolver(p, w["kappa"])
    s.step(5000)
    u, rho = s.fields()
    s.close()
    po = O.Params(nx=100, ny=100, tau=w["tau"], eps=w["eps"], nu=w["nu"])
    r = O.run(po, w["kappa"], w["g"], max_steps=5000)
    rho_o, ux, uy = O.moments(po, w["kappa"], r.f, w["g"])
    u = u.cpu().numpy()
    scale = np.abs(ux).max()
    assert np.abs(u[0] - ux).max() < 1e-10 * scale and np.abs(u[1] - uy).max() < 1e-10 * scale
    # the density: 5000 steps of rounding (the GPU keeps deviations from rho0,
    # the oracle full populations) at tau 0.53, where sound waves barely decay
    assert np.abs(rho.cpu().numpy() - rho_o).max() < 5e-12


@pytest.mark.parametrize("tau,bound", [(0.8, 2e-6), (0.53, 1e-5)])
def test_fine_f32_arithmetic_mode(L, tau, bound):
    """LBM_F32_FAST (FP32 state and FP32 collision arithmetic): against the
    oracle over the 20000 steps of the fine workload on a 128 x 128 field of
    the same statistics, in relative L2 of the velocity (measured 1.9e-7 at
    tau 0.8 and 3.8e-6 at tau 0.53; with rounded weights and 2 tau as a
    product of two rounded constants it was 3.5e-6 and 2.6e-5); multi-step
    launches bit-identical to single steps; the Guo form refused."""
    nx = ny = 128
    k = I.lognormal_kappa(nx, ny, 1.5, 8.0, seed=2)
    g = (1e-6, 0.0)
    nu = 0.1 if tau == 0.8 else (tau - 0.5) / 3.0
    u_o, _, _ = _oracle_run(nx, ny, k, tau, 0.4, nu, g, 1, 20000)
    u_g, _, _, _ = _gpu_run(L, nx, ny, k, tau, 0.4, nu, g, 1, 20000, L.LBM_F32_FAST)
    err = np.sqrt(np.sum((u_g - u_o) ** 2) / np.sum(u_o ** 2))
    assert err < bound, err
    p = L.make_params(150, 45, 0.7, 0.4, 0.1, 1.0, 1e-6, 3e-7, 1, L.LBM_F32_FAST)
    kk = I.lognormal_kappa(150, 45, 1.5, 6.0, seed=11)
    a, b = L.FineSolver(p, kk), L.FineSolver(p, kk)
    a.step(29)
    for _ in range(29):
        b.step(1)
    assert np.array_equal(a.populations().cpu().numpy(), b.populations().cpu().numpy())
    with pytest.raises(L.LbmError):   # the Guo form runs in FP64 arithmetic only
        L.FineSolver(L.make_params(16, 16, 0.8, 0.4, 0.1, 1.0, 1e-6, 0.0, 1, L.LBM_F32_FAST,
                                   L.LBM_PERM_SCALAR, L.LBM_SCHEME_GUO), np.ones((16, 16)))


@pytest.mark.parametrize("ratio", [50.0, 100.0])
def test_table3_refined_cell_matches_oracle(L, golden, ratio):
    """Table 3's refined checkerboard (Sec. 4.2.2: squares of 100 points,
    dx 1e-3 m, dt 1e-5 s, tau 1/2): the 200 x 200 periodic cell run to steady
    state with FP64 state against the oracle's exact fixed point (stored by
    tests/golden/make_table3_1000.py) at 1e-7."""
    U = I.LatticeUnits(dx=1e-3, dt=1e-5)
    field = I.checkerboard_field(1000, 10, 1e-12, ratio * 1e-12)[:200, :200].copy()
    g, nu = float(U.force(2.0)), U.nu(2e-6)
    p = L.make_params(200, 200, 0.5, 0.8, nu, 1.0, g, 0.0, 0, L.LBM_F64)
    s = L.FineSolver(p, U.kappa(field))
    st, done, mu = s.step(2_000_000, 1e-12, 10000)
    s.close()
    assert st == L.LBM_OK, (st, done)
    kxx = float(U.kappa_to_phys(nu * mu[0] / g)) / 1e-12
    want = {float(r): float(k) for r, k, _ in golden("table3_1000_oracle.txt")}[ratio]
    assert kxx == pytest.approx(want, rel=1e-7), (kxx, want)


def test_fine_f32_arithmetic_full_workload(L):
    """The benchmarked fine step as it runs there: the 2048^2 workload (sigma
    1.5, correlation 32, walls, tau 0.8) for its 20000 steps in LBM_F32_FAST
    against the FP64-state solver (which matches the oracle to rounding):
    within 1e-5 in relative L2 of the velocity field (measured 2.7e-6), the
    domain-mean velocity within 2e-6 (measured 8.9e-7)."""
    w = I.workload_fine(seed=1)
    k = w["kappa"]
    n = k.shape[0]
    us = {}
    for name, dt in (("f64", L.LBM_F64), ("fast", L.LBM_F32_FAST)):
        s = L.FineSolver(L.make_params(n, n, 0.8, 0.4, 0.1, 1.0, 1e-6, 0.0, 1, dt), k)
        st, done, _ = s.step(20000, 0.0, 0)
        assert st == L.LBM_OK and done == 20000
        u, _ = s.fields()
        us[name] = u.cpu().numpy()
        s.close()
    d = us["fast"] - us["f64"]
    err = np.sqrt(np.sum(d ** 2) / np.sum(us["f64"] ** 2))
    assert err < 1e-5, err
    assert abs(us["fast"][0].mean() / us["f64"][0].mean() - 1) < 2e-6
