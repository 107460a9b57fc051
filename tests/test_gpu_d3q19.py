"""GPU parity of the D3Q19 fine-grid step (lbm3d_*) against the FP64 D3Q19
oracle, through the C ABI.

Tolerances: FP64 populations agree with the oracle to rounding (1e-15
absolute; the velocity, a difference of O(0.1) populations divided by rho,
within 1e-10 of its largest value of ~1e-4); FP32 populations (deviations
from rest, FP64 arithmetic) keep the velocity within 1e-5 of its largest
value.
"""
import numpy as np
import pytest

from oracle import d3q19 as D
from paper_1312_0195_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def L():
    from paper_1312_0195_amd import lbm
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lbm.lib()
    return lbm


def _solver(L, kappa, tau, g, walls, dtype, eps=0.4, nu=0.1):
    nz, ny, nx = kappa.shape
    p = L.make_params3(nx, ny, nz, tau, eps, nu, 1.0, g, walls, dtype)
    return L.Solver3D(p, kappa), D.Params3(nx=nx, ny=ny, nz=nz, tau=tau, eps=eps, nu=nu,
                                           walls_z=walls)


def _oracle_f(f_dev):
    """GPU layout [19][nz][ny][nx] -> oracle layout [nz][ny][nx][19]."""
    return np.ascontiguousarray(np.moveaxis(f_dev.cpu().numpy(), 0, -1))


# ragged in x (a 64-wide tile plus a tail) and in y (tiles of 4 rows)
SHAPES = [(70, 9, 11), (5, 3, 4), (64, 4, 2)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("walls", [0, 1])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_steps_from_rest_match_oracle(L, shape, walls, dtype):
    nx, ny, nz = shape
    kappa = I.lognormal_kappa3(nx, ny, nz, 1.0, 3.0, seed=5)
    g = (1e-5, -4e-6, 2.5e-6)
    pd = L.LBM_F64 if dtype == "f64" else L.LBM_F32_SHIFTED
    s, p = _solver(L, kappa, 0.8, g, walls, pd)
    steps = 24
    st, done, mu = s.step(steps)
    assert st == L.LBM_OK and done == steps
    f = D.rest_state(p)
    for _ in range(steps):
        f = D.step(p, kappa, f, g)
    _, uo, _ = D.moments(p, kappa, f, g)
    u, rho = s.fields()
    u = u.cpu().numpy()
    scale = np.abs(uo).max()
    tol = 1e-10 if dtype == "f64" else 1e-5
    assert np.abs(u - uo).max() / scale < tol
    assert np.allclose(mu, uo.reshape(3, -1).mean(axis=1), rtol=0, atol=tol * scale)
    ro, _, _ = D.moments(p, kappa, f, g)
    assert np.abs(rho.cpu().numpy() - ro).max() < (1e-14 if dtype == "f64" else 1e-9)
    if dtype == "f64":
        assert np.abs(_oracle_f(s.populations()) - f).max() < 1e-15
    s.close()


@pytest.mark.parametrize("shape", [(70, 9, 70), (40, 17, 33), (5, 3, 1), (1, 1, 3), (33, 8, 2),
                                   (64, 16, 32)])
@pytest.mark.parametrize("walls", [0, 1])
def test_two_step_launches_match_single_steps_bitwise(L, shape, walls):
    """FP32 state: the two-steps-per-launch kernel (z-marching through a ring
    of planes in LDS; chunks of 32 planes, halo tiles that wrap several times
    on narrow grids) leaves exactly the state of single-step launches."""
    nx, ny, nz = shape
    kappa = I.lognormal_kappa3(nx, ny, nz, 1.0, 2.0, seed=8)
    g = (1e-5, 3e-6, -2e-6)
    a, _ = _solver(L, kappa, 0.7, g, walls, L.LBM_F32_SHIFTED)
    b, _ = _solver(L, kappa, 0.7, g, walls, L.LBM_F32_SHIFTED)
    a.step(10)                       # five two-step launches
    for _ in range(10):
        b.step(1)                    # ten single-step launches
    fa, fb = a.populations().cpu().numpy(), b.populations().cpu().numpy()
    assert np.array_equal(fa, fb)
    assert np.abs(fa - D.rest_state(D.Params3(nx=nx, ny=ny, nz=nz, tau=0.7, eps=0.4, nu=0.1))
                  .transpose(3, 0, 1, 2)).max() > 0
    a.close()
    b.close()


@pytest.mark.parametrize("walls", [0, 1])
@pytest.mark.parametrize("tau", [0.5, 0.53, 1.3])
def test_random_state_one_step_f64(L, walls, tau):
    """From a random perturbed state (lbm3d_set_populations): one step equals
    the oracle's step, population by population."""
    nx, ny, nz = 67, 6, 7
    rng = np.random.default_rng(11)
    kappa = np.exp(rng.standard_normal((nz, ny, nx)))
    g = (2e-5, 1e-5, -3e-5)
    s, p = _solver(L, kappa, tau, g, walls, L.LBM_F64)
    f0 = D.rest_state(p) * (1 + 1e-3 * rng.standard_normal((nz, ny, nx, 19)))
    s.set_populations(torch.as_tensor(np.ascontiguousarray(np.moveaxis(f0, -1, 0))))
    assert np.abs(_oracle_f(s.populations()) - f0).max() == 0.0
    s.step(1)
    f1 = D.step(p, kappa, f0, g)
    assert np.abs(_oracle_f(s.populations()) - f1).max() < 2e-16 * 8
    s.step(3)
    for _ in range(3):
        f1 = D.step(p, kappa, f1, g)
    assert np.abs(_oracle_f(s.populations()) - f1).max() < 2e-16 * 32
    s.close()


def test_mass_conservation_and_uniform_closed_form(L):
    """Walls and periodic z: total mass is conserved to rounding; a uniform
    field follows the closed-form transient j_n = (kappa G / nu)(1 - r^n)."""
    rng = np.random.default_rng(3)
    nx, ny, nz = 40, 8, 12
    kappa = np.exp(rng.standard_normal((nz, ny, nx)))
    s, p = _solver(L, kappa, 0.7, (1e-4, 0.0, -1e-4), 1, L.LBM_F64)
    f0 = D.rest_state(p) * (1 + 1e-3 * rng.standard_normal((nz, ny, nx, 19)))
    s.set_populations(torch.as_tensor(np.ascontiguousarray(np.moveaxis(f0, -1, 0))))
    m0 = f0.sum()
    s.step(50)
    assert abs(s.populations().sum().item() - m0) < 1e-12 * m0
    s.close()
    kap, eps, nu, gx = 0.7, 0.4, 0.1, 1e-5
    s, p = _solver(L, np.full((nz, ny, nx), kap), 0.9, (gx, 0.5 * gx, -gx), 0, L.LBM_F32_SHIFTED)
    d = eps * nu / (2 * kap)
    r = (1 - d) / (1 + d)
    for n in (1, 7, 40):
        s.step(n - s.steps_total)
        f = s.populations().cpu().numpy()
        E, _, _ = D.lattice()
        jx = np.tensordot(E[:, 0].astype(float), f, axes=(0, 0))
        want = kap * gx / nu * (1 - r ** n)
        assert np.allclose(jx, want, rtol=1e-5)
    s.close()


def test_rejects_bad_kappa(L):
    k = np.ones((4, 4, 64))
    k[2, 1, 7] = 0.0
    with pytest.raises(L.LbmError):
        _solver(L, k, 0.8, (1e-6, 0, 0), 0, L.LBM_F32_SHIFTED)


class _Cells:
    """f[z, y, x] / kappa[z, y, x] lookups served from gathered cells."""

    def __init__(self, table):
        self.t = table

    def __getitem__(self, key):
        return self.t[tuple(int(v) for v in key)]


def test_full_size_sampled_cells(L):
    """The D3Q19 workload at full size (256^3, sigma 1.5, walls in z) in the
    launch configuration the benchmark times: 12 steps from rest in two-step
    launches equal 12 single-step launches bitwise; then one more step on the
    GPU is checked at sampled cells (including the walls and the periodic
    faces) against the oracle's step of the same state."""
    w = I.workload_d3q19()
    kappa = w["kappa"]
    nz, ny, nx = kappa.shape
    s, p = _solver(L, kappa, w["tau"], w["g"], w["walls_z"], L.LBM_F32_SHIFTED, w["eps"], w["nu"])
    s.step(12)                                  # six two-step launches (runs of 128 planes)
    f_t = s.populations()                       # FP64 [19][nz][ny][nx] on the device
    ref, _ = _solver(L, kappa, w["tau"], w["g"], w["walls_z"], L.LBM_F32_SHIFTED, w["eps"], w["nu"])
    for _ in range(12):
        ref.step(1)                             # single-step launches
    assert torch.equal(ref.populations(), f_t)
    ref.close()
    rng = np.random.default_rng(2)
    cells = np.stack([rng.integers(0, nx, 40), rng.integers(0, ny, 40), rng.integers(0, nz, 40)], 1)
    cells = np.concatenate([cells, [[0, 0, 0], [nx - 1, ny - 1, nz - 1], [5, 0, nz - 1],
                                    [nx - 1, 3, 0]]])
    need = set()
    for x, y, z in cells:
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    need.add(((z + dz) % nz, (y + dy) % ny, (x + dx) % nx))
    need = sorted(need)
    idx = torch.as_tensor(np.array(need), device=f_t.device)
    vals = f_t[:, idx[:, 0], idx[:, 1], idx[:, 2]].T.cpu().numpy()
    ftab = {c: vals[i] for i, c in enumerate(need)}
    ktab = {c: kappa[c] for c in need}
    want = D.step_at(p, _Cells(ktab), _Cells(ftab), cells, w["g"])
    s.step(1)
    f_n = s.populations()
    ci = torch.as_tensor(cells, device=f_n.device)
    got = f_n[:, ci[:, 2], ci[:, 1], ci[:, 0]].T.cpu().numpy()
    # FP32 storage of the deviations: compare the deviations from rest
    _, W, _ = D.lattice()
    dev_w = want - W
    err = np.abs((got - W) - dev_w).max() / np.abs(dev_w).max()
    assert err < 1e-6, err
    s.close()


def test_large_grid_two_step_equals_single_steps_and_oracle(L):
    """A 640 x 640 x 600 grid (246M cells, 37 GB of FP32 state per solver,
    walls in z): six steps in two-step launches equal six single-step
    launches bitwise, and sampled cells (corners, walls, far end of the index
    range) match the oracle run on windows around them (after n steps a cell
    depends only on cells within n lattice steps). The permeability is a
    smooth closed-form pattern built on the device."""
    nx, ny, nz = 640, 640, 600
    g = (1e-6, 2e-7, 0.0)

    def kap_np(z, y, x):
        return np.exp(1.2 * np.sin(2 * np.pi * x / 97.0)[None, None, :] *
                      np.cos(2 * np.pi * y / 131.0)[None, :, None] *
                      np.sin(2 * np.pi * z / 89.0 + 0.3)[:, None, None])

    dev = torch.device("cuda")
    xt = torch.arange(nx, device=dev, dtype=torch.float64)
    yt = torch.arange(ny, device=dev, dtype=torch.float64)
    zt = torch.arange(nz, device=dev, dtype=torch.float64)
    kt = torch.exp(1.2 * torch.sin(2 * np.pi * xt / 97.0)[None, None, :] *
                   torch.cos(2 * np.pi * yt / 131.0)[None, :, None] *
                   torch.sin(2 * np.pi * zt / 89.0 + 0.3)[:, None, None]).contiguous()
    p = L.make_params3(nx, ny, nz, 0.8, 0.4, 0.1, 1.0, g, 1, L.LBM_F32_SHIFTED)
    a = L.Solver3D(p, kt)
    b = L.Solver3D(p, kt)
    del kt
    n = 6
    a.step(n)
    for _ in range(n):
        b.step(1)
    ua, _ = a.fields()
    a.close()
    ub, _ = b.fields()
    b.close()
    assert torch.equal(ua, ub)
    del ub
    samples = [(0, 0, 0), (nx - 1, ny - 1, nz - 1), (nx - 1, 0, nz - 1), (320, 321, 300),
               (5, ny - 2, 1), (600, 17, 598)]
    hw = n + 1
    pd = D.Params3
    for x0, y0, z0 in samples:
        xs = np.arange(x0 - hw, x0 + hw + 1) % nx
        ys = np.arange(y0 - hw, y0 + hw + 1) % ny
        zlo, zhi = max(0, z0 - hw), min(nz - 1, z0 + hw)
        zs = np.arange(zlo, zhi + 1)
        kw = np.ascontiguousarray(kap_np(zs, ys, xs))
        po = pd(nx=len(xs), ny=len(ys), nz=len(zs), tau=0.8, eps=0.4, nu=0.1, walls_z=1)
        f = D.run(po, kw, g, max_steps=n)[0]
        _, uo, _ = D.moments(po, kw, f, g)
        want = uo[:, z0 - zlo, hw, hw]
        got = ua[:, z0, y0, x0].cpu().numpy()
        scale = np.abs(want).max()
        assert np.abs(got - want).max() / scale < 1e-5, (x0, y0, z0, got, want)
