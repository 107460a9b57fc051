"""Pins of the D3Q19 oracle (oracle/d3q19.py) against what the lattice's
definition and the mathematics fix, and against the independent
two-dimensional oracle (oracle/lbm_oracle.c) through exact projections."""
import itertools

import numpy as np
import pytest

from oracle import d3q19 as D
from oracle import oracle as O

TAUS = [0.5, 0.53, 0.8, 1.3]


def test_lattice_is_d3q19():
    """The 19 velocities are the origin, the 6 nearest and the 12
    next-nearest neighbours of the cubic lattice; weights 1/3, 1/18, 1/36;
    moments up to fourth order are those of the isotropic Gaussian:
    sum w = 1, sum w e = 0, sum w e_i e_j = c_s^2 delta_ij, odd moments zero,
    sum w e_i e_j e_k e_l = c_s^4 (d_ij d_kl + d_ik d_jl + d_il d_jk)."""
    E, W, OPP = D.lattice()
    want = {v for v in itertools.product((-1, 0, 1), repeat=3) if sum(c * c for c in v) <= 2}
    assert {tuple(int(c) for c in e) for e in E} == want and len(E) == 19
    n2 = (E * E).sum(axis=1)
    assert np.all(W[n2 == 0] == 1 / 3) and np.all(W[n2 == 1] == 1 / 18)
    assert np.all(W[n2 == 2] == 1 / 36)
    assert np.all(E[OPP] == -E)
    cs2 = 1 / 3
    assert W.sum() == pytest.approx(1.0, abs=1e-15)
    d = np.eye(3)
    for i in range(3):
        assert abs((W * E[:, i]).sum()) < 1e-16
        for j in range(3):
            assert (W * E[:, i] * E[:, j]).sum() == pytest.approx(cs2 * d[i, j], abs=1e-15)
            for k in range(3):
                assert abs((W * E[:, i] * E[:, j] * E[:, k]).sum()) < 1e-16
                for m in range(3):
                    iso = cs2 ** 2 * (d[i, j] * d[k, m] + d[i, k] * d[j, m] + d[i, m] * d[j, k])
                    got = (W * E[:, i] * E[:, j] * E[:, k] * E[:, m]).sum()
                    assert got == pytest.approx(iso, abs=1e-15), (i, j, k, m)


@pytest.mark.parametrize("tau", TAUS)
def test_uniform_transient_closed_form(tau):
    """Uniform kappa, periodic, from rest: the state stays uniform and
    j_n = (rho kappa G / nu)(1 - r^n), r = (1 - d)/(1 + d), d = eps nu / (2 kappa)
    (the collision maps j to 2 rho u - j; the lattice does not enter)."""
    kappa, eps, nu, g = 0.7, 0.4, 0.1, 1e-5
    G = (g, 0.5 * g, -0.25 * g)
    p = D.Params3(nx=3, ny=4, nz=5, tau=tau, eps=eps, nu=nu)
    k = np.full((5, 4, 3), kappa)
    d = eps * nu / (2 * kappa)
    r = (1 - d) / (1 + d)
    E, _, _ = D.lattice()
    f = D.rest_state(p)
    for n in range(1, 40):
        f = D.step(p, k, f, G)
        want = kappa * g / nu * (1 - r ** n)
        for c, s in enumerate((1.0, 0.5, -0.25)):
            assert np.allclose((f * E[:, c]).sum(axis=3), s * want, rtol=1e-10, atol=2e-16)
        assert np.allclose(f.sum(axis=3), 1.0, rtol=0, atol=1e-14)


@pytest.mark.parametrize("walls", [0, 1])
def test_mass_conservation(walls):
    rng = np.random.default_rng(5)
    p = D.Params3(nx=5, ny=4, nz=6, tau=0.7, eps=0.5, nu=0.2, walls_z=walls)
    k = np.exp(rng.standard_normal((6, 4, 5)))
    f = D.rest_state(p) * (1 + 1e-3 * rng.standard_normal((6, 4, 5, 19)))
    m0 = f.sum()
    for _ in range(30):
        f = D.step(p, k, f, (1e-4, -2e-4, 3e-4))
        assert abs(f.sum() - m0) < 1e-13 * m0


def _lift(f2, W2, E3, W3, ax):
    """Spread a D2Q9 state over the D3Q19 populations that project onto each
    of its velocities along axis `ax` (1: y, 2: z) in proportion to their
    weights; the 3-D grid is invariant along that axis."""
    ex2, ey2, _, _ = O.lattice()
    keep = [0, 2] if ax == 1 else [0, 1]      # 3-D components that form the 2-D plane
    out = np.zeros(f2.shape[:2] + (19,))
    for a3 in range(19):
        e = E3[a3][keep]
        a2 = int(np.flatnonzero((ex2 == e[0]) & (ey2 == e[1]))[0])
        out[..., a3] = f2[..., a2] * W3[a3] / W2[a2]
    return out


def _project(f3, E3, ax):
    ex2, ey2, _, _ = O.lattice()
    keep = [0, 2] if ax == 1 else [0, 1]
    out = np.zeros(f3.shape[:-1] + (9,))
    for a3 in range(19):
        e = E3[a3][keep]
        a2 = int(np.flatnonzero((ex2 == e[0]) & (ey2 == e[1]))[0])
        out[..., a2] += f3[..., a3]
    return out


@pytest.mark.parametrize("tau", TAUS)
def test_z_invariant_flow_reduces_to_d2q9(tau):
    """A state and field invariant along z, lifted symmetrically in e_z, with
    no force along z: summing the populations over e_z gives exactly the
    D2Q9 step of the two-dimensional oracle (the D3Q19 weights project onto
    the D2Q9 ones and u_z stays zero). Pins the x-y part of the lattice, the
    collision and the streaming against independent C code."""
    rng = np.random.default_rng(9)
    nx, ny, nz = 7, 6, 3
    k2 = np.exp(rng.standard_normal((ny, nx)))
    p2 = O.Params(nx=nx, ny=ny, tau=tau, eps=0.4, nu=0.1)
    p3 = D.Params3(nx=nx, ny=ny, nz=nz, tau=tau, eps=0.4, nu=0.1)
    _, _, W2, _ = O.lattice()
    E3, W3, _ = D.lattice()
    f2 = O.rest_state(p2) * (1 + 1e-3 * rng.standard_normal((ny, nx, 9)))
    f3 = np.broadcast_to(_lift(f2, W2, E3, W3, 2), (nz, ny, nx, 19)).copy()
    k3 = np.broadcast_to(k2, (nz, ny, nx)).copy()
    g = (2e-5, -1e-5)
    for _ in range(25):
        f2 = O.step(p2, k2, f2, g)
        f3 = D.step(p3, k3, f3, (g[0], g[1], 0.0))
    for z in range(nz):
        assert np.max(np.abs(_project(f3[z], E3, 2) - f2)) < 1e-14
    _, u3, _ = D.moments(p3, k3, f3, (g[0], g[1], 0.0))
    _, ux2, uy2 = O.moments(p2, k2, f2, g)
    assert np.allclose(u3[0, 1], ux2, rtol=1e-9, atol=1e-17)
    assert np.allclose(u3[1, 1], uy2, rtol=1e-9, atol=1e-17)
    assert np.max(np.abs(u3[2])) < 1e-18


@pytest.mark.parametrize("tau", [0.5, 0.8])
def test_y_invariant_channel_with_z_walls_reduces_to_d2q9(tau):
    """The x-z plane: a field and state invariant along y, bounce-back walls
    in z, projected over e_y, against the two-dimensional oracle with walls
    in y (its y is the 3-D z). Pins the z part of the lattice and the walls."""
    rng = np.random.default_rng(13)
    nx, ny, nz = 6, 2, 7
    k2 = np.exp(rng.standard_normal((nz, nx)))
    p2 = O.Params(nx=nx, ny=nz, tau=tau, eps=0.6, nu=0.2, walls_y=1)
    p3 = D.Params3(nx=nx, ny=ny, nz=nz, tau=tau, eps=0.6, nu=0.2, walls_z=1)
    _, _, W2, _ = O.lattice()
    E3, W3, _ = D.lattice()
    f2 = O.rest_state(p2) * (1 + 1e-3 * rng.standard_normal((nz, nx, 9)))
    lifted = _lift(f2, W2, E3, W3, 1)                       # [nz, nx, 19]
    f3 = np.ascontiguousarray(np.broadcast_to(lifted[:, None], (nz, ny, nx, 19)))
    k3 = np.ascontiguousarray(np.broadcast_to(k2[:, None, :], (nz, ny, nx)))
    g = (3e-5, 1e-5)                                        # (x, z)
    for _ in range(25):
        f2 = O.step(p2, k2, f2, g)
        f3 = D.step(p3, k3, f3, (g[0], 0.0, g[1]))
    for y in range(ny):
        assert np.max(np.abs(_project(f3[:, y], E3, 1) - f2)) < 1e-14


def test_axis_permutation_symmetry():
    """A fully three-dimensional periodic field: relabelling the axes of the
    field and of the drive relabels the velocity (the lattice is invariant
    under the permutations of the axes)."""
    rng = np.random.default_rng(17)
    k = np.exp(rng.standard_normal((4, 5, 6)))       # [z, y, x]
    p = D.Params3(nx=6, ny=5, nz=4, tau=0.8, eps=0.4, nu=0.1)
    G = (1e-5, 3e-6, -2e-6)
    f = D.run(p, k, G, max_steps=60)[0]
    _, u, _ = D.moments(p, k, f, G)
    # swap x and z: new array axes [x, y, z] -> field k' [z'=x, y, x'=z]
    kt = np.ascontiguousarray(np.transpose(k, (2, 1, 0)))
    pt = D.Params3(nx=4, ny=5, nz=6, tau=0.8, eps=0.4, nu=0.1)
    Gt = (G[2], G[1], G[0])
    ft = D.run(pt, kt, Gt, max_steps=60)[0]
    _, ut, _ = D.moments(pt, kt, ft, Gt)
    assert np.allclose(ut[0], np.transpose(u[2], (2, 1, 0)), rtol=1e-11, atol=1e-20)
    assert np.allclose(ut[2], np.transpose(u[0], (2, 1, 0)), rtol=1e-11, atol=1e-20)
    assert np.allclose(ut[1], np.transpose(u[1], (2, 1, 0)), rtol=1e-11, atol=1e-20)
    # swap y and z
    ky = np.ascontiguousarray(np.transpose(k, (1, 0, 2)))
    py = D.Params3(nx=6, ny=4, nz=5, tau=0.8, eps=0.4, nu=0.1)
    Gy = (G[0], G[2], G[1])
    fy = D.run(py, ky, Gy, max_steps=60)[0]
    _, uy, _ = D.moments(py, ky, fy, Gy)
    assert np.allclose(uy[1], np.transpose(u[2], (1, 0, 2)), rtol=1e-11, atol=1e-20)
    assert np.allclose(uy[2], np.transpose(u[1], (1, 0, 2)), rtol=1e-11, atol=1e-20)


def test_layered_means_along_z():
    """Layers along z (kappa a function of z only, periodic): driven along
    the layers at tau 1/2 Darcy's law is local and the mean velocity gives
    the arithmetic mean of kappa; driven across them, the flux is the same in
    every layer and the harmonic mean results (Tables 1 and 2 in 3-D)."""
    kz = np.roll(np.repeat([0.1, 0.7, 0.3, 2.0], 6), 3)
    p = D.Params3(nx=1, ny=1, nz=24, tau=0.5, eps=0.4, nu=0.1)
    k = kz[:, None, None].copy()
    g = 1e-6
    f, n, ok = D.run(p, k, (0.0, g, 0.0), max_steps=100000, check_every=500, tol=1e-11)
    assert ok
    kyy = 0.1 * D.mean_velocity(p, k, f, (0.0, g, 0.0))[1] / g
    assert kyy == pytest.approx(kz.mean(), rel=1e-8)
    p8 = D.Params3(nx=1, ny=1, nz=24, tau=0.8, eps=0.4, nu=0.1)
    f, n, ok = D.run(p8, k, (0.0, 0.0, g), max_steps=100000, check_every=500, tol=1e-11)
    assert ok
    kzz = 0.1 * D.mean_velocity(p8, k, f, (0.0, 0.0, g))[2] / g
    assert kzz == pytest.approx(1.0 / np.mean(1.0 / kz), rel=1e-6)


def test_step_at_matches_full_step():
    """The sampled step (one cell at a time from the definition of the pull)
    equals the full step at those cells, with walls."""
    rng = np.random.default_rng(23)
    p = D.Params3(nx=5, ny=4, nz=6, tau=0.9, eps=0.5, nu=0.2, walls_z=1)
    k = np.exp(rng.standard_normal((6, 4, 5)))
    f = D.rest_state(p) * (1 + 1e-3 * rng.standard_normal((6, 4, 5, 19)))
    G = (1e-4, 0.0, -1e-4)
    full = D.step(p, k, f, G)
    cells = np.array([[0, 0, 0], [4, 3, 5], [2, 1, 3], [0, 3, 5], [4, 0, 0]])
    got = D.step_at(p, k, f, cells, G)
    for i, (x, y, z) in enumerate(cells):
        assert np.allclose(got[i], full[z, y, x], rtol=0, atol=1e-16)
