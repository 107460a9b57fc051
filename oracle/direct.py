"""Exact steady state of the oracle's time step by a sparse direct solve.

TEST INFRASTRUCTURE ONLY (used by the tests to pin the time-stepping oracle).

With the linear equilibrium of Eq. feq, the drag of Eq. f_m-depends-on-u and
the body force entering as rho G, one time step of Sec. 2.2 is a linear,
homogeneous map f -> T f: rho u and rho u_eq are linear in f, and streaming
(periodic or bounce-back) is a permutation. A steady state is a fixed point
T f = f; mass conservation makes the columns of T - I sum to zero, so one
equation is replaced by the total-mass condition sum f = N rho0.

T is read off the oracle's own step function by probing (nine probes, one
per population). The solve then gives the fixed point to which time stepping
converges, independent of how long a run would take.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import oracle as O


def _probe(p: O.Params, perm, g, force):
    """Columns of the one-step map, read off the oracle's step by probing.

    Output entry (cell d, population a) comes from exactly one source cell:
    d - e_a, or d itself after a bounce-back at a wall. So adding 1 to
    population b of every cell at once changes each output entry by the single
    matrix element that links it to its own source; nine probes (b = 0..8)
    recover the whole matrix. Returns (rows, cols, vals) of T - applied to the
    perturbation only, i.e. the linear part."""
    ex, ey, _, _ = O.lattice()
    nx, ny = p.nx, p.ny
    n = nx * ny
    f0 = O.rest_state(p)
    base = O.step(p, perm, f0, g, force)
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    src = np.empty((ny, nx, 9), np.int64)
    for a in range(9):
        sy = yy - ey[a]
        sx = (xx - ex[a]) % nx
        if p.walls_y:
            out_of = (sy < 0) | (sy >= ny)
            sy = np.where(out_of, yy, sy % ny)
            sx = np.where(out_of, xx, sx)
        else:
            sy = sy % ny
        src[:, :, a] = sy * nx + sx
    rows = np.arange(n * 9)
    R, C, V = [], [], []
    for b in range(9):
        probe = f0.copy()
        probe[:, :, b] += 1.0
        d = (O.step(p, perm, probe, g, force) - base).ravel()
        R.append(rows); C.append(src.ravel() * 9 + b); V.append(d)
    return np.concatenate(R), np.concatenate(C), np.concatenate(V), 9 * n


def _unit_force(p: O.Params, g, force):
    """Split the drive into a scale s and a unit-size pattern."""
    if force is not None:
        force = np.ascontiguousarray(force, dtype=np.float64)
        s = float(np.abs(force).max())
        return s, (0.0, 0.0), (force / s if s > 0 else force)
    s = float(np.hypot(g[0], g[1]))
    return s, ((g[0] / s, g[1] / s) if s > 0 else (0.0, 0.0)), None


def transition_parts(p: O.Params, perm, g=(0.0, 0.0), force=None):
    """(T0, B, s): the step is f -> T0 f + s B f, where T0 is the step without
    drive, B its part proportional to the (unit) drive and s the drive size.
    The step is affine in G at fixed f, so B is read exactly from a probe with
    a unit-size drive; keeping s B apart from T0 avoids burying the tiny drive
    terms in the O(1) entries of T0."""
    s, gu, fu = _unit_force(p, g, force)
    r0, c0, v0, m = _probe(p, perm, (0.0, 0.0), None)
    r1, c1, v1, _ = _probe(p, perm, gu, fu)
    assert np.array_equal(r0, r1) and np.array_equal(c0, c1)
    T0 = sp.csr_matrix((v0, (r0, c0)), shape=(m, m))
    B = sp.csr_matrix((v1 - v0, (r0, c0)), shape=(m, m))
    return T0, B, s


def transition_matrix(p: O.Params, perm, g=(0.0, 0.0), force=None) -> sp.csr_matrix:
    """Sparse T with f_next.ravel() = T @ f.ravel() for one oracle step."""
    T0, B, s = transition_parts(p, perm, g, force)
    return (T0 + s * B).tocsr()


def steady_state(p: O.Params, perm, g=(0.0, 0.0), force=None) -> np.ndarray:
    """Fixed point of the step with total mass N rho0; returns [ny, nx, 9].

    Solved for the deviation d = f - f_rest from the rest state, which is a
    fixed point of the undriven step: (T0 + s B - I) d = -s B f_rest with
    sum d = 0 in place of the first (redundant) equation."""
    T0, B, s = transition_parts(p, perm, g, force)
    m = T0.shape[0]
    f_rest = O.rest_state(p).ravel()
    A = (T0 + s * B - sp.identity(m, format="csr")).tolil()
    A[0, :] = np.ones(m)
    rhs = -s * (B @ f_rest)
    rhs[0] = 0.0
    d = spla.spsolve(A.tocsc(), rhs)
    return (f_rest + d).reshape(p.ny, p.nx, 9)


def steady_mean_velocity(p: O.Params, perm, g=(0.0, 0.0), force=None,
                         margin: int = 0) -> np.ndarray:
    """Mean flow velocity of the steady state over the whole domain or, with
    margin m > 0, over the inner window [m, nx - m) x [m, ny - m) only
    (oversampling: the cells next to the artificial periodic boundary are
    left out of the average)."""
    f = steady_state(p, perm, g, force)
    if margin == 0:
        return O.mean_velocity(p, perm, f, g, force)
    _, ux, uy = O.moments(p, perm, f, g, force)
    w = (slice(margin, p.ny - margin), slice(margin, p.nx - margin))
    return np.array([ux[w].mean(), uy[w].mean()])


def keff_direct(kappa_patch, tau: float, eps: float, nu: float, g: float = 1e-6,
                margin: int = 0) -> np.ndarray:
    """Eq. tensor-kappa from the exact steady states of the two periodic local
    runs; returns [kxx, kxy, kyx, kyy]. margin > 0 averages the velocity over
    the inner window only (see steady_mean_velocity)."""
    k = np.ascontiguousarray(kappa_patch, dtype=np.float64)
    ny, nx = k.shape
    if margin < 0 or nx - 2 * margin < 1 or ny - 2 * margin < 1:
        raise ValueError("margin leaves no inner window")
    p = O.Params(nx=nx, ny=ny, tau=tau, eps=eps, nu=nu)
    u1 = steady_mean_velocity(p, k, (g, 0.0), margin=margin)
    u2 = steady_mean_velocity(p, k, (0.0, g), margin=margin)
    return np.array([nu * u1[0] / g, nu * u2[0] / g, nu * u1[1] / g, nu * u2[1] / g])
