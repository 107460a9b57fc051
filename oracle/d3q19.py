"""Plain FP64 CPU reference of the method on the D3Q19 lattice.

TEST INFRASTRUCTURE ONLY: the checker of the HIP path's three-dimensional
step. Only the test suite, the smoke check and the benchmark's CPU-baseline
leg may use it. It shares no code with the GPU library.

Sec. 2 states that three-dimensional problems use the D3Q19 lattice (Qian,
d'Humieres and Lallemand, 1992) with its own velocities and weights and
otherwise unchanged algorithms. So this module is the Shan-Chen form of
Sec. 2.2 (Eqs. feq, explicit-u-in-Guo, final-ueq-of-S-C, f-evolution-of-S-C)
with three velocity components:

    rho = sum_a f_a,   j = sum_a e_a f_a
    u    = (j + eps rho G / 2) / (rho (1 + eps nu / (2 kappa)))
    u_eq = 2 tau u + (1 - 2 tau) j / rho
    f_eq = w_a rho (1 + e_a . u_eq / c_s^2),   c_s^2 = 1/3
    f_a(x + e_a, t + 1) = f_a + (f_eq - f_a) / tau

in lattice units, with a scalar permeability kappa per cell and a uniform
body force G. The lattice is periodic in x and y; in z it is periodic or has
halfway bounce-back walls half a cell outside the first and last planes (a
population that would leave returns to its cell as the opposite one), the
three-dimensional counterpart of the walls of the two-dimensional oracle.

Arrays are cell-major, f[z, y, x, a]. The step is written as the evolution
equation states it: collide every cell, then move each post-collision value
to x + e_a (np.roll per population).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

CS2 = 1.0 / 3.0


def lattice():
    """(E [19, 3] int, W [19], OPP [19]): rest vector, the six vectors along
    the axes (+x, -x, +y, -y, +z, -z), then the twelve diagonals of the
    coordinate planes (xy, xz, yz), each as +/+, -/-, +/-, -/+."""
    E = [(0, 0, 0),
         (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
         (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
         (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
         (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]
    E = np.array(E, dtype=np.int64)
    n2 = (E * E).sum(axis=1)
    W = np.where(n2 == 0, 1.0 / 3.0, np.where(n2 == 1, 1.0 / 18.0, 1.0 / 36.0))
    OPP = np.array([int(np.flatnonzero((E == -e).all(axis=1))[0]) for e in E])
    return E, W, OPP


@dataclass
class Params3:
    nx: int
    ny: int
    nz: int
    tau: float
    eps: float
    nu: float
    rho0: float = 1.0
    walls_z: int = 0


def rest_state(p: Params3) -> np.ndarray:
    _, W, _ = lattice()
    return np.broadcast_to(W * p.rho0, (p.nz, p.ny, p.nx, 19)).copy()


def moments(p: Params3, kappa, f, g=(0.0, 0.0, 0.0)):
    """(rho [nz, ny, nx], u [3, nz, ny, nx], j [3, nz, ny, nx]): density,
    flow velocity (Eq. explicit-u-in-Guo with three components) and
    momentum of the pre-collision state f."""
    E, _, _ = lattice()
    f = np.asarray(f, dtype=np.float64)
    kappa = np.asarray(kappa, dtype=np.float64)
    rho = f.sum(axis=3)
    j = np.stack([(f * E[:, d]).sum(axis=3) for d in range(3)])
    denom = rho * (1.0 + p.eps * p.nu / (2.0 * kappa))
    u = np.stack([(j[d] + 0.5 * p.eps * rho * g[d]) / denom for d in range(3)])
    return rho, u, j


def collide(p: Params3, kappa, f, g=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Post-collision populations of every cell (Eq. f-evolution-of-S-C)."""
    E, W, _ = lattice()
    rho, u, j = moments(p, kappa, f, g)
    ueq = 2.0 * p.tau * u + (1.0 - 2.0 * p.tau) * j / rho
    eu = np.einsum("ad,dzyx->zyxa", E.astype(np.float64), ueq)
    feq = W * rho[..., None] * (1.0 + eu / CS2)
    return f + (feq - f) / p.tau


def stream(p: Params3, fs) -> np.ndarray:
    """Move every post-collision f_a(x) to x + e_a."""
    E, _, OPP = lattice()
    out = np.empty_like(fs)
    for a in range(19):
        ex, ey, ez = (int(v) for v in E[a])
        out[..., a] = np.roll(fs[..., a], shift=(ez, ey, ex), axis=(0, 1, 2))
        if p.walls_z and ez != 0:
            # the plane that np.roll filled from across the domain instead gets
            # the population that left through the wall next to it, reversed
            zin = 0 if ez > 0 else p.nz - 1
            out[zin, :, :, a] = fs[zin, :, :, OPP[a]]
    return out


def step(p: Params3, kappa, f, g=(0.0, 0.0, 0.0)) -> np.ndarray:
    return stream(p, collide(p, kappa, f, g))


def mean_velocity(p: Params3, kappa, f, g=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Volume average of the flow velocity (Sec. 3)."""
    _, u, _ = moments(p, kappa, f, g)
    return u.reshape(3, -1).mean(axis=1)


def run(p: Params3, kappa, g, f=None, max_steps=1000, check_every=0, tol=0.0):
    """Run from f (rest state if None) for at most max_steps steps, stopping
    once the mean velocity changes by <= tol times its norm between checks
    taken every check_every steps. Returns (f, steps, converged)."""
    f = rest_state(p) if f is None else np.array(f, dtype=np.float64, copy=True)
    prev = None
    for n in range(1, max_steps + 1):
        f = step(p, kappa, f, g)
        if check_every and n % check_every == 0:
            mu = mean_velocity(p, kappa, f, g)
            if not np.isfinite(mu).all():
                return f, n, False
            if prev is not None and tol > 0 and \
                    np.linalg.norm(mu - prev) <= tol * np.linalg.norm(mu):
                return f, n, True
            prev = mu
    return f, max_steps, False


def step_at(p: Params3, kappa, f, cells, g=(0.0, 0.0, 0.0)) -> np.ndarray:
    """The populations that one step gives at the listed cells only
    ([n, 3] integer (x, y, z)): population a at x comes from the collision at
    x - e_a (or, across a wall, from population opp(a) of x itself). For
    sampled checks of grids too large to step whole; [n, 19]."""
    E, _, OPP = lattice()
    cells = np.asarray(cells, dtype=np.int64)
    out = np.empty((len(cells), 19))
    # f and kappa are only indexed cell by cell ([z, y, x]), so any object
    # with that lookup serves (e.g. the gathered neighbourhoods of samples)
    for i, (x, y, z) in enumerate(cells):
        for a in range(19):
            sx, sy, sz = x - E[a, 0], y - E[a, 1], z - E[a, 2]
            pop = a
            if p.walls_z and not (0 <= sz < p.nz):
                sx, sy, sz, pop = x, y, z, OPP[a]
            sx, sy, sz = sx % p.nx, sy % p.ny, sz % p.nz
            cell_f = np.asarray(f[sz, sy, sx], dtype=np.float64).reshape(1, 1, 1, 19)
            cell_k = np.full((1, 1, 1), float(kappa[sz, sy, sx]))
            out[i, a] = collide(p, cell_k, cell_f, g)[0, 0, 0, pop]
    return out
