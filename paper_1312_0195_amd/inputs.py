"""Seeded synthetic inputs for the upscaled Brinkman LBM.

This module only builds inputs: permeability fields, patch lists and unit
conversions. It holds none of the lattice Boltzmann arithmetic, so both the
HIP path and the CPU oracle may take their inputs from here.

Permeability fields follow the paper where it defines them
(Sec. 4.1 block field, Eq. kappa-forcemodel; Sec. 4.2 layered and checkerboard
fields; Sec. 4.3 five-block field, Eq. finekappa-fiveblock, and its coarse
counterpart, Eq. coarsekappa-fiveblock). The paper does not say how a random
heterogeneous field is generated, so the log-normal fields here are our own
recipe: a periodic Gaussian random field Z with Gaussian covariance
C(r) = sigma^2 exp(-r^2 / (2 l^2)), made by filtering white noise in Fourier
space, rescaled to sample mean 0 and sample standard deviation sigma, and
K = exp(Z).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# ----------------------------------------------------------------------------
# Random fields
# ----------------------------------------------------------------------------


def grf_logk(nx: int, ny: int, sigma: float, corr_len: float, seed: int) -> np.ndarray:
    """Periodic Gaussian random field Z of shape [ny, nx] (x fastest), FP64.

    White noise W ~ N(0, 1) from numpy's PCG64 stream ``default_rng(seed)`` is
    filtered by sqrt(S(k)) with S(k) proportional to exp(-l^2 |k|^2 / 2), the
    spectrum of a Gaussian covariance of correlation length ``corr_len``
    cells. The result is rescaled to sample mean 0 and sample std ``sigma``.
    """
    if nx <= 0 or ny <= 0:
        raise ValueError("grid sides must be positive")
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((ny, nx))
    kx = 2.0 * np.pi * np.fft.fftfreq(nx)
    ky = 2.0 * np.pi * np.fft.fftfreq(ny)
    k2 = ky[:, None] ** 2 + kx[None, :] ** 2
    filt = np.exp(-0.25 * corr_len * corr_len * k2)  # sqrt of exp(-l^2 k^2 / 2)
    z = np.fft.ifft2(np.fft.fft2(w) * filt).real
    z -= z.mean()
    sd = z.std()
    if sd > 0:
        z *= sigma / sd
    return np.ascontiguousarray(z)


def grf_logk3(nx: int, ny: int, nz: int, sigma: float, corr_len: float, seed: int) -> np.ndarray:
    """Three-dimensional counterpart of :func:`grf_logk`, shape [nz, ny, nx]
    (x fastest), same recipe (FP32 white noise and transforms to keep the
    memory of large grids modest; the result is FP64)."""
    if nx <= 0 or ny <= 0 or nz <= 0:
        raise ValueError("grid sides must be positive")
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((nz, ny, nx), dtype=np.float32)
    kz = 2.0 * np.pi * np.fft.fftfreq(nz)
    ky = 2.0 * np.pi * np.fft.fftfreq(ny)
    kx = 2.0 * np.pi * np.fft.rfftfreq(nx)                # real transform: x halved
    wf = np.fft.rfftn(w, axes=(0, 1, 2))
    k2 = kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2
    wf *= np.exp(-0.25 * corr_len * corr_len * k2).astype(np.float32)
    del k2
    z = np.fft.irfftn(wf, s=(nz, ny, nx), axes=(0, 1, 2)).astype(np.float64)
    del wf
    z -= z.mean()
    sd = z.std()
    if sd > 0:
        z *= sigma / sd
    return np.ascontiguousarray(z)


def lognormal_kappa3(nx: int, ny: int, nz: int, sigma: float, corr_len: float,
                     seed: int) -> np.ndarray:
    """K = exp(Z) with Z from :func:`grf_logk3`, [nz, ny, nx]."""
    return np.exp(grf_logk3(nx, ny, nz, sigma, corr_len, seed))


def lognormal_kappa(nx: int, ny: int, sigma: float, corr_len: float, seed: int) -> np.ndarray:
    """K = exp(Z) with Z from :func:`grf_logk` (lattice units, median 1)."""
    return np.exp(grf_logk(nx, ny, sigma, corr_len, seed))


def channelize(kappa: np.ndarray, frac: float = 0.05, width: int = 8,
               factor: float = 1e3, seed: int = 1) -> np.ndarray:
    """Multiply x-aligned streaks of rows by ``factor``.

    The rows are split into slots of ``width`` rows; round(frac * ny / width)
    slots, drawn without replacement with ``default_rng(seed)``, become
    high-permeability channels. Returns a new array.
    """
    ny = kappa.shape[0]
    nslots = ny // width
    nstreak = max(1, int(round(frac * ny / width)))
    rng = np.random.default_rng(seed)
    slots = rng.choice(nslots, size=min(nstreak, nslots), replace=False)
    out = kappa.copy()
    for s in slots:
        out[s * width:(s + 1) * width, :] *= factor
    return out


# ----------------------------------------------------------------------------
# Fields the paper defines (physical units, m^2)
# ----------------------------------------------------------------------------


def block_field(n: int = 100, k_in: float = 1e-6, k_out: float = 1e-5) -> np.ndarray:
    """Sec. 4.1, Eq. kappa-forcemodel: k_in for 31 <= i, j <= 70 (1-based
    point indices), k_out elsewhere, on an n x n grid."""
    k = np.full((n, n), k_out)
    idx = np.arange(1, n + 1)
    inside = (idx >= 31) & (idx <= 70)
    k[np.ix_(inside, inside)] = k_in
    return k


def layered_field(n: int = 100, nlayers: int = 10, k1: float = 1e-12,
                  k2: float = 2e-12) -> np.ndarray:
    """Sec. 4.2.1: n x n grid cut into ``nlayers`` equal layers parallel to the
    y axis (so kappa varies with x). Odd-numbered layers (1-based) hold k1,
    even-numbered layers k2."""
    width = n // nlayers
    layer = np.arange(n) // width          # 0-based layer of each column x
    kx = np.where(layer % 2 == 0, k1, k2)  # 0-based even == 1-based odd
    return np.ascontiguousarray(np.broadcast_to(kx[None, :], (n, n)))


def checkerboard_field(n: int = 100, nsq: int = 10, k1: float = 1e-12,
                       k2: float = 2e-12) -> np.ndarray:
    """Sec. 4.2.2: n x n grid cut into nsq x nsq squares, alternating k1/k2."""
    width = n // nsq
    bi = np.arange(n) // width
    parity = (bi[:, None] + bi[None, :]) % 2
    return np.where(parity == 0, k1, k2).astype(np.float64)


def sinusoid_kappa(x: np.ndarray, y: np.ndarray, k_const: float) -> np.ndarray:
    """Sec. 4.3 background permeability 10 (1 + sin(80 pi x) cos(80 pi y)) k_const."""
    return 10.0 * (1.0 + np.sin(80.0 * np.pi * x) * np.cos(80.0 * np.pi * y)) * k_const


def cell_coords(n: int, dx: float, offset: float = 0.5) -> np.ndarray:
    """Coordinates x_i = (i + offset) dx of n grid points (offset 0.5 = cell
    centres, offset 0 = nodes)."""
    return (np.arange(n) + offset) * dx


def sinusoid_patch(side: int = 10, dx: float = 0.0025, k_const: float = 1e-13,
                   offset: float = 0.5, origin: tuple[int, int] = (0, 0)) -> np.ndarray:
    """One side x side subdomain of the Sec. 4.3 sinusoidal background field,
    starting at point index ``origin`` = (i0, j0)."""
    i0, j0 = origin
    x = cell_coords(side, dx, offset) + i0 * dx
    y = cell_coords(side, dx, offset) + j0 * dx
    return np.ascontiguousarray(sinusoid_kappa(x[None, :], y[:, None], k_const))


def five_block_field(n: int = 400, dx: float = 0.0025, k_const: float = 1e-13,
                     offset: float = 0.5) -> np.ndarray:
    """Sec. 4.3, Eq. finekappa-fiveblock on an n x n grid of spacing dx."""
    x = cell_coords(n, dx, offset)
    X, Y = np.meshgrid(x, x, indexing="xy")  # X varies along axis 1 (x fastest)
    k = sinusoid_kappa(X, Y, k_const)
    eps = 1e-12

    def box(lo_x, hi_x, lo_y, hi_y):
        return ((X >= lo_x - eps) & (X <= hi_x + eps) & (Y >= lo_y - eps) & (Y <= hi_y + eps))

    mask = (box(0.45, 0.55, 0.45, 0.55) | box(0.2, 0.3, 0.2, 0.3) | box(0.7, 0.8, 0.7, 0.8)
            | box(0.2, 0.3, 0.7, 0.8) | box(0.7, 0.8, 0.2, 0.3))
    k[mask] = k_const
    return np.ascontiguousarray(k)


def five_block_coarse(nc: int = 40, k_const: float = 1e-13, k_star: float = 8.485) -> np.ndarray:
    """Sec. 4.3, Eq. coarsekappa-fiveblock: the coarse scalar field on nc x nc
    points with 1-based indices (I, J); ``k_star`` is the multiple of k_const
    used outside the five blocks."""
    I = np.arange(1, nc + 1)
    X, Y = np.meshgrid(I, I, indexing="xy")

    def box(a, b, c, d):
        return (X >= a) & (X <= b) & (Y >= c) & (Y <= d)

    mask = (box(19, 22, 19, 22) | box(9, 12, 9, 12) | box(29, 32, 29, 32)
            | box(9, 12, 29, 32) | box(29, 32, 9, 12))
    return np.where(mask, k_const, k_star * k_const).astype(np.float64)


# ----------------------------------------------------------------------------
# Physical <-> lattice units
# ----------------------------------------------------------------------------


@dataclass(frozen=True)
class LatticeUnits:
    """Lattice spacing dx [m] and time step dt [s]; c = dx / dt."""
    dx: float
    dt: float

    def nu(self, nu_phys: float) -> float:
        return nu_phys * self.dt / (self.dx * self.dx)

    def kappa(self, k_phys):
        return np.asarray(k_phys, dtype=np.float64) / (self.dx * self.dx)

    def force(self, g_phys):
        return np.asarray(g_phys, dtype=np.float64) * self.dt * self.dt / self.dx

    def tau(self, nu_eff_phys: float) -> float:
        """tau from nu_eff = c_s^2 (tau - 1/2) dt with c_s^2 = dx^2 / (3 dt^2)."""
        return 0.5 + 3.0 * nu_eff_phys * self.dt / (self.dx * self.dx)

    def velocity_to_phys(self, u_lat):
        return np.asarray(u_lat) * self.dx / self.dt

    def kappa_to_phys(self, k_lat):
        return np.asarray(k_lat) * self.dx * self.dx


# ----------------------------------------------------------------------------
# Patch lists for the local problems
# ----------------------------------------------------------------------------


def tile_patches(nx: int, ny: int, side: int):
    """Origins of the side x side tiling of an nx x ny field: tile (I, J)
    covers [side*I, side*I + side) x [side*J, side*J + side). Returns
    (x0, y0, sides) int32 arrays, row-major over J then I."""
    if nx % side or ny % side:
        raise ValueError("tiling needs side | nx and side | ny")
    J, I = np.meshgrid(np.arange(ny // side), np.arange(nx // side), indexing="ij")
    x0 = (I.ravel() * side).astype(np.int32)
    y0 = (J.ravel() * side).astype(np.int32)
    return x0, y0, np.full(x0.shape, side, np.int32)


def mixed_patches(n: int, nx: int, ny: int, seed: int,
                  sides=(16, 24, 32, 48, 64)):
    """n patches with side drawn uniformly from ``sides`` and origin uniform in
    [0, nx) x [0, ny) (patches wrap periodically over the field)."""
    rng = np.random.default_rng(seed)
    s = rng.choice(np.asarray(sides, np.int32), size=n)
    x0 = rng.integers(0, nx, size=n, dtype=np.int64).astype(np.int32)
    y0 = rng.integers(0, ny, size=n, dtype=np.int64).astype(np.int32)
    return x0, y0, s.astype(np.int32)


def cut_patch(field: np.ndarray, x0: int, y0: int, side: int) -> np.ndarray:
    """Periodic side x side window of ``field`` starting at (x0, y0)."""
    ny, nx = field.shape
    ys = (y0 + np.arange(side)) % ny
    xs = (x0 + np.arange(side)) % nx
    return np.ascontiguousarray(field[np.ix_(ys, xs)])


# ----------------------------------------------------------------------------
# Named workloads (lattice units; eps = 0.4, tau = 0.8, nu = nu_eff = 0.1,
# rho0 = 1, g = 1e-6 unless stated)
# ----------------------------------------------------------------------------

COMMON = dict(tau=0.8, eps=0.4, nu=0.1, rho0=1.0, g=1e-6)


def workload_small(seed: int = 1) -> dict:
    """64 x 64, sigma 1, correlation length 8, walls in y, run to steady state."""
    return dict(nx=64, ny=64, kappa=lognormal_kappa(64, 64, 1.0, 8.0, seed),
                walls_y=1, **COMMON)


def workload_fine(seed: int = 1, n: int = 2048) -> dict:
    """n x n (2048 by default), sigma 1.5, correlation length 32, walls in y."""
    return dict(nx=n, ny=n, kappa=lognormal_kappa(n, n, 1.5, 32.0, seed),
                walls_y=1, **COMMON)


def workload_upscale(seed: int = 1, n: int = 4096, channels: bool = False) -> dict:
    """n x n (4096 by default), sigma 2, correlation length 64 n / 4096 (64 at
    full size), fully periodic; optionally with 5% of rows in x-aligned
    streaks of width 8 at K x 1e3."""
    k = lognormal_kappa(n, n, 2.0, 64.0 * n / 4096.0, seed)
    if channels:
        k = channelize(k, 0.05, 8, 1e3, seed)
    return dict(nx=n, ny=n, kappa=k, walls_y=0, **COMMON)


def workload_sec41() -> dict:
    """Sec. 4.1 (the comparison of the two force forms, the paper's only
    timing): 100 x 100 periodic, dx 0.01 m, dt 1e-4 s, tau 0.53, nu 2e-6
    m^2/s, eps 0.8, G = (2, 0) m/s^2, the block field of Eq.
    kappa-forcemodel; 200 000 steps. Lattice units."""
    U = LatticeUnits(0.01, 1e-4)
    return dict(nx=100, ny=100, kappa=np.ascontiguousarray(U.kappa(block_field(100))),
                tau=0.53, eps=0.8, nu=float(U.nu(2e-6)), g=(float(U.force(2.0)), 0.0),
                steps=200_000, units=U)


def workload_d3q19(seed: int = 1, n: int = 256) -> dict:
    """D3Q19 fine grid: n^3 (256^3 by default), sigma 1.5, correlation length
    16 n / 256, walls in z (x and y periodic), the same physics as the
    two-dimensional fine workload, force along x."""
    return dict(nx=n, ny=n, nz=n, kappa=lognormal_kappa3(n, n, n, 1.5, 16.0 * n / 256.0, seed),
                walls_z=1, tau=0.8, eps=0.4, nu=0.1, g=(1e-6, 0.0, 0.0))


def surrogate_fields(n_fields: int, seed: int, n: int = 256,
                     sigma_range=(0.5, 2.5), corr_range=(4.0, 32.0)):
    """Yield (sigma, corr_len, field) for training fields: sigma and the
    correlation length drawn uniformly from the given ranges, one fresh GRF
    seed per field."""
    rng = np.random.default_rng(seed)
    for i in range(n_fields):
        sg = float(rng.uniform(*sigma_range))
        cl = float(rng.uniform(*corr_range))
        fseed = int(rng.integers(0, 2**31 - 1))
        yield sg, cl, lognormal_kappa(n, n, sg, cl, fseed)


def log_patches(field: np.ndarray, side: int = 32) -> np.ndarray:
    """All side x side tiles of a field as log K, shape [n, side, side]."""
    ny, nx = field.shape
    t = np.log(field).reshape(ny // side, side, nx // side, side).transpose(0, 2, 1, 3)
    return np.ascontiguousarray(t.reshape(-1, side, side))


__all__ = [n for n in dir() if not n.startswith("_") and n not in ("annotations", "math")]
