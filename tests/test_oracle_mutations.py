"""Planted mistakes in the Python parts of the oracle (on the CPU): each
plausible slip must make at least one pin fail. This checks the pins, not
the GPU path; the mistakes live only inside these tests (monkeypatch)."""
import numpy as np
import pytest

from oracle import d3q19 as D
from oracle import direct as DS

import test_oracle_d3q19 as P3
import test_oracle_pins as P2


def _fails(fn, *args):
    with pytest.raises(AssertionError):
        fn(*args)


def test_d3q19_wrong_edge_vector_fails_lattice_pin(monkeypatch):
    E, W, OPP = D.lattice()
    bad = E.copy()
    bad[18] = [0, -1, -1]              # a duplicated edge vector instead of (0, -1, +1)
    monkeypatch.setattr(D, "lattice", lambda: (bad, W, OPP))
    _fails(P3.test_lattice_is_d3q19)


def test_d3q19_wrong_weight_fails_pins(monkeypatch):
    E, W, OPP = D.lattice()
    bad = W.copy()
    bad[7:] = 1.0 / 35.0
    monkeypatch.setattr(D, "lattice", lambda: (E, bad, OPP))
    _fails(P3.test_lattice_is_d3q19)
    _fails(P3.test_z_invariant_flow_reduces_to_d2q9, 0.8)


def test_d3q19_wrong_shift_sign_fails_projection_pin(monkeypatch):
    good = D.collide

    def collide(p, kappa, f, g=(0.0, 0.0, 0.0)):
        E, W, _ = D.lattice()
        rho, u, j = D.moments(p, kappa, f, g)
        ueq = 2.0 * p.tau * u - (1.0 - 2.0 * p.tau) * j / rho   # sign slip
        eu = np.einsum("ad,dzyx->zyxa", E.astype(np.float64), ueq)
        feq = W * rho[..., None] * (1.0 + eu / D.CS2)
        return f + (feq - f) / p.tau

    monkeypatch.setattr(D, "collide", collide)
    _fails(P3.test_z_invariant_flow_reduces_to_d2q9, 0.8)
    monkeypatch.setattr(D, "collide", good)
    P3.test_z_invariant_flow_reduces_to_d2q9(0.8)   # the unpatched oracle passes


def test_d3q19_wall_on_wrong_plane_fails_channel_pin(monkeypatch):
    E, _, OPP = D.lattice()

    def stream(p, fs):
        out = np.empty_like(fs)
        for a in range(19):
            ex, ey, ez = (int(v) for v in E[a])
            out[..., a] = np.roll(fs[..., a], shift=(ez, ey, ex), axis=(0, 1, 2))
            if p.walls_z and ez != 0:
                zin = p.nz - 1 if ez > 0 else 0              # the wrong plane
                out[zin, :, :, a] = fs[zin, :, :, OPP[a]]
        return out

    monkeypatch.setattr(D, "stream", stream)
    _fails(P3.test_y_invariant_channel_with_z_walls_reduces_to_d2q9, 0.8)


@pytest.mark.parametrize("lo,hi", [(1, 0), (0, 1)])
def test_window_off_by_one_fails_window_pins(monkeypatch, lo, hi):
    O = DS.O

    def steady_mean_velocity(p, perm, g=(0.0, 0.0), force=None, margin=0):
        f = DS.steady_state(p, perm, g, force)
        if margin == 0:
            return O.mean_velocity(p, perm, f, g, force)
        _, ux, uy = O.moments(p, perm, f, g, force)
        w = (slice(margin, p.ny - margin), slice(margin + lo, p.nx - margin + hi))
        return np.array([ux[w].mean(), uy[w].mean()])

    monkeypatch.setattr(DS, "steady_mean_velocity", steady_mean_velocity)
    failed = 0
    for fn, args in ((P2.test_window_parallel_layers_local_darcy_law, (5,)),
                     (P2.test_window_symmetries_and_full_window, ())):
        try:
            fn(*args)
        except AssertionError:
            failed += 1
    assert failed >= 1
