"""Planted mistakes in the Python parts of the oracle (on the CPU): each
plausible slip must make at least one pin fail. This checks the pins, not
the GPU path; the mistakes live only inside these tests (monkeypatch)."""
import numpy as np
import pytest

from oracle import d3q19 as D
from oracle import direct as DS

import test_cnn_oracle as PC
import test_oracle_d3q19 as P3
import test_oracle_pins as P2
from oracle import cnn_oracle as CO


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


def _any_fails(fns):
    failed = 0
    for fn in fns:
        try:
            fn()
        except AssertionError:
            failed += 1
    return failed


def test_cnn_shift_reversed_fails_conv_pin(monkeypatch):
    monkeypatch.setattr(CO, "_shift", lambda a, dy, dx: np.roll(a, shift=(dy, dx), axis=(1, 2)))
    _fails(PC.test_conv_matches_brute_force_loops)


def test_cnn_backward_slips_fail_gradient_pin(monkeypatch):
    good_bwd = CO.conv3x3_backward

    def bwd_wrong_way(a, W, g):
        da = np.zeros_like(a)
        dW = np.zeros_like(W)
        for t, (dy, dx) in enumerate(CO.TAPS):
            dW[t] = np.einsum("bhwi,bhwo->io", CO._shift(a, dy, dx), g)
            da += CO._shift(g @ W[t].T, dy, dx)          # sent back the wrong way
        return da, dW, g.sum(axis=(0, 1, 2))

    monkeypatch.setattr(CO, "conv3x3_backward", bwd_wrong_way)
    _fails(PC.test_gradients_match_central_differences)
    monkeypatch.setattr(CO, "conv3x3_backward", good_bwd)
    PC.test_gradients_match_central_differences()         # the unpatched oracle passes


def test_cnn_transpose_first_fails_transform_pin(monkeypatch):
    def transform(logk, sym):
        t, fx, fy = sym & 1, (sym >> 1) & 1, (sym >> 2) & 1
        a = np.asarray(logk)
        if t:
            a = np.swapaxes(a, 1, 2)                      # transpose before the mirrors
        if fx:
            a = a[:, :, ::-1]
        if fy:
            a = a[:, ::-1, :]
        return np.ascontiguousarray(a)

    monkeypatch.setattr(CO, "transform", transform)
    assert _any_fails([PC.test_transform_matches_pixel_loops_and_forms_the_group,
                       PC.test_symmetric_prediction_is_equivariant]) >= 1


def test_cnn_adam_without_bias_correction_fails_pin(monkeypatch):
    def adam_step(p, g, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        for k in p:
            m = state.setdefault("m_" + k, np.zeros_like(p[k]))
            v = state.setdefault("v_" + k, np.zeros_like(p[k]))
            m[...] = b1 * m + (1 - b1) * g[k]
            v[...] = b2 * v + (1 - b2) * g[k] ** 2
            p[k] = p[k] - lr * m / (np.sqrt(v) + eps)

    monkeypatch.setattr(CO, "adam_step", adam_step)
    _fails(PC.test_adam_first_step_is_signed_learning_rate)


def test_cnn_series_parallel_axes_swapped_fails_pin(monkeypatch):
    good = CO.series_parallel
    monkeypatch.setattr(CO, "series_parallel", lambda x: good(np.swapaxes(x, 1, 2)))
    _fails(PC.test_series_parallel_features_of_layered_patch)
