"""Pins of the FP64 surrogate-network oracle (forward, backward, Adam)."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import cnn_oracle as C


def _small(seed=0):
    p = C.init_params(C=4, hidden=5, seed=seed)
    rng = np.random.default_rng(seed + 1)
    for k in p:
        if k.startswith("b") or k.startswith("c"):
            p[k] = 0.1 * rng.standard_normal(p[k].shape)
    x = rng.standard_normal((3, 6, 7))
    t = rng.standard_normal((3, 2))
    return p, x, t


def test_conv_matches_brute_force_loops():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((2, 5, 6, 3))
    W = rng.standard_normal((9, 3, 4))
    b = rng.standard_normal(4)
    out = C.conv3x3(a, W, b)
    B, H, Wd, _ = a.shape
    ref = np.zeros((B, H, Wd, 4))
    for n in range(B):
        for y in range(H):
            for x in range(Wd):
                for co in range(4):
                    s = b[co]
                    for t, (dy, dx) in enumerate(C.TAPS):
                        for ci in range(3):
                            s += a[n, (y + dy) % H, (x + dx) % Wd, ci] * W[t, ci, co]
                    ref[n, y, x, co] = s
    assert np.allclose(out, ref, rtol=1e-13, atol=1e-13)


def test_conv_matches_scipy_wrap_correlation():
    rng = np.random.default_rng(4)
    a = rng.standard_normal((1, 9, 8, 1))
    W = rng.standard_normal((9, 1, 1))
    k = W[:, 0, 0].reshape(3, 3)  # rows dy = -1..1, cols dx = -1..1
    ref = ndimage.correlate(a[0, :, :, 0], k, mode="wrap")
    assert np.allclose(C.conv3x3(a, W, np.zeros(1))[0, :, :, 0], ref, rtol=1e-13, atol=1e-13)


def test_gradients_match_central_differences():
    p, x, t = _small()
    y, cache = C.forward(p, x)
    g = C.backward(p, cache, y, t)
    h = 1e-6
    rng = np.random.default_rng(9)
    for k in p:
        flat = p[k].reshape(-1)
        idx = rng.choice(flat.size, size=min(6, flat.size), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + h
            lp = C.loss(C.forward(p, x)[0], t)
            flat[i] = old - h
            lm = C.loss(C.forward(p, x)[0], t)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            an = g[k].reshape(-1)[i]
            assert abs(fd - an) <= 1e-6 * max(1e-3, abs(fd)), (k, i, fd, an)


def test_network_is_invariant_to_circular_shifts():
    p = C.init_params(C=6, hidden=7, seed=2)
    rng = np.random.default_rng(5)
    x = rng.standard_normal((2, 10, 10))
    y0, _ = C.forward(p, x)
    y1, _ = C.forward(p, np.roll(x, (3, -4), axis=(1, 2)))
    assert np.allclose(y0, y1, rtol=1e-12, atol=1e-14)


def test_input_is_centred_and_mean_feeds_the_head():
    p = C.init_params(C=4, hidden=5, seed=1)
    rng = np.random.default_rng(6)
    x = rng.standard_normal((2, 6, 6))
    _, c1 = C.forward(p, x)
    _, c2 = C.forward(p, x + 3.0)
    assert np.allclose(c1["acts"][4], c2["acts"][4], rtol=1e-12)
    assert np.allclose(c2["m"] - c1["m"], 3.0)


def test_adam_first_step_is_signed_learning_rate():
    p = {"w": np.array([1.0, -2.0, 0.5])}
    g = {"w": np.array([0.3, -1e-3, 5.0])}
    st = {}
    C.adam_step(p, g, st, lr=1e-2, eps=1e-12)
    assert np.allclose(p["w"], [1.0 - 1e-2, -2.0 + 1e-2, 0.5 - 1e-2], rtol=1e-9)


def test_forward_flop_count():
    # 2 * 1024 * 9 * (32 + 3 * 32 * 32) + MLP = 57.2 MFLOP per 32 x 32 patch
    f = C.flops_forward()
    assert 57.1e6 < f < 57.3e6


def test_series_parallel_features_of_layered_patch():
    """Layers constant along x: flow along the layers sees the arithmetic mean
    of the layer values, flow across them the harmonic mean (both estimates of
    each pair coincide for a layered medium)."""
    rng = np.random.default_rng(11)
    layers = rng.normal(0.0, 1.0, 8)
    x = np.repeat(layers[:, None], 5, axis=1)[None]  # [1, 8 rows, 5 columns]
    k = np.exp(layers)
    f = C.series_parallel(x)[0]
    assert np.allclose(f[:2], np.log(k.mean()), rtol=0, atol=1e-13)
    assert np.allclose(f[2:], -np.log(np.mean(1.0 / k)), rtol=0, atol=1e-13)


def test_series_parallel_lower_estimate_below_upper():
    """The mean of harmonic means never exceeds the harmonic mean of the
    arithmetic means (concavity of the harmonic mean), in either direction."""
    rng = np.random.default_rng(12)
    f = C.series_parallel(rng.normal(0.0, 1.5, (20, 9, 7)))
    assert (f[:, 0] <= f[:, 1] + 1e-14).all() and (f[:, 2] <= f[:, 3] + 1e-14).all()
    assert (f[:, 1] - f[:, 0] > 1e-3).all()


def test_transform_matches_pixel_loops_and_forms_the_group():
    rng = np.random.default_rng(13)
    a = rng.standard_normal((1, 4, 4))
    seen = set()
    for s in range(8):
        t = C.transform(a, s)
        for y in range(4):
            for x in range(4):
                u, v = (y, x) if s & 1 else (x, y)
                if s & 2:
                    u = 3 - u
                if s & 4:
                    v = 3 - v
                assert t[0, y, x] == a[0, v, u]
        seen.add(t.tobytes())
    assert len(seen) == 8


def test_symmetric_prediction_is_equivariant():
    """Averaging over the whole group makes the prediction equivariant: a
    transformed patch gets the same K_eff, with kxx and kyy exchanged when the
    symmetry transposes."""
    p = C.init_params(C=4, hidden=6, seed=3)
    rng = np.random.default_rng(14)
    x = rng.standard_normal((2, 6, 6))
    y = C.predict_symmetric(p, x)
    for s in range(8):
        ys = C.predict_symmetric(p, C.transform(x, s))
        assert np.allclose(ys, y[:, ::-1] if s & 1 else y, rtol=1e-12, atol=1e-13)
    # one evaluation alone is not (a generic network breaks the symmetry)
    y1 = C.predict_symmetric(p, x, n_sym=1)
    y1t = C.predict_symmetric(p, C.transform(x, 1), n_sym=1)
    assert np.abs(y1t[:, ::-1] - y1).max() > 1e-6
