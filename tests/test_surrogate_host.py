"""Host-side pieces of the surrogate: parameter layout, the committed model,
the range detector and the patch mosaic (no GPU)."""
import os

import numpy as np
import pytest

from oracle import cnn_oracle as C
from paper_1312_0195_amd import inputs as I
from paper_1312_0195_amd import lbm as L
from paper_1312_0195_amd import surrogate as S
from paper_1312_0195_amd import train_surrogate as T


def test_parameter_count_matches_the_oracle_layout():
    p = C.init_params(C=32, hidden=32)
    assert L.lbm_cnn_param_count() == sum(v.size for v in p.values())
    assert S.init_params().size == L.lbm_cnn_param_count()


def test_committed_model_loads():
    assert os.path.exists(T.DEFAULT_MODEL)
    m = S.Surrogate.load(T.DEFAULT_MODEL)
    assert m.params.dtype == np.float32 and m.params.size == L.lbm_cnn_param_count()
    assert np.isfinite(m.params).all() and len(m.history) > 0
    # a calibrated detector: finite thresholds, a positive definite inverse covariance
    assert np.isfinite(m.det_d2_max) and m.det_d2_max > 0 and np.isfinite(m.spread_max) and m.spread_max > 0
    assert m.det_mean.shape == (6,) and np.all(np.linalg.eigvalsh(m.det_icov) > 0)


def _detector(mean, cov, d2_max, spread_max=np.inf):
    return S.Surrogate(S.init_params(), np.asarray(mean, float), np.linalg.inv(np.asarray(cov, float)),
                       d2_max, spread_max)


def test_range_detector_mahalanobis():
    """Stage one accepts a patch when the squared Mahalanobis distance of its
    detector features from the in-range mean is at most det_d2_max: here the
    features (std, rx, ry, the two estimate gaps, the difference of the upper
    estimates) with a diagonal covariance, so the distance is a sum of
    squared z-scores; NaN statistics are never accepted."""
    mean = [1.0, 0.9, 0.9, 0.6, 0.6, 0.0]
    sd = np.array([0.5, 0.05, 0.05, 0.3, 0.3, 0.2])
    m = _detector(mean, np.diag(sd ** 2), 9.0)
    st = np.array([[0.0, 1.0, 0.9, 0.9, -0.3, 0.3, -0.3, 0.3],      # at the mean
                   [0.0, 2.4, 0.9, 0.9, -0.3, 0.3, -0.3, 0.3],      # std 2.8 sd away
                   [0.0, 2.6, 0.9, 0.9, -0.3, 0.3, -0.3, 0.3],      # 3.2 sd away
                   [0.0, 1.0, 0.96, 0.84, -0.3, 0.3, -0.3, 0.3],    # rx and ry 1.2 sd each
                   [0.0, 1.0, 0.9, 0.9, np.nan, 0.3, -0.3, 0.3]])
    d2 = m.distance2(st)
    assert np.allclose(d2[:4], [0.0, (1.4 / 0.5) ** 2, (1.6 / 0.5) ** 2, 2 * 1.2 ** 2])
    assert np.isinf(d2[4])
    assert list(m.in_range(st)) == [True, True, False, True, False]


def test_range_detector_correlated_features():
    """With correlated features the distance follows the inverse covariance,
    not per-feature bounds: two features that move together in range are
    accepted together and rejected when they move apart by the same amount."""
    cov = np.eye(6)
    cov[1, 2] = cov[2, 1] = 0.95
    m = _detector(np.zeros(6), cov, 4.0)
    st = np.zeros((2, 8))
    st[0, 2:4] = [1.5, 1.5]    # rx and ry together
    st[1, 2:4] = [1.5, -1.5]   # apart
    f = S.detector_features(st)
    d2 = np.einsum("ij,jk,ik->i", f, np.linalg.inv(cov), f)
    assert np.allclose(m.distance2(st), d2)
    assert d2[0] < 4.0 < d2[1]
    assert list(m.in_range(st)) == [True, False]


def test_spread_stage():
    """Stage two accepts a patch when the larger of its two outputs' spreads
    is at most spread_max; NaN is never accepted."""
    m = _detector(np.zeros(6), np.eye(6), np.inf, 0.05)
    spread = np.array([[0.01, 0.04], [0.06, 0.0], [0.05, 0.05], [np.nan, 0.0]])
    assert list(m.confident(spread)) == [True, False, True, False]


def test_mosaic_keeps_fields_and_tiles():
    fields = [np.full((64, 64), i + 1.0) for i in range(5)]
    big, x0, y0 = S.mosaic(fields)
    assert len(x0) == 5 * 4
    for i, (a, b) in enumerate(zip(x0, y0)):
        patch = I.cut_patch(big, a, b, 32)
        assert (patch == i // 4 + 1).all()


def test_test_set_mix():
    big, x0, y0, oor = T.test_set(n_total=64 * 20, frac_oor=0.1, seed=3)
    assert len(x0) == 64 * 20 and (oor > 0).sum() == 128
    assert set(np.unique(oor[oor > 0])) == {1, 2}  # two out-of-range fields: kinds 1 and 2


def test_detector_features():
    """The six detector features from the eight statistics columns."""
    st = np.array([[0.0, 1.0, 0.9, 0.8, -0.3, 0.3, -0.2, 0.5],
                   [0.0, 2.0, 0.5, 0.7, -2.0, 2.0, -0.3, 0.3]])
    f = S.detector_features(st)
    assert f.shape == (2, 6)
    assert np.allclose(f[0], [1.0, 0.9, 0.8, 0.6, 0.7, -0.2])
    assert np.allclose(f[1], [2.0, 0.5, 0.7, 4.0, 0.6, 1.7])


def test_detector_round_trips_through_save(tmp_path):
    m = _detector(np.arange(6.0), np.diag(np.arange(1.0, 7.0)), 12.5, 0.031)
    m.history = [1.0, 0.5]
    path = str(tmp_path / "m.npz")
    m.save(path)
    r = S.Surrogate.load(path)
    assert np.array_equal(r.det_mean, m.det_mean) and np.array_equal(r.det_icov, m.det_icov)
    assert r.det_d2_max == 12.5 and r.spread_max == 0.031 and r.n_sym == m.n_sym
