"""Host-side pieces of the surrogate: parameter layout, the committed model,
the range detector and the patch mosaic (no GPU)."""
import os

import numpy as np

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
    assert np.isfinite(m.params).all()
    assert (m.stat_lo < m.stat_hi).all() and len(m.history) > 0


def test_range_detector():
    m = S.Surrogate(S.init_params(), np.array([0.5, 0.8, 0.8, -0.05]),
                    np.array([3.0, 1.0, 1.0, 0.05]))
    stats = np.array([[0.0, 1.0, 0.9, 0.9],     # inside
                      [0.0, 3.5, 0.9, 0.9],     # std too large
                      [0.0, 1.0, 0.99, 0.85]])  # anisotropic
    assert list(m.in_range(stats)) == [True, False, False]


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


def test_detector_uses_series_parallel_gaps():
    """With the eight-column statistics the detector also bounds the gap
    between the upper and lower series/parallel estimates."""
    st = np.array([[0.0, 1.0, 0.9, 0.9, -0.3, 0.3, -0.3, 0.3],
                   [0.0, 1.0, 0.9, 0.9, -2.0, 2.0, -0.3, 0.3]])
    f = S.detector_features(st)
    assert f.shape == (2, 7) and np.allclose(f[:, 4], [0.6, 4.0])
    m = S.Surrogate(S.init_params(), np.array([0.5, 0.8, 0.8, -0.05, 0.0, 0.0, -1.0]),
                    np.array([3.0, 1.0, 1.0, 0.05, 1.0, 1.0, 1.0]))
    assert list(m.in_range(st)) == [True, False]


def test_range_detector_equals_the_feature_matrix_test():
    """in_range (column by column) flags exactly the rows whose detector
    features leave [stat_lo, stat_hi], NaN rows included, for the committed
    model's bounds and for a model that bounds only the first four features."""
    rng = np.random.default_rng(4)
    st = rng.normal(size=(5000, 8)) * 0.6 + np.array([0, 1, 0.9, 0.9, -0.3, 0.3, -0.3, 0.3])
    st[::37, rng.integers(0, 8)] = np.nan
    m = S.Surrogate.load(T.DEFAULT_MODEL)
    short = S.Surrogate(S.init_params(), np.array([0.5, 0.8, 0.8, -0.05]), np.array([3.0, 1.0, 1.0, 0.05]))
    for model in (m, short):
        f = S.detector_features(st)[:, :len(model.stat_lo)]
        want = ((f >= model.stat_lo) & (f <= model.stat_hi)).all(axis=1)
        got = model.in_range(st)
        assert got.dtype == bool and np.array_equal(got, want)
        assert 0 < want.sum() < len(want)
