"""Pins of the learned-predictor oracle (oracle/learned.py) against closed
forms, invariances, finite differences and library routines."""
import numpy as np
import pytest

from oracle import learned as Lr
from paper_2106_03138_amd import inputs as I


def _q(m, n, seed):
    return I.haar_cols(m, n, np.random.default_rng(seed))


def test_parameter_count():
    assert Lr.NPARAM == 16 * 64 + 64 + 64 * 64 + 64 + 64 * 3 + 3 == 5443


def test_sample_columns_spread():
    for n in (1, 5, 63, 64, 65, 200, 512):
        s = Lr.sample_columns(n)
        assert len(s) == min(64, n)
        assert np.all(np.diff(s) > 0) and s[0] == 0 and s[-1] < n


def test_features_orthogonal_columns_closed_form():
    """Orthogonal columns: every cosine is 0; the norm quantiles are the order
    statistics of log10(s / max s) of the prescribed norms."""
    m, n = 120, 50
    s = np.geomspace(3.0, 3e-6, n)[np.random.default_rng(2).permutation(n)]
    a = _q(m, n, 1) * s[None, :]
    f = Lr.features(a)
    ell = np.sort(np.log10(s / s.max()))
    want = [ell[int(np.floor((k + 1) / 10 * (n - 1)))] for k in range(9)]
    np.testing.assert_allclose(f[:9], want, atol=1e-12)
    assert np.allclose(f[12:16], 0.0, atol=1e-12)
    np.testing.assert_allclose(f[9:12], [np.log2(m), np.log2(n), n / m], rtol=1e-15)


def test_features_rank_one_all_cosines_one():
    a = I.rank1(40, 30, 3)
    f = Lr.features(a)
    np.testing.assert_allclose(f[12:16], [1.0, 1.0, 1.0, 1.0], atol=1e-12)


def test_features_equal_norms_and_zero_matrix():
    a = _q(60, 20, 4) * 2.5
    assert np.allclose(Lr.features(a)[:9], 0.0, atol=1e-14)
    z = Lr.features(np.zeros((10, 7)))
    assert np.allclose(z[:9], 0.0) and np.allclose(z[12:], 0.0)
    np.testing.assert_allclose(z[9:12], [np.log2(10), np.log2(7), 0.7])


def test_features_scale_and_sign_invariance():
    rng = np.random.default_rng(5)
    a = rng.standard_normal((90, 70)) * np.exp(rng.uniform(-3, 3, 70))[None, :]
    f0 = Lr.features(a)
    np.testing.assert_allclose(Lr.features(7.25 * a), f0, atol=1e-12)
    np.testing.assert_allclose(Lr.features(-a), f0, atol=1e-12)


def test_features_two_columns_by_hand():
    """Two columns at a known angle: the only cosine is cos(angle)."""
    ang = 0.3
    a = np.zeros((4, 2))
    a[0, 0] = 2.0
    a[0, 1], a[1, 1] = np.cos(ang), np.sin(ang)
    f = Lr.features(a)
    assert f[12] == pytest.approx(np.cos(ang), abs=1e-15)
    assert f[13] == f[14] == pytest.approx(np.cos(ang), abs=1e-15)
    assert f[15] == 1.0
    # norms 2 and 1: log10 values 0 and log10(1/2)
    assert f[0] == pytest.approx(np.log10(0.5), abs=1e-15)


def test_mlp_zero_weights_output_bias():
    theta = np.zeros(Lr.NPARAM)
    theta[-3:] = [0.1, -0.2, 0.3]
    y, _ = Lr.mlp_forward(theta, np.random.default_rng(0).standard_normal((5, 16)))
    np.testing.assert_allclose(y, np.tile([0.1, -0.2, 0.3], (5, 1)), atol=0)


def test_mlp_gradient_matches_finite_differences():
    rng = np.random.default_rng(7)
    theta = rng.standard_normal(Lr.NPARAM) * 0.3
    x = rng.standard_normal((6, 16))
    y = rng.standard_normal((6, 3))
    g = Lr.mlp_grad(theta, x, y)
    idx = rng.choice(Lr.NPARAM, 400, replace=False)
    idx = np.concatenate([idx, [0, 1023, 1024, 5439, 5440, 5442]])
    h = 1e-6
    for i in idx:
        e = np.zeros(Lr.NPARAM)
        e[i] = h
        fd = (Lr.mlp_loss(theta + e, x, y) - Lr.mlp_loss(theta - e, x, y)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 + 1e-6 * abs(fd), (i, fd, g[i])


def test_adam_first_step_is_lr_times_sign():
    """With zero moments, the bias-corrected first step is lr g / (|g| + eps)."""
    rng = np.random.default_rng(1)
    th = rng.standard_normal(50)
    g = rng.standard_normal(50)
    t1, _, _ = Lr.adam_step(th, g, np.zeros(50), np.zeros(50), 1, lr=0.01)
    np.testing.assert_allclose(t1 - th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_adam_minimizes_a_quadratic():
    c = np.linspace(-2, 3, 20)
    th = np.zeros(20)
    mom, vel = np.zeros(20), np.zeros(20)
    for t in range(1, 3001):
        th, mom, vel = Lr.adam_step(th, th - c, mom, vel, t, lr=0.05)
    assert np.max(np.abs(th - c)) < 1e-3


def test_quality_rule_and_numerical_rank():
    s = np.geomspace(1.0, 1e-16, 100)
    nr = Lr.numerical_rank(s, 100)
    assert nr == int(np.sum(s > np.finfo(float).eps * 100))
    assert Lr.quality_ok(s.copy(), s, 100)
    # the rule compares sorted |r_ii| with sigma: on a flat spectrum one entry
    # 20x too small sorts last and breaks the band
    flat = np.ones(30)
    d = flat.copy()
    d[7] *= 0.05
    assert not Lr.quality_ok(d, flat, 30)
    d[7] = 0.2
    assert Lr.quality_ok(d, flat, 30)
    assert Lr.quality_ok(np.zeros(3), np.zeros(3), 3)


def test_ice_diagonal_exact():
    d = np.array([3.0, -0.5, 2.0, 0.01, 7.0])
    assert Lr.ice_sigma_min(np.diag(d)) == pytest.approx(0.01, rel=1e-14)


@pytest.mark.parametrize("seed", range(4))
def test_ice_is_an_upper_bound_of_sigma_min(seed):
    """The estimate is ||x^T R|| for a unit x, so it can never be below sigma_min
    (library SVD); on these matrices it is also within a factor 10 of it."""
    rng = np.random.default_rng(seed)
    k = 40
    r = np.triu(rng.standard_normal((k, k))) + np.diag(np.geomspace(1, 1e-4, k))
    smin = np.linalg.svd(r, compute_uv=False)[-1]
    est = Lr.ice_sigma_min(r)
    assert est >= smin * (1 - 1e-12)
    assert est <= 10 * smin
