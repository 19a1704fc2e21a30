"""Pins of the variance-component oracle (oracle/vc.py) against what the model
fixes independently of its code: the closed-form OLS likelihood at h2 = 0, the
Gaussian density of y (ML) and of its error contrasts (REML), flatness when
Phi = I, invariances of the estimates, and a fine-grid check that the search
returns the maximiser."""
import math

import numpy as np
import pytest
from scipy.stats import multivariate_normal

from oracle import vc
from synth import make_workload


def _data(n=120, seed=3, h2=0.6):
    w = make_workload(2, n=n, m=10, t=3, kin_cols=2 * n)
    return w.Phi, np.asarray(w.XL), np.asarray(w.Y)


def test_ml_at_h2_zero_is_ols():
    Phi, X, Y = _data()
    y = Y[:, 0]
    n = len(y)
    beta, *_ = np.linalg.lstsq(X, y, rcond=None)
    rss = float(np.sum((y - X @ beta) ** 2))
    expect = -0.5 * n * (math.log(2 * math.pi * rss / n) + 1.0)
    ll, s2 = vc.loglik(Phi, X, y, 0.0, vc.ML)
    assert abs(ll - expect) < 1e-9 * abs(expect)
    assert abs(s2 - rss / n) < 1e-12 * s2


@pytest.mark.parametrize("h2", [0.0, 0.3, 0.85])
def test_ml_is_the_gaussian_density_at_the_estimates(h2):
    Phi, X, Y = _data()
    y = Y[:, 1]
    n = len(y)
    ll, s2 = vc.loglik(Phi, X, y, h2, vc.ML)
    H = h2 * Phi + (1 - h2) * np.eye(n)
    Hi = np.linalg.inv(H)
    beta = np.linalg.solve(X.T @ Hi @ X, X.T @ Hi @ y)
    dens = multivariate_normal(mean=X @ beta, cov=s2 * H).logpdf(y)
    assert abs(ll - dens) < 1e-8 * abs(dens)


@pytest.mark.parametrize("h2", [0.0, 0.45, 0.97])
def test_reml_is_the_density_of_the_error_contrasts(h2):
    """With K (n x (n-p)) orthonormal and K^T X = 0, the REML likelihood is the
    density of K^T y ~ N(0, s2 K^T H K) at the REML s2."""
    Phi, X, Y = _data()
    y = Y[:, 2]
    n, p = X.shape
    ll, s2 = vc.loglik(Phi, X, y, h2, vc.REML)
    Q, _ = np.linalg.qr(X, mode="complete")
    K = Q[:, p:]
    H = h2 * Phi + (1 - h2) * np.eye(n)
    dens = multivariate_normal(mean=np.zeros(n - p), cov=s2 * (K.T @ H @ K)).logpdf(K.T @ y)
    assert abs(ll - dens) < 1e-8 * abs(dens)


def test_identity_kinship_gives_a_flat_likelihood():
    _, X, Y = _data()
    n = X.shape[0]
    for method in (vc.ML, vc.REML):
        vals = [vc.loglik(np.eye(n), X, Y[:, 0], h, method)[0] for h in (0.0, 0.2, 0.7, 1.0)]
        assert max(vals) - min(vals) < 1e-9 * abs(vals[0])


@pytest.mark.parametrize("method", [vc.ML, vc.REML])
def test_estimate_is_the_maximiser_on_a_fine_grid(method):
    Phi, X, Y = _data()
    for j in range(Y.shape[1]):
        h2, s2, ll = vc.estimate(Phi, X, Y[:, j], method)
        fine = max(vc.loglik(Phi, X, Y[:, j], h, method)[0] for h in np.linspace(0, 1, 2001))
        assert ll >= fine - 1e-9 * abs(fine)
        assert 0.0 <= h2 <= 1.0 and s2 > 0


@pytest.mark.parametrize("method", [vc.ML, vc.REML])
def test_invariances_of_the_estimates(method):
    """y -> c y: h2 unchanged, s2 -> c^2 s2; y + X gamma: unchanged; X -> X T: unchanged."""
    Phi, X, Y = _data()
    y = Y[:, 0]
    h2, s2, ll = vc.estimate(Phi, X, y, method)
    h2c, s2c, _ = vc.estimate(Phi, X, -3.0 * y, method)
    assert abs(h2c - h2) < 1e-6 and abs(s2c - 9.0 * s2) < 1e-6 * 9.0 * s2
    h2g, s2g, llg = vc.estimate(Phi, X, y + X @ np.array([1.0, -2.0, 0.05]), method)
    assert abs(h2g - h2) < 1e-6 and abs(s2g - s2) < 1e-6 * s2 and abs(llg - ll) < 1e-8 * abs(ll)
    T = np.array([[1.0, 0.5, 2.0], [0.0, 3.0, -1.0], [0.0, 0.0, 0.2]])
    h2t, s2t, llt = vc.estimate(Phi, X @ T, y, method)
    assert abs(h2t - h2) < 1e-6 and abs(s2t - s2) < 1e-6 * s2 and abs(llt - ll) < 1e-8 * abs(ll)


def test_recovers_a_large_heritability():
    """Statistical sanity: n = 600 individuals drawn with h2 = 0.9 (config recipe) give a large estimate."""
    w = make_workload(2, n=600, m=10, t=12, kin_cols=1200)
    h2, _, _ = vc.estimate_all(w.Phi, np.asarray(w.XL), np.asarray(w.Y))
    assert np.corrcoef(h2, w.h2)[0, 1] > 0.5
