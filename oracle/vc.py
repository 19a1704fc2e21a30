"""CPU FP64 oracle of the variance-component step (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this module.  It fits the reduced model of the first step of the two-step
analysis (supplementary notes, section 1: y ~ N(X_L beta, s2 (h2 Phi + (1 - h2)
I)), X = [1 | L]) for one trait, by maximum likelihood or restricted maximum
likelihood (the discussion of the parameter estimation in section 4 names
both).  s2 and beta are profiled out in closed form, h2 maximises the profile
log-likelihood over [0, 1].  Every evaluation goes through a dense Cholesky
factorisation of H = h2 Phi + (1 - h2) I (no eigendecomposition):

    ML   : s2 = RSS / n,        l = -1/2 [n (log(2 pi s2) + 1) + log det H]
    REML : s2 = RSS / (n - p),  l = -1/2 [(n - p)(log(2 pi s2) + 1) + log det H
                                         + log det(X^T H^-1 X) - log det(X^T X)]

with RSS = (y - X beta)^T H^-1 (y - X beta), beta = (X^T H^-1 X)^-1 X^T H^-1 y.
The search (the paper only says "an iterative procedure"; this is the reading
taken, the GPU path follows the same steps): the 101 points h2 = 0, 0.01, ...,
1, then a golden-section search on the bracket around the best of them (ties
to the smaller h2) down to a width of 1e-7, and the better of its midpoint and
the best grid point.
Parity status: pinned by tests/test_oracle_vc.py (closed form at h2 = 0, the
Gaussian density of y and of its error contrasts, flatness for Phi = I,
invariances, a fine-grid check of the maximiser)."""
from __future__ import annotations

import math

import numpy as np
from scipy.linalg import solve_triangular

ML, REML = 0, 1
GRID = 100
TOL = 1e-7
_GOLD = (math.sqrt(5.0) - 1.0) / 2.0


def loglik(Phi, XL, y, h2, method):
    """(log-likelihood, s2 estimate) at heritability h2; (-inf, nan) if H is not positive definite."""
    n, p = XL.shape
    H = h2 * Phi + (1.0 - h2) * np.eye(n)
    try:
        L = np.linalg.cholesky(H)
    except np.linalg.LinAlgError:
        return -math.inf, math.nan
    Xw = solve_triangular(L, XL, lower=True)
    yw = solve_triangular(L, y, lower=True)
    A = Xw.T @ Xw
    beta = np.linalg.solve(A, Xw.T @ yw)
    r = yw - Xw @ beta
    rss = float(r @ r)
    logdet_h = 2.0 * float(np.sum(np.log(np.diag(L))))
    if method == ML:
        s2 = rss / n
        return -0.5 * (n * (math.log(2.0 * math.pi * s2) + 1.0) + logdet_h), s2
    s2 = rss / (n - p)
    logdet_a = float(np.linalg.slogdet(A)[1])
    logdet_x = float(np.linalg.slogdet(XL.T @ XL)[1])
    return -0.5 * ((n - p) * (math.log(2.0 * math.pi * s2) + 1.0) + logdet_h + logdet_a - logdet_x), s2


def estimate(Phi, XL, y, method=REML):
    """(h2, s2, log-likelihood) maximising the profile likelihood over h2 in [0, 1]."""
    f = lambda h: loglik(Phi, XL, y, h, method)[0]
    hs = [i / GRID for i in range(GRID + 1)]
    ls = [f(h) for h in hs]
    best = max(range(GRID + 1), key=lambda i: (ls[i], -i))
    a, b = hs[max(best - 1, 0)], hs[min(best + 1, GRID)]
    c, d = b - _GOLD * (b - a), a + _GOLD * (b - a)
    fc, fd = f(c), f(d)
    while b - a > TOL:
        if fc >= fd:
            b, d, fd = d, c, fc
            c = b - _GOLD * (b - a)
            fc = f(c)
        else:
            a, c, fc = c, d, fd
            d = a + _GOLD * (b - a)
            fd = f(d)
    x = 0.5 * (a + b)
    lx = f(x)
    h2 = x if lx > ls[best] else hs[best]
    ll, s2 = loglik(Phi, XL, y, h2, method)
    return h2, s2, ll


def estimate_all(Phi, XL, Y, method=REML):
    """Arrays (h2, s2, loglik) for every column of Y."""
    out = np.array([estimate(Phi, XL, Y[:, j], method) for j in range(Y.shape[1])])
    return out[:, 0], out[:, 1], out[:, 2]
