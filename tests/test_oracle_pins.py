"""Pins of the CPU oracle against facts that do not come from the oracle itself.

The paper prints no worked numeric example, so every pin is a closed form, a
special case that reduces to a textbook or library routine, exact rational
arithmetic, brute force on tiny inputs, or an invariant of the GLS estimator
(supplementary notes, section 1, equations GLS and probDef).  Each is chosen so
that a dropped term, a wrong sign or index, or a transposed operand in the
oracle fails at least one of them.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle

RTOL = 1e-11


def _rand_problem(rng, n, pL, t=1, ng=3, kin=None):
    A = rng.normal(size=(n, kin or 2 * n))
    Phi = A @ A.T / A.shape[1] + 0.05 * np.eye(n)
    XL = np.c_[np.ones(n), rng.normal(size=(n, pL - 1)) * 3 + 1] if pL else np.zeros((n, 0))
    G = rng.integers(0, 3, size=(n, ng)).astype(float)
    Y = rng.normal(size=(n, t)) * 2 + 5
    h2 = rng.uniform(0.05, 0.95, t)
    s2 = rng.uniform(0.5, 2.0, t)
    return Phi, XL, G, Y, h2, s2


def _cells(ng, t):
    ii, jj = np.meshgrid(np.arange(ng), np.arange(t), indexing="ij")
    return ii.ravel(), jj.ravel()


def _gls_numpy(Phi, X, y, h2, s2):
    """GLS through an explicit library solve with M (library routine special case)."""
    n = Phi.shape[0]
    M = s2 * (h2 * Phi + (1 - h2) * np.eye(n))
    MiX = np.linalg.solve(M, X)
    Miy = np.linalg.solve(M, y)
    S = X.T @ MiX
    return np.linalg.solve(S, X.T @ Miy), np.linalg.inv(S)


# --------------------------------------------------------------------------- closed forms


def test_ols_closed_form_at_h2_zero():
    """h2 = 0 gives M = s2 I, so with X_L = [1] the SNP effect is the simple
    regression slope, the intercept ybar - b gbar, and Var = s2 (X^T X)^{-1}
    with Var(b) = s2 / Sxx written out by hand."""
    rng = np.random.default_rng(1)
    n = 40
    Phi, _, G, Y, _, _ = _rand_problem(rng, n, 0, ng=4)
    XL = np.ones((n, 1))
    s2 = 2.3
    b, var, flag = oracle.gls_cells(Phi, XL, G, Y, [0.0], [s2], np.arange(4), np.zeros(4, int))
    assert (flag == 0).all()
    y = Y[:, 0]
    for i in range(4):
        g = G[:, i]
        gb, yb = g.mean(), y.mean()
        sxx = ((g - gb) ** 2).sum()
        slope = ((g - gb) * (y - yb)).sum() / sxx
        np.testing.assert_allclose(b[i, 1], slope, rtol=RTOL)
        np.testing.assert_allclose(b[i, 0], yb - slope * gb, rtol=RTOL)
        # model-consistent Var = (X^T M^{-1} X)^{-1} = s2 (X^T X)^{-1}
        np.testing.assert_allclose(var[i, 1, 1], s2 / sxx, rtol=RTOL)
        np.testing.assert_allclose(var[i, 0, 1], -s2 * gb / sxx, rtol=RTOL)
        np.testing.assert_allclose(var[i, 0, 0], s2 * (1.0 / n + gb * gb / sxx), rtol=RTOL)


def test_identity_kinship_is_ols():
    """Phi = I makes M = s2 I for every h2: ordinary least squares (numpy lstsq)."""
    rng = np.random.default_rng(2)
    n, pL = 30, 3
    _, XL, G, Y, h2, s2 = _rand_problem(rng, n, pL, t=2)
    b, var, flag = oracle.gls_cells(np.eye(n), XL, G, Y, h2, s2, *_cells(3, 2))
    for c, (i, j) in enumerate(zip(*_cells(3, 2))):
        X = np.c_[XL, G[:, i]]
        ref, *_ = np.linalg.lstsq(X, Y[:, j], rcond=None)
        np.testing.assert_allclose(b[c], ref, rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(var[c], s2[j] * np.linalg.inv(X.T @ X), rtol=1e-10)


def test_diagonal_kinship_is_weighted_least_squares():
    """Diagonal Phi: weights 1 / (s2 (h2 phi_kk + 1 - h2)), i.e. lstsq on
    rows scaled by the square roots of the weights."""
    rng = np.random.default_rng(3)
    n, pL = 25, 2
    _, XL, G, Y, h2, s2 = _rand_problem(rng, n, pL, t=2)
    phi = rng.uniform(0.2, 3.0, n)
    b, var, flag = oracle.gls_cells(np.diag(phi), XL, G, Y, h2, s2, *_cells(3, 2))
    for c, (i, j) in enumerate(zip(*_cells(3, 2))):
        wts = 1.0 / (s2[j] * (h2[j] * phi + 1 - h2[j]))
        X = np.c_[XL, G[:, i]] * np.sqrt(wts)[:, None]
        ref, *_ = np.linalg.lstsq(X, Y[:, j] * np.sqrt(wts), rcond=None)
        np.testing.assert_allclose(b[c], ref, rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(var[c], np.linalg.inv(X.T @ X), rtol=1e-10)


# --------------------------------------------------------------------------- brute force


def _gauss_jordan_inverse(A):
    """Explicit inverse by Gauss-Jordan elimination with partial pivoting,
    row operations in numpy long double."""
    n = A.shape[0]
    W = np.concatenate([A.astype(np.longdouble), np.eye(n, dtype=np.longdouble)], axis=1)
    for col in range(n):
        piv = col + int(np.argmax(np.abs(W[col:, col])))
        W[[col, piv]] = W[[piv, col]]
        W[col] /= W[col, col]
        for r in range(n):
            if r != col:
                W[r] -= W[r, col] * W[col]
    return W[:, n:]


@pytest.mark.parametrize("n,pL,seed", [(8, 2, 4), (12, 3, 5), (16, 3, 6), (16, 1, 7)])
def test_explicit_inverse_brute_force(n, pL, seed):
    """b = (X^T M^{-1} X)^{-1} X^T M^{-1} y with M^{-1} formed explicitly."""
    rng = np.random.default_rng(seed)
    Phi, XL, G, Y, h2, s2 = _rand_problem(rng, n, pL, t=2)
    b, var, flag = oracle.gls_cells(Phi, XL, G, Y, h2, s2, *_cells(3, 2))
    for c, (i, j) in enumerate(zip(*_cells(3, 2))):
        M = s2[j] * (h2[j] * Phi + (1 - h2[j]) * np.eye(n))
        Mi = _gauss_jordan_inverse(M)
        X = np.c_[XL, G[:, i]].astype(np.longdouble)
        y = Y[:, j].astype(np.longdouble)
        S = X.T @ Mi @ X
        Si = _gauss_jordan_inverse(S)
        ref = Si @ (X.T @ Mi @ y)
        np.testing.assert_allclose(b[c], ref.astype(float), rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(var[c], Si.astype(float), rtol=1e-10, atol=1e-14)


def _frac_solve(A, B):
    """Exact solution of A X = B over the rationals (Gauss-Jordan)."""
    n = len(A)
    W = [list(A[r]) + list(B[r]) for r in range(n)]
    for col in range(n):
        piv = next(r for r in range(col, n) if W[r][col] != 0)
        W[col], W[piv] = W[piv], W[col]
        inv = 1 / W[col][col]
        W[col] = [v * inv for v in W[col]]
        for r in range(n):
            if r != col and W[r][col] != 0:
                f = W[r][col]
                W[r] = [a - f * bb for a, bb in zip(W[r], W[col])]
    return [row[n:] for row in W]


@pytest.mark.parametrize("n,seed", [(4, 11), (5, 12), (6, 13)])
def test_exact_rational(n, seed):
    """Rational Phi, h2, s2, X and y: the GLS estimate and its covariance are
    rational; computed exactly with fractions and compared at 1e-13."""
    rng = np.random.default_rng(seed)
    A = rng.integers(-3, 4, size=(n, n + 2))
    Phi = [[Fraction(int(v), n + 2) for v in row] for row in (A @ A.T)]
    for k in range(n):
        Phi[k][k] += Fraction(1, 10)
    h2, s2 = Fraction(3, 7), Fraction(5, 4)
    XL = [[Fraction(1), Fraction(int(rng.integers(0, 2)))] for _ in range(n)]
    g = [Fraction(int(v)) for v in rng.integers(0, 3, n)]
    y = [Fraction(int(v), 3) for v in rng.integers(-20, 20, n)]
    M = [[s2 * (h2 * Phi[r][c] + ((1 - h2) if r == c else 0)) for c in range(n)] for r in range(n)]
    X = [XL[r] + [g[r]] for r in range(n)]
    MiX = _frac_solve(M, X)
    Miy = [row[0] for row in _frac_solve(M, [[v] for v in y])]
    p = 3
    S = [[sum(X[r][a] * MiX[r][c] for r in range(n)) for c in range(p)] for a in range(p)]
    rhs = [[sum(X[r][a] * Miy[r] for r in range(n))] for a in range(p)]
    bex = [row[0] for row in _frac_solve(S, rhs)]
    Sinv = _frac_solve(S, [[Fraction(int(a == c)) for c in range(p)] for a in range(p)])
    f = lambda M_: np.array([[float(v) for v in row] for row in M_])
    b, var, flag = oracle.gls_cells(f(Phi), f(XL), np.array([[float(v)] for v in g]),
                                    np.array([[float(v)] for v in y]), [float(h2)], [float(s2)],
                                    [0], [0])
    np.testing.assert_allclose(b[0], [float(v) for v in bex], rtol=1e-13)
    np.testing.assert_allclose(var[0], f(Sinv), rtol=1e-13)


# --------------------------------------------------------------------------- invariants


def _problem(seed=21, n=60, pL=3, t=3, ng=5):
    rng = np.random.default_rng(seed)
    return _rand_problem(rng, n, pL, t=t, ng=ng)


def test_normal_equation_residual():
    """X_i^T M_j^{-1} (y_j - X_i b_ij) = 0 (normalised)."""
    Phi, XL, G, Y, h2, s2 = _problem()
    n = Phi.shape[0]
    b, var, flag = oracle.gls_cells(Phi, XL, G, Y, h2, s2, *_cells(5, 3))
    for c, (i, j) in enumerate(zip(*_cells(5, 3))):
        M = s2[j] * (h2[j] * Phi + (1 - h2[j]) * np.eye(n))
        L = np.linalg.cholesky(M)
        X = np.c_[XL, G[:, i]]
        Xp = np.linalg.solve(L, X)
        yp = np.linalg.solve(L, Y[:, j])
        res = Xp.T @ (yp - Xp @ b[c])
        assert np.abs(res).max() / (np.linalg.norm(Xp) * np.linalg.norm(yp)) < 1e-13


def test_matches_library_gls():
    """Against an explicit numpy GLS with M solves (library special case)."""
    Phi, XL, G, Y, h2, s2 = _problem(seed=22)
    b, var, flag = oracle.gls_cells(Phi, XL, G, Y, h2, s2, *_cells(5, 3))
    for c, (i, j) in enumerate(zip(*_cells(5, 3))):
        rb, rv = _gls_numpy(Phi, np.c_[XL, G[:, i]], Y[:, j], h2[j], s2[j])
        np.testing.assert_allclose(b[c], rb, rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(var[c], rv, rtol=1e-10, atol=1e-14)


def test_linearity_in_y():
    Phi, XL, G, Y, h2, s2 = _problem(seed=23, t=2)
    h2 = np.array([h2[0]] * 3)
    s2 = np.array([s2[0]] * 3)
    al, be = 1.7, -0.6
    Y3 = np.c_[Y, al * Y[:, 0] + be * Y[:, 1]]
    b, var, flag = oracle.gls_cells(Phi, XL, G, Y3, h2, s2, *_cells(5, 3))
    b = b.reshape(5, 3, -1)
    var = var.reshape(5, 3, *var.shape[1:])
    np.testing.assert_allclose(b[:, 2], al * b[:, 0] + be * b[:, 1], rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(var[:, 0], var[:, 1], rtol=1e-12)
    np.testing.assert_allclose(var[:, 0], var[:, 2], rtol=1e-12)


def test_equivariance():
    """y + delta g_i shifts only the SNP effect by delta; y + X_L gamma shifts
    only the covariate effects by gamma."""
    Phi, XL, G, Y, h2, s2 = _problem(seed=24, t=1)
    i = 2
    delta, gam = 0.37, np.array([1.5, -0.25, 0.8])
    Yx = np.c_[Y[:, 0], Y[:, 0] + delta * G[:, i], Y[:, 0] + XL @ gam]
    b, var, flag = oracle.gls_cells(Phi, XL, G, Yx, [h2[0]] * 3, [s2[0]] * 3, [i, i, i], [0, 1, 2])
    np.testing.assert_allclose(b[1, -1], b[0, -1] + delta, rtol=1e-10)
    np.testing.assert_allclose(b[1, :-1], b[0, :-1], rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(b[2, :-1], b[0, :-1] + gam, rtol=1e-10)
    np.testing.assert_allclose(b[2, -1], b[0, -1], rtol=1e-9, atol=1e-11)


def test_scale_law():
    """y -> c y with s2 -> c^2 s2: b -> c b and the standard errors -> |c| SE."""
    Phi, XL, G, Y, h2, s2 = _problem(seed=25, t=1)
    c = -3.5
    b0, v0, _ = oracle.gls_cells(Phi, XL, G, Y, h2, s2, np.arange(5), np.zeros(5, int))
    b1, v1, _ = oracle.gls_cells(Phi, XL, G, c * Y, h2, c * c * s2, np.arange(5), np.zeros(5, int))
    np.testing.assert_allclose(b1, c * b0, rtol=1e-10)
    se0 = np.sqrt(np.diagonal(v0, axis1=1, axis2=2))
    se1 = np.sqrt(np.diagonal(v1, axis1=1, axis2=2))
    np.testing.assert_allclose(se1, abs(c) * se0, rtol=1e-10)


def test_reparametrisation_and_permutation():
    """X_L -> X_L T leaves the SNP effect and its SE unchanged; so does any
    permutation of the individuals applied to Phi, X_L, g and y."""
    Phi, XL, G, Y, h2, s2 = _problem(seed=26, t=2)
    rng = np.random.default_rng(0)
    T = np.triu(rng.normal(size=(3, 3))) + 3 * np.eye(3)
    perm = rng.permutation(Phi.shape[0])
    cells = _cells(5, 2)
    b0, v0, _ = oracle.gls_cells(Phi, XL, G, Y, h2, s2, *cells)
    b1, v1, _ = oracle.gls_cells(Phi, XL @ T, G, Y, h2, s2, *cells)
    b2, v2, _ = oracle.gls_cells(Phi[np.ix_(perm, perm)], XL[perm], G[perm], Y[perm], h2, s2, *cells)
    np.testing.assert_allclose(b1[:, -1], b0[:, -1], rtol=1e-9)
    np.testing.assert_allclose(v1[:, -1, -1], v0[:, -1, -1], rtol=1e-9)
    np.testing.assert_allclose(b2, b0, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(v2, v0, rtol=1e-9)


def test_centering_invariance():
    """g -> g - X_L gamma (any gamma) leaves the SNP effect and SE unchanged."""
    Phi, XL, G, Y, h2, s2 = _problem(seed=27, t=2)
    gam = np.array([0.7, -1.1, 0.05])
    Gc = G - (XL @ gam)[:, None]
    cells = _cells(5, 2)
    b0, v0, _ = oracle.gls_cells(Phi, XL, G, Y, h2, s2, *cells)
    b1, v1, _ = oracle.gls_cells(Phi, XL, Gc, Y, h2, s2, *cells)
    np.testing.assert_allclose(b1[:, -1], b0[:, -1], rtol=1e-9)
    np.testing.assert_allclose(v1[:, -1, -1], v0[:, -1, -1], rtol=1e-9)


def test_trait_specific_covariance_and_cell_order():
    """Every cell uses its own trait's M_j, independent of the order of cells."""
    Phi, XL, G, Y, h2, s2 = _problem(seed=28, t=3)
    ii, jj = _cells(5, 3)
    rng = np.random.default_rng(1)
    perm = rng.permutation(ii.size)
    b0, v0, _ = oracle.gls_cells(Phi, XL, G, Y, h2, s2, ii, jj)
    b1, v1, _ = oracle.gls_cells(Phi, XL, G, Y, h2, s2, ii[perm], jj[perm])
    np.testing.assert_array_equal(b1, b0[perm])
    for c in range(ii.size):
        bj, _ = _gls_numpy(Phi, np.c_[XL, G[:, ii[c]]], Y[:, jj[c]], h2[jj[c]], s2[jj[c]])
        np.testing.assert_allclose(b0[c], bj, rtol=1e-10, atol=1e-12)


def test_variance_conventions():
    """var_paper multiplies the model-consistent covariance by s2_j."""
    Phi, XL, G, Y, h2, s2 = _problem(seed=29, t=2)
    cells = _cells(5, 2)
    _, v0, _ = oracle.gls_cells(Phi, XL, G, Y, h2, s2, *cells)
    _, v1, _ = oracle.gls_cells(Phi, XL, G, Y, h2, s2, *cells, var_paper=True)
    np.testing.assert_allclose(v1, v0 * s2[cells[1]][:, None, None], rtol=1e-14)


# --------------------------------------------------------------------------- degenerate cases


def test_degenerate_snps_flagged():
    """A monomorphic SNP (collinear with the intercept), an all-zero SNP and a
    SNP equal to a covariate column make S singular: NaN and a flag."""
    Phi, XL, G, Y, h2, s2 = _problem(seed=30, t=1)
    XL[:, 1] = (np.arange(XL.shape[0]) % 2).astype(float)
    n = Phi.shape[0]
    Gd = np.c_[np.ones(n) * 2, np.zeros(n), XL[:, 1], 2 * XL[:, 1] - XL[:, 0], G[:, 0]]
    b, var, flag = oracle.gls_cells(Phi, XL, Gd, Y, h2, s2, np.arange(5), np.zeros(5, int))
    assert list(flag) == [oracle.SNP_DEGENERATE] * 4 + [oracle.OK]
    assert np.isnan(b[:4]).all() and np.isnan(var[:4]).all()
    assert np.isfinite(b[4]).all()


def _near_collinear_snps(rho, seed=33, n=60):
    """A problem and SNP columns g = X_L gamma + eps r, r orthogonal to X_L in
    the M^{-1} inner product, with eps chosen so that the share of g's
    M^{-1}-weighted squared norm outside span(X_L) is rho[k] for column k;
    returns the problem and that share recomputed with numpy solves."""
    rng = np.random.default_rng(seed)
    Phi, XL, _, Y, h2, s2 = _rand_problem(rng, n, 3, t=1, ng=1)
    M = s2[0] * (h2[0] * Phi + (1 - h2[0]) * np.eye(n))
    Mi = lambda v: np.linalg.solve(M, v)
    P = XL @ np.linalg.solve(XL.T @ Mi(XL), XL.T @ Mi(np.eye(n)))  # M^{-1}-orthogonal projector on X_L
    base = XL @ np.array([1.3, -0.7, 0.02])
    r = rng.normal(size=n)
    r = r - P @ r
    A, R = base @ Mi(base), r @ Mi(r)
    G = np.stack([base + np.sqrt(q * A / (R * (1 - q))) * r for q in rho], 1)
    share = np.array([(g - P @ g) @ Mi(g - P @ g) / (g @ Mi(g)) for g in G.T])
    return Phi, XL, G, Y, h2, s2, share


RHO_KEPT = [1e-8, 1e-9, 2e-10]    # above the degeneracy threshold 1e-10
RHO_FLAGGED = [5e-11, 1e-12, 0.0]  # at or below it


def _threshold_pin_holds():
    """The oracle flags a cell exactly when the share of the SNP's
    M^{-1}-weighted squared norm outside the covariates is <= 1e-10 (the
    relative pivot test of reading R8), at shares a factor of two and more on
    either side of the threshold; the kept cells match a numpy solve."""
    rho = RHO_KEPT + RHO_FLAGGED
    Phi, XL, G, Y, h2, s2, share = _near_collinear_snps(rho)
    np.testing.assert_allclose(share[:len(RHO_KEPT)], RHO_KEPT, rtol=1e-3)
    assert (share[len(RHO_KEPT):] <= 0.6e-10).all()
    b, var, flag = oracle.gls_cells(Phi, XL, G, Y, h2, s2, np.arange(len(rho)), np.zeros(len(rho), int))
    want = [oracle.OK] * len(RHO_KEPT) + [oracle.SNP_DEGENERATE] * len(RHO_FLAGGED)
    if list(flag) != want:
        return False
    for c in range(len(RHO_KEPT)):
        rb, rv = _gls_numpy(Phi, np.c_[XL, G[:, c]], Y[:, 0], h2[0], s2[0])
        # conditioning grows like 1 / rho: relative accuracy ~1e-16 / rho
        if not np.allclose(b[c, -1], rb[-1], rtol=1e-5) or not np.allclose(var[c, -1, -1], rv[-1, -1], rtol=1e-5):
            return False
    return bool(np.isnan(b[len(RHO_KEPT):]).all())


def test_degeneracy_threshold():
    assert _threshold_pin_holds()


@pytest.mark.parametrize("tol", ["1e-3", "1e-14"])
def test_degeneracy_threshold_pin_catches_a_wrong_constant(tmp_path, tol):
    """A mutant oracle built with another pivot threshold fails the pin."""
    import ctypes

    from oracle.build import build
    path = build(out=str(tmp_path / "liboracle_mutant.so"), defines=[f"ORACLE_DEGEN_TOL={tol}"])
    good = oracle._lib()
    mutant = ctypes.CDLL(path)
    mutant.oracle_gls.argtypes = good.oracle_gls.argtypes
    mutant.oracle_gls.restype = good.oracle_gls.restype
    try:
        oracle._LIB = mutant
        assert not _threshold_pin_holds()
    finally:
        oracle._LIB = good
    assert _threshold_pin_holds()


def test_boundaries_and_not_spd():
    """h2 = 0 and h2 = 1 are valid for a positive-definite Phi; h2 = 1 with an
    indefinite Phi makes M_j indefinite, flagged per cell."""
    Phi, XL, G, Y, h2, s2 = _problem(seed=31, t=2)
    b, var, flag = oracle.gls_cells(Phi, XL, G, Y, [0.0, 1.0], s2, *_cells(5, 2))
    assert (flag == 0).all()
    for c, (i, j) in enumerate(zip(*_cells(5, 2))):
        rb, _ = _gls_numpy(Phi, np.c_[XL, G[:, i]], Y[:, j], [0.0, 1.0][j], s2[j])
        np.testing.assert_allclose(b[c], rb, rtol=1e-9, atol=1e-12)
    w, V = np.linalg.eigh(Phi)
    w[0] = -0.5
    Pbad = (V * w) @ V.T
    b, var, flag = oracle.gls_cells(Pbad, XL, G, Y, [1.0, 0.5], s2, *_cells(5, 2))
    f = flag.reshape(5, 2)
    assert (f[:, 0] == oracle.M_NOT_SPD).all() and np.isnan(b.reshape(5, 2, -1)[:, 0]).all()
    # h2 = 0.5 keeps 0.5*w + 0.5 > 0 for w = -0.5?  0.25 - ... : 0.5*(-0.5)+0.5 = 0.25 > 0
    assert (f[:, 1] == oracle.OK).all()


def test_rejects_bad_arguments():
    Phi, XL, G, Y, h2, s2 = _problem(seed=32, t=1)
    with pytest.raises(ValueError):
        oracle.gls_cells(Phi, XL, G, Y, h2, s2, [7], [0])
    with pytest.raises(ValueError):
        oracle.gls_cells(Phi, XL, G, Y, h2, s2, [0], [3])

# --------------------------------------------------------------------------- extended-precision route


def test_extended_precision_route_matches_the_oracle():
    """oracle.extended (the same route in 64-bit-significand arithmetic) agrees
    with the FP64 oracle on well-conditioned problems."""
    from oracle import extended
    Phi, XL, G, Y, h2, s2 = _problem(seed=40, n=50, t=3, ng=4)
    cells = _cells(4, 3)
    b, var, flag = oracle.gls_cells(Phi, XL, G, Y, h2, s2, *cells)
    be, ve, fe = extended.gls_cells(Phi, XL, G, Y, h2, s2, *cells)
    assert (flag == fe).all()
    np.testing.assert_allclose(be, b, rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(ve, var, rtol=1e-11, atol=1e-15)
    bp, vp, _ = extended.gls_cells(Phi, XL, G, Y, h2, s2, *cells, var_paper=True)
    np.testing.assert_allclose(vp, ve * s2[cells[1]][:, None, None], rtol=1e-15)


@pytest.mark.parametrize("n,seed", [(5, 14), (6, 15)])
def test_extended_precision_route_exact_rational(n, seed):
    """Rational inputs exactly representable in FP64: the extended route's
    b and Var match the exact rational solution to about 2^-60."""
    from oracle import extended
    rng = np.random.default_rng(seed)
    A = rng.integers(-3, 4, size=(n, n + 2))
    Phi = [[Fraction(int(v), 8) for v in row] for row in (A @ A.T)]
    for k in range(n):
        Phi[k][k] += Fraction(1, 4)
    h2, s2 = Fraction(3, 8), Fraction(5, 4)
    XL = [[Fraction(1), Fraction(int(rng.integers(0, 2)))] for _ in range(n)]
    g = [Fraction(int(v)) for v in rng.integers(0, 3, n)]
    y = [Fraction(int(v), 4) for v in rng.integers(-20, 20, n)]
    M = [[s2 * (h2 * Phi[r][c] + ((1 - h2) if r == c else 0)) for c in range(n)] for r in range(n)]
    X = [XL[r] + [g[r]] for r in range(n)]
    MiX = _frac_solve(M, X)
    Miy = [row[0] for row in _frac_solve(M, [[v] for v in y])]
    p = 3
    S = [[sum(X[r][a] * MiX[r][c] for r in range(n)) for c in range(p)] for a in range(p)]
    rhs = [[sum(X[r][a] * Miy[r] for r in range(n))] for a in range(p)]
    bex = [row[0] for row in _frac_solve(S, rhs)]
    f = lambda M_: np.array([[float(v) for v in row] for row in M_])
    b, var, flag = extended.gls_cells(f(Phi), f(XL), np.array([[float(v)] for v in g]),
                                      np.array([[float(v)] for v in y]), [float(h2)], [float(s2)], [0], [0])
    assert flag[0] == 0
    np.testing.assert_allclose(b[0], [float(v) for v in bex], rtol=4e-16)


def test_extended_precision_route_near_collinear():
    """At shares 1e-8 .. 2e-10 outside span(X_L) the extended route flags as
    the FP64 oracle does and matches the numpy solve of the pin above; the
    FP64 oracle's distance from it stays within its rounding bound
    10 n u / share in SE units."""
    from oracle import extended
    rho = RHO_KEPT + RHO_FLAGGED
    Phi, XL, G, Y, h2, s2, share = _near_collinear_snps(rho)
    cells = (np.arange(len(rho)), np.zeros(len(rho), int))
    b, var, flag = oracle.gls_cells(Phi, XL, G, Y, h2, s2, *cells)
    be, ve, fe = extended.gls_cells(Phi, XL, G, Y, h2, s2, *cells)
    assert list(fe) == list(flag)
    n, u = Phi.shape[0], 2.0 ** -53
    for c, q in enumerate(RHO_KEPT):
        se = np.sqrt(ve[c, -1, -1])
        assert abs(b[c, -1] - be[c, -1]) / se < 10 * n * u / q
