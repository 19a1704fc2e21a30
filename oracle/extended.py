"""The oracle's route in extended precision: TEST INFRASTRUCTURE ONLY (tests
may call it; the GPU library never does, and it shares no code with it).

The same definition as ``oracle.gls_cells`` (supplementary notes, section 1,
equations GLS and probDef, by the Cholesky route of the single-instance
CLAK-Chol algorithm of section 2): per trait M_j = s2 (h2 Phi + (1 - h2) I) =
L L^T, X' = L^{-1} [X_L | g], y' = L^{-1} y, S = X'^T X', b = S^{-1} X'^T y',
Var = S^{-1}, with the same relative pivot test for a degenerate SNP; every
operation in numpy ``longdouble`` (the x87 80-bit format on x86-64: a 64-bit
significand, unit roundoff 2^-64 against 2^-53 in FP64).

It serves ill-conditioned cases in which the FP64 oracle's own rounding is
larger than the parity bars: a SNP whose share of squared norm outside span(X_L)
is rho leaves the Schur complement of S with relative error about n u / rho
(u the unit roundoff), and a kernel with condition number kappa loses about
kappa n u.  Pinned by tests/test_oracle_pins.py (agreement with the FP64 oracle
on well-conditioned problems, exact rational arithmetic on small ones).
"""
from __future__ import annotations

import numpy as np

LD = np.longdouble
DEGEN_TOL = 1e-10  # relative pivot test, as the FP64 oracle


def _chol_lower(A):
    """A = L L^T, L lower triangular, column by column; None if a pivot is not positive."""
    n = A.shape[0]
    L = np.zeros_like(A)
    for j in range(n):
        d = A[j, j] - L[j, :j] @ L[j, :j]
        if not d > 0:
            return None
        L[j, j] = np.sqrt(d)
        if j + 1 < n:
            L[j + 1:, j] = (A[j + 1:, j] - L[j + 1:, :j] @ L[j, :j]) / L[j, j]
    return L


def _forward(L, B):
    """Solves L X = B (B: n x k) by forward substitution."""
    X = np.array(B, dtype=LD)
    for i in range(L.shape[0]):
        if i:
            X[i] -= L[i, :i] @ X[:i]
        X[i] /= L[i, i]
    return X


def gls_cells(Phi, XL, G, Y, h2, s2, snp_idx, trait_idx, var_paper: bool = False):
    """Extended-precision values for the cells (G[:, snp_idx[c]], Y[:, trait_idx[c]]).

    Arguments as ``oracle.gls_cells``.  Returns b (cells, p), var (cells, p, p)
    as float64 (rounded once at the end) and flag (cells,) with the FP64
    oracle's codes (0 ok, 1 degenerate SNP, 2 M_j not positive definite,
    3 covariates singular)."""
    Phi = np.asarray(Phi, dtype=LD)
    n = Phi.shape[0]
    XL = np.asarray(XL, dtype=LD).reshape(n, -1)
    G = np.asarray(G, dtype=LD).reshape(n, -1)
    Y = np.asarray(Y, dtype=LD).reshape(n, -1)
    snp = np.asarray(snp_idx, dtype=np.int64).ravel()
    tr = np.asarray(trait_idx, dtype=np.int64).ravel()
    pL = XL.shape[1]
    p = pL + 1
    b = np.full((snp.size, p), np.nan)
    var = np.full((snp.size, p, p), np.nan)
    flag = np.zeros(snp.size, dtype=np.int32)
    for j in np.unique(tr):
        cells = np.flatnonzero(tr == j)
        hj, sj = LD(float(h2[j])), LD(float(s2[j]))
        M = sj * (hj * Phi + (LD(1) - hj) * np.eye(n, dtype=LD))
        L = _chol_lower(M)
        if L is None:
            flag[cells] = 2
            continue
        cols = np.unique(snp[cells])
        W = _forward(L, np.concatenate([XL, Y[:, [j]], G[:, cols]], axis=1))
        XLp, yp, Gp = W[:, :pL], W[:, pL], W[:, pL + 1:]
        where = {int(s): k for k, s in enumerate(cols)}
        for c in cells:
            X = np.concatenate([XLp, Gp[:, [where[int(snp[c])]]]], axis=1)
            S = X.T @ X
            r = X.T @ yp
            Ls = np.zeros((p, p), dtype=LD)
            bad = 0
            for jj in range(p):
                for ii in range(jj, p):
                    v = S[ii, jj] - Ls[ii, :jj] @ Ls[jj, :jj]
                    if ii == jj:
                        if not v > LD(DEGEN_TOL) * S[jj, jj]:
                            bad = 1 if jj == p - 1 else 3
                            break
                        Ls[jj, jj] = np.sqrt(v)
                    else:
                        Ls[ii, jj] = v / Ls[jj, jj]
                if bad:
                    break
            if bad:
                flag[c] = bad
                continue
            Li = _forward(Ls, np.eye(p, dtype=LD))  # L_S^{-1}
            Sinv = Li.T @ Li                         # S^{-1} = L_S^{-T} L_S^{-1}
            bc = Sinv @ r
            b[c] = bc.astype(np.float64)
            var[c] = (Sinv * (sj if var_paper else LD(1))).astype(np.float64)
    return b, var, flag
