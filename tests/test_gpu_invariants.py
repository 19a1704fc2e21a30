"""Invariants of the GLS solution checked on the HIP path's own outputs (both
precisions): linearity in y, equivariance under y + delta g and y + X_L gamma,
the scale law, reparametrisation of the covariates, permutation of the
individuals, and the normal-equation residual X^T M^{-1} (y - X b) = 0
(supplementary notes, section 1, equations GLS and probDef).  SE depends on
y only through nothing at all, so it must come out bitwise equal wherever only
y changes."""
import dataclasses

import numpy as np
import pytest

from synth import make_workload

from _helpers import gpu_run

pytestmark = pytest.mark.gpu
PRECS = [(0, 1e-9), (1, 1e-6)]  # (CLAK precision, bar in SE units / relative)


@dataclasses.dataclass
class Inputs:
    """A workload with replaceable pieces; genotypes optionally permuted."""
    n: int
    m: int
    t: int
    pL: int
    block: int
    Phi: np.ndarray
    XL: np.ndarray
    Y: np.ndarray
    h2: np.ndarray
    s2: np.ndarray
    base: object
    perm: np.ndarray = None

    def genotypes(self, start, count, ld=None):
        g = self.base.genotypes(start, count)
        if self.perm is not None:
            g = np.ascontiguousarray(g[:, self.perm])
        if ld is not None and ld > self.n:
            out = np.zeros((count, ld), np.uint8)
            out[:, :self.n] = g
            return out
        return g


def _inputs(t=4):
    w = make_workload(2, n=300, m=240, t=t, kin_cols=600)
    return Inputs(w.n, w.m, w.t, w.pL, w.m, w.Phi, np.asfortranarray(w.XL), np.asfortranarray(w.Y), w.h2.copy(),
                  w.s2.copy(), w)


def _run(x, prec, flags=0):
    return gpu_run(x, prec, flags=flags, block=x.m)


@pytest.mark.parametrize("prec,tol", PRECS)
def test_linearity_in_y(prec, tol):
    x = _inputs()
    rng = np.random.default_rng(5)
    y2 = np.asfortranarray(rng.standard_normal(x.Y.shape) * 3.0 + 1.0)
    print(f"linearity prec={prec}", flush=True)
    b1, se1, _ = _run(x, prec)
    b2, se2, _ = _run(dataclasses.replace(x, Y=y2), prec)
    alpha, beta = 0.7, -1.9
    b3, se3, _ = _run(dataclasses.replace(x, Y=np.asfortranarray(alpha * x.Y + beta * y2)), prec)
    assert np.array_equal(se1, se2) and np.array_equal(se1, se3)
    err = np.max(np.abs(b3 - (alpha * b1 + beta * b2)) / se1)
    print(f"linearity: max |b3 - (a b1 + c b2)| / SE = {err:.3e}")
    assert err < 3 * tol


@pytest.mark.parametrize("prec,tol", PRECS)
def test_equivariance(prec, tol):
    """y_j + delta_j g_{i_j} moves b_{i_j j} by delta_j; y + X_L gamma moves no SNP effect."""
    x = _inputs()
    print(f"equivariance prec={prec}", flush=True)
    b, se, _ = _run(x, prec)
    snps = np.array([3, 77, 150, 239])
    delta = np.array([0.25, -1.5, 4.0, 0.01])
    g = x.base.genotypes(0, x.m).astype(np.float64)
    y2 = x.Y.copy(order="F")
    for j in range(x.t):
        y2[:, j] += delta[j] * g[snps[j]]
    b2, se2, _ = _run(dataclasses.replace(x, Y=y2), prec)
    assert np.array_equal(se, se2)
    moved = b2[snps, np.arange(x.t)] - b[snps, np.arange(x.t)]
    err = np.max(np.abs(moved - delta) / se[snps, np.arange(x.t)])
    print(f"snp shift: {err:.3e}")
    assert err < 2 * tol
    gamma = np.array([[2.0, -1.0, 0.5, 3.0], [0.5, 0.5, -2.0, 1.0], [0.03, -0.01, 0.02, 0.0]])
    b3, se3, _ = _run(dataclasses.replace(x, Y=np.asfortranarray(x.Y + x.XL @ gamma)), prec)
    assert np.array_equal(se, se3)
    err = np.max(np.abs(b3 - b) / se)
    print(f"covariate shift: {err:.3e}")
    assert err < 2 * tol


@pytest.mark.parametrize("prec,tol", PRECS)
def test_scale_law(prec, tol):
    """y -> c y with s2 -> c^2 s2: b -> c b, SE -> |c| SE (model-consistent variance)."""
    x = _inputs()
    c = -2.5
    print(f"scale prec={prec}", flush=True)
    b, se, _ = _run(x, prec)
    b2, se2, _ = _run(dataclasses.replace(x, Y=np.asfortranarray(c * x.Y), s2=c * c * x.s2), prec)
    eb = np.max(np.abs(b2 - c * b) / (abs(c) * se))
    es = np.max(np.abs(se2 - abs(c) * se) / (abs(c) * se))
    print(f"scale: eps_b={eb:.3e} eps_se={es:.3e}")
    assert eb < 2 * tol and es < 2 * tol


@pytest.mark.parametrize("prec,tol", PRECS)
def test_reparametrised_covariates(prec, tol):
    """X_L -> X_L T (T invertible) spans the same space: SNP effects and SEs unchanged."""
    x = _inputs()
    T = np.array([[1.0, 0.3, -20.0], [0.0, 2.0, 0.5], [0.0, 0.0, 0.1]])
    print(f"reparametrisation prec={prec}", flush=True)
    b, se, _ = _run(x, prec)
    b2, se2, _ = _run(dataclasses.replace(x, XL=np.asfortranarray(x.XL @ T)), prec)
    eb = np.max(np.abs(b2 - b) / se)
    es = np.max(np.abs(se2 - se) / se)
    print(f"reparametrisation: eps_b={eb:.3e} eps_se={es:.3e}")
    assert eb < 2 * tol and es < 2 * tol


@pytest.mark.parametrize("prec,tol", PRECS)
def test_permuted_individuals(prec, tol):
    """Relabelling the individuals (rows of Phi, X_L, Y and genotypes) changes nothing."""
    x = _inputs()
    p = np.random.default_rng(9).permutation(x.n)
    print(f"permutation prec={prec}", flush=True)
    b, se, _ = _run(x, prec)
    xp = dataclasses.replace(x, Phi=np.ascontiguousarray(x.Phi[np.ix_(p, p)]), XL=np.asfortranarray(x.XL[p]),
                             Y=np.asfortranarray(x.Y[p]), perm=p)
    b2, se2, _ = _run(xp, prec)
    eb = np.max(np.abs(b2 - b) / se)
    es = np.max(np.abs(se2 - se) / se)
    print(f"permutation: eps_b={eb:.3e} eps_se={es:.3e}")
    assert eb < 2 * tol and es < 2 * tol


@pytest.mark.parametrize("prec,tol", PRECS)
def test_normal_equation_residual(prec, tol):
    """With the full vector b_ij: ||X^T M^{-1} (y - X b)|| / (||L^{-1} X||_F ||L^{-1} y||) ~ 0, M = L L^T."""
    from paper_1207_2169_amd import clak
    x = _inputs(t=3)
    print(f"residual prec={prec}", flush=True)
    b, se, _ = _run(x, prec, flags=clak.CLAK_OUT_FULL)
    G = x.base.genotypes(0, x.m).astype(np.float64)
    worst = 0.0
    for j in range(x.t):
        M = x.s2[j] * (x.h2[j] * x.Phi + (1.0 - x.h2[j]) * np.eye(x.n))
        L = np.linalg.cholesky(M)
        yw = np.linalg.solve(L, x.Y[:, j])
        XLw = np.linalg.solve(L, x.XL)
        Gw = np.linalg.solve(L, G.T)  # (n, m)
        for i in range(0, x.m, 7):
            Xw = np.column_stack([XLw, Gw[:, i]])
            r = Xw.T @ (yw - Xw @ b[i, j])
            worst = max(worst, np.linalg.norm(r) / (np.linalg.norm(Xw) * np.linalg.norm(yw)))
    print(f"residual: {worst:.3e}")
    assert worst < tol
