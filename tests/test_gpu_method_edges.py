"""The method's edge cases on the HIP path against the oracle, in both
precisions (supplementary notes, section 1: h2 in [0, 1]; section 3 with
equation Eig0: any orthonormal eigenbasis of Phi gives the same M_j^{-1}):

* h2 = 0 (M_j = s2 I, ordinary least squares) and h2 = 1 (M_j = s2 Phi);
* a nearly singular Phi (eigenvalues down to 1e-7) at h2 = 1, 0.999 and 0.5;
* eigenbases of a Phi with a 40-fold eigenvalue that differ by a random
  rotation of that eigenspace (and by column signs), passed through
  clak_set_eigen, against the oracle and against each other;
* the degeneracy threshold (reading R8): a SNP whose share of squared norm
  outside the covariates is 1e-8 is solved, one at 1e-12 is flagged, by the
  GPU and the oracle alike.

Bars: 1e-9 (FP64 path) and 1e-6 (mixed) in SE units, except where stated.
The two ill-conditioned cases are compared with the oracle's route in
extended precision (oracle.extended), since there the FP64 oracle's own
rounding exceeds the FP64 bar."""
import dataclasses

import numpy as np
import pytest

from synth import make_workload

from _helpers import errors, gpu_run, oracle_cells

pytestmark = pytest.mark.gpu
PRECS = [(0, 1e-9), (1, 1e-6)]


def _all(m, t):
    ii, jj = np.meshgrid(np.arange(m), np.arange(t), indexing="ij")
    return ii.ravel(), jj.ravel()


def _compare(w, prec, tol, label, **kw):
    b, se, fl = gpu_run(w, prec, block=w.m, **kw)
    ii, jj = _all(w.m, w.t)
    rb, rse, rfl = oracle_cells(w, ii, jj)
    assert np.array_equal(fl.ravel() == 0, rfl == 0), "degeneracy flags differ"
    ok = rfl == 0
    eb, es = errors(b.ravel()[ok], se.ravel()[ok], rb[ok, -1], rse[ok])
    print(f"{label} prec={prec}: eps_b={eb:.3e} eps_se={es:.3e} cells={int(ok.sum())}", flush=True)
    assert eb < tol and es < tol
    return b, se


@pytest.mark.parametrize("prec,tol", PRECS)
def test_heritability_at_zero_and_one(prec, tol):
    w = make_workload(2, n=300, m=200, t=6, kin_cols=600)
    w.h2 = np.array([0.0, 1.0, 0.0, 1.0, 0.5, 1.0])
    w.s2 = np.array([1.0, 1.0, 2.5, 0.4, 1.0, 3.0])
    _compare(w, prec, tol, "h2 in {0, 1}")


def _extended_cells(w):
    """b, SE and flags of every cell from the extended-precision route of the oracle."""
    from oracle import extended
    ii, jj = _all(w.m, w.t)
    G = np.concatenate([w.genotypes(0, w.m)]).T.astype(np.float64)
    b, var, fl = extended.gls_cells(w.Phi, w.XL, G, w.Y, w.h2, w.s2, ii, jj)
    return b[:, -1], np.sqrt(var[:, -1, -1]), fl


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("lo,hi", [(1e-5, 1e-4), (1e-7, 1e-5)])
def test_nearly_singular_kinship(prec, lo, hi):
    """Phi with its 30 smallest eigenvalues set to lo .. hi (condition number
    kappa ~ 3 / lo) at h2 = 1, 0.999, 0.5, 1, 0; the phenotypes are drawn from
    that model.  Reference: the oracle's route in extended precision; the FP64
    oracle's own distance from it is checked against its rounding bound
    n kappa u.  Bars: the usual 1e-9 (FP64) and 1e-6 (mixed), raised to
    n kappa u where the backward error of the factorisation of Phi (the
    eigensolver's, like the oracle's Cholesky, is about n u ||Phi||, i.e.
    n kappa u relative to the smallest eigenvalues that weigh most at
    h2 ~ 1) is larger."""
    w = make_workload(2, n=300, m=200, t=5, kin_cols=600)
    ev, V = np.linalg.eigh(w.Phi)
    ev[:30] = np.geomspace(lo, hi, 30)
    w.Phi = np.asfortranarray(0.5 * ((V * ev) @ V.T + ((V * ev) @ V.T).T))
    w.h2 = np.array([1.0, 0.999, 0.5, 1.0, 0.0])
    rng = np.random.default_rng(3)
    LP = V * np.sqrt(ev)
    w.Y = np.asfortranarray(w.XL @ rng.normal(size=(w.pL, w.t)) + np.sqrt(w.s2) * (
        np.sqrt(w.h2) * (LP @ rng.normal(size=(w.n, w.t))) + np.sqrt(1 - w.h2) * rng.normal(size=(w.n, w.t))))
    kappa = ev.max() / ev.min()
    u = 2.0 ** -53
    tol = max(1e-9 if prec == 0 else 1e-6, w.n * kappa * u)
    print(f"condition number of Phi {kappa:.2e}, bar {tol:.2e}", flush=True)
    b, se, fl = gpu_run(w, prec, block=w.m)
    rb, rse, rfl = _extended_cells(w)
    assert (rfl == 0).all() and (fl == 0).all()
    eb, es = errors(b.ravel(), se.ravel(), rb, rse)
    ii, jj = _all(w.m, w.t)
    ob, ose, _ = oracle_cells(w, ii, jj)
    eo = float(np.max(np.abs(ob[:, -1] - rb) / rse))
    print(f"nearly singular Phi prec={prec}: eps_b={eb:.3e} eps_se={es:.3e}; FP64 oracle vs extended {eo:.3e}",
          flush=True)
    assert eb < tol and es < tol
    assert eo < kappa * w.n * u  # the FP64 oracle within its own rounding bound


def _degenerate_eigenbases(seed=21, n=280, mult=40):
    """A Phi with one eigenvalue of multiplicity `mult` and two orthonormal
    eigenbases of it that differ by a random rotation of that eigenspace and
    by the signs of the other eigenvectors."""
    w = make_workload(2, n=n, m=160, t=4, kin_cols=2 * n)
    ev, V = np.linalg.eigh(w.Phi)
    ev[100:100 + mult] = 0.37
    rng = np.random.default_rng(seed)
    Q, R = np.linalg.qr(rng.standard_normal((mult, mult)))
    Q = Q * np.sign(np.diag(R))
    V2 = V.copy()
    V2[:, 100:100 + mult] = V[:, 100:100 + mult] @ Q
    V2 = V2 * np.where(rng.random(n) < 0.5, -1.0, 1.0)
    w.Phi = np.asfortranarray((V * ev) @ V.T)
    w.Phi = np.asfortranarray(0.5 * (w.Phi + w.Phi.T))
    return w, ev, V, V2


@pytest.mark.parametrize("prec,tol", PRECS)
def test_eigenbasis_invariance_in_a_degenerate_eigenspace(prec, tol):
    w, ev, V, V2 = _degenerate_eigenbases()
    assert np.abs(V2[:, 100:140].T @ V[:, 100:140] - np.eye(40)).max() > 0.1  # the bases really differ
    b1, se1 = _compare(w, prec, tol, "eigenbasis 1", eigen=(V, ev))
    b2, se2 = _compare(w, prec, tol, "eigenbasis 2 (rotated degenerate eigenspace)", eigen=(V2, ev))
    d = float(np.max(np.abs(b1 - b2) / se1))
    print(f"|b(basis 1) - b(basis 2)| / SE = {d:.3e}", flush=True)
    assert d < 2 * tol and float(np.max(np.abs(se1 - se2) / se1)) < 2 * tol


def _near_collinear_covariate(w, rho, seed=5):
    """X_L = [1, sex, g0 + delta r] for SNP 0's genotypes g0 and a random r,
    with delta set so that g0's share of squared norm outside span(X_L) is
    rho; returns that share as recomputed by a least-squares solve."""
    g0 = w.genotypes(0, 1)[0].astype(np.float64)
    r = np.random.default_rng(seed).standard_normal(w.n)
    delta = np.sqrt(rho) * np.linalg.norm(g0) / np.linalg.norm(r)
    for _ in range(3):  # the projector depends (weakly) on delta
        XL = np.c_[np.ones(w.n), w.XL[:, 1], g0 + delta * r]
        res = g0 - XL @ np.linalg.lstsq(XL, g0, rcond=None)[0]
        share = res @ res / (g0 @ g0)
        delta *= np.sqrt(rho / share)
    XL = np.c_[np.ones(w.n), w.XL[:, 1], g0 + delta * r]
    res = g0 - XL @ np.linalg.lstsq(XL, g0, rcond=None)[0]
    return np.asfortranarray(XL), res @ res / (g0 @ g0)


@pytest.mark.parametrize("prec", [0, 1])
def test_degeneracy_threshold_agrees_with_the_oracle(prec):
    """A SNP nearly in span(X_L): share 1e-8 is solved, share 1e-12 is flagged,
    by the GPU and the oracle alike (reading R8).  Values are compared with
    the oracle's route in extended precision: the FP64 oracle itself forms
    the Schur complement of this SNP with a relative error of about n u /
    share (~3e-6 here).  Bars: 1e-8 (FP64 path) and 1e-6 (mixed; its rotation
    and centring use the same digit-encoded Z^T, so the centred SNP carries no
    error from the collinear part)."""
    base = make_workload(2, n=256, m=64, t=3, kin_cols=512)
    for rho, flagged in ((1e-8, False), (1e-12, True)):
        XL, share = _near_collinear_covariate(base, rho)
        assert 0.5 * rho < share < 2 * rho
        w = dataclasses.replace(base, XL=XL)
        b, se, fl = gpu_run(w, prec, block=w.m)
        ii, jj = _all(w.m, w.t)
        _, _, ofl = oracle_cells(w, ii, jj)
        rb, rse, rfl = _extended_cells(w)
        rfl, ofl = rfl.reshape(w.m, w.t), ofl.reshape(w.m, w.t)
        print(f"share={share:.2e} prec={prec}: gpu flags {fl[0].tolist()} oracle flags {ofl[0].tolist()} "
              f"extended {rfl[0].tolist()}", flush=True)
        assert (ofl[0] != 0).all() == flagged and (rfl[0] != 0).all() == flagged and (fl[0] != 0).all() == flagged
        assert (ofl[1:] == 0).all() and (rfl[1:] == 0).all() and (fl[1:] == 0).all()
        if not flagged:
            rb, rse = rb.reshape(w.m, w.t), rse.reshape(w.m, w.t)
            e0 = float(np.max(np.abs(b[0] - rb[0]) / rse[0]))
            eb, es = errors(b.ravel(), se.ravel(), rb.ravel(), rse.ravel())
            print(f"  near-collinear SNP: eps_b={e0:.3e}; all cells eps_b={eb:.3e} eps_se={es:.3e}", flush=True)
            assert e0 < (1e-8 if prec == 0 else 1e-6)
            assert eb < (1e-8 if prec == 0 else 1e-6) and es < (1e-8 if prec == 0 else 1e-6)
        else:
            assert np.isnan(b[0]).all() and np.isnan(se[0]).all()
