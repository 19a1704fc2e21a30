"""Parity of the mixed-precision HIP path (CLAK_PREC_MIXED: int8 digit-plane
MFMA with exact int32 accumulation, FP64 Schur solve) with the CPU oracle.

Bar: the stated target, eps_b = max |b - b_ref| / SE_ref <= 1e-6 and
eps_SE = max |SE - SE_ref| / SE_ref <= 1e-6.  A CPU emulation of this
encoding (four digit planes of Z^T, four of x and of the operand, products
of weight >= 256^-4 dropped) predicts ~4e-9 at n = 1000."""
import numpy as np

import oracle
import pytest

from synth import make_workload

from _helpers import errors, gpu_run, oracle_cells

pytestmark = pytest.mark.gpu
TOL = 1e-6


def _all_cells(m, t):
    ii, jj = np.meshgrid(np.arange(m), np.arange(t), indexing="ij")
    return ii.ravel(), jj.ravel()


@pytest.mark.parametrize("cfg,kw,block", [
    (0, dict(), 2000),
    (2, dict(n=300, m=333, t=37, kin_cols=600), 200),
    (2, dict(n=1000, m=150, t=20), 150),
    (4, dict(n=600, m=300, t=1, kin_cols=1200), 128),
    (4, dict(n=700, m=200, t=40, kin_cols=1400), 200),
])
def test_mixed_vs_oracle(cfg, kw, block):
    from paper_1207_2169_amd import clak
    w = make_workload(cfg, **kw)
    print(f"mixed cfg={cfg} n={w.n} m={w.m} t={w.t}", flush=True)
    b, se, fl = gpu_run(w, clak.CLAK_PREC_MIXED, block=block)
    ii, jj = _all_cells(w.m, w.t)
    rb, rse, rfl = oracle_cells(w, ii, jj)
    assert (fl == 0).all()
    eb, es = errors(b.ravel(), se.ravel(), rb[:, -1], rse)
    print(f"eps_b={eb:.3e} eps_se={es:.3e}")
    assert eb < TOL and es < TOL


def test_mixed_wide_trait_tiles_sampled():
    """m = 2048 SNPs x t = 1000 traits in one block: 16 SNP tiles x 16 tiles of
    64 traits fill exactly one dispatch round, so the grid kernel takes its
    64-trait tile (two trait groups per work-group).  Every cell must be
    finite and unflagged; 30000 sampled cells, plus all cells of the traits
    and SNPs at tile edges and the ragged trait tail, match the oracle."""
    from paper_1207_2169_amd import clak
    w = make_workload(2, n=256, m=2048, t=1000, kin_cols=512)
    print(f"mixed wide tiles n={w.n} m={w.m} t={w.t}", flush=True)
    b, se, fl = gpu_run(w, clak.CLAK_PREC_MIXED, block=2048, out_dtype="f64")
    assert (fl == 0).all() and np.isfinite(b).all() and np.isfinite(se).all()
    rng = np.random.default_rng(7)
    ii = rng.integers(0, w.m, 30000)
    jj = rng.integers(0, w.t, 30000)
    edge_t = np.array([0, 31, 32, 63, 64, 127, 128, 959, 960, 991, 992, 999])
    edge_s = np.array([0, 31, 32, 127, 128, 1023, 1024, 2047])
    e1 = np.meshgrid(np.arange(0, w.m, 37), edge_t, indexing="ij")
    e2 = np.meshgrid(edge_s, np.arange(w.t), indexing="ij")
    ii = np.concatenate([ii, e1[0].ravel(), e2[0].ravel()])
    jj = np.concatenate([jj, e1[1].ravel(), e2[1].ravel()])
    rb, rse, rfl = oracle_cells(w, ii, jj)
    eb, es = errors(b[ii, jj], se[ii, jj], rb[:, -1], rse)
    print(f"eps_b={eb:.3e} eps_se={es:.3e} cells={ii.size}")
    assert eb < TOL and es < TOL


@pytest.mark.parametrize("cfg,kw", [(2, dict(n=200, m=70, t=5, kin_cols=400)),
                                    (4, dict(n=300, m=90, t=6, kin_cols=600))])
def test_mixed_full_vector_and_paper_variance(cfg, kw):
    from paper_1207_2169_amd import clak
    w = make_workload(cfg, **kw)
    flags = clak.CLAK_OUT_FULL | clak.CLAK_VAR_PAPER
    print(f"mixed full vector / paper variance cfg={cfg} p_L={w.pL}", flush=True)
    b, se, fl = gpu_run(w, clak.CLAK_PREC_MIXED, flags=flags, block=w.m, g_dtype="f16")
    ii, jj = _all_cells(w.m, w.t)
    rb, rse, rfl = oracle_cells(w, ii, jj, var_paper=True)
    # each covariate effect in units of its own standard error (the diagonal of
    # the oracle's model-consistent Var(b) = (X^T M^-1 X)^-1)
    G = np.concatenate([w.genotypes(int(s), 1) for s in range(w.m)]).T.astype(np.float64)
    _, var, _ = oracle.gls_cells(w.Phi, w.XL, G, w.Y, w.h2, w.s2, ii, jj)
    se_cov = np.sqrt(np.diagonal(var, axis1=1, axis2=2)[:, :-1])
    bf = b.reshape(-1, w.pL + 1)
    eb_cov = float(np.max(np.abs(bf[:, :-1] - rb[:, :-1]) / se_cov))
    print(f"eps_b snp={np.max(np.abs(bf[:, -1] - rb[:, -1]) / rse):.3e} covariates={eb_cov:.3e}", flush=True)
    assert np.max(np.abs(bf[:, -1] - rb[:, -1]) / rse) < TOL
    assert np.max(np.abs(se.ravel() - rse) / rse) < TOL
    assert eb_cov < TOL
