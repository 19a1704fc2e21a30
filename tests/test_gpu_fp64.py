"""Parity of the FP64 HIP path (CLAK_PREC_FP64) with the CPU oracle.

Tolerance: the FP64 eigen route differs from the oracle's Cholesky route only
by rounding; a CPU emulation of this route in FP64 gives eps_b ~ 1e-10 at
n = 1000, so the bar is 1e-9 in SE units for b and 1e-9 relative for SE."""
import numpy as np
import pytest

from synth import make_workload

from _helpers import errors, gpu_run, oracle_cells

pytestmark = pytest.mark.gpu
TOL = 1e-9


def _all_cells(m, t):
    ii, jj = np.meshgrid(np.arange(m), np.arange(t), indexing="ij")
    return ii.ravel(), jj.ravel()


def test_config0_full_grid():
    """n=256, m=2000, t=1: every cell against the oracle."""
    from paper_1207_2169_amd import clak
    w = make_workload(0)
    print("config 0 FP64 full grid", flush=True)
    b, se, fl = gpu_run(w, clak.CLAK_PREC_FP64, block=2000)
    ii, jj = _all_cells(w.m, w.t)
    rb, rse, rfl = oracle_cells(w, ii, jj)
    assert (rfl == 0).all() and (fl == 0).all()
    eb, es = errors(b.ravel(), se.ravel(), rb[:, -1], rse)
    print(f"eps_b={eb:.3e} eps_se={es:.3e}")
    assert eb < TOL and es < TOL


def test_multi_trait_ragged_blocks():
    """n=300 (padded to 384), m=333 in blocks of 200 and 133, t=37 (not a
    multiple of the 16-trait tile): all 12321 cells."""
    from paper_1207_2169_amd import clak
    w = make_workload(2, n=300, m=333, t=37, kin_cols=600)
    print("multi-trait ragged FP64", flush=True)
    b, se, fl = gpu_run(w, clak.CLAK_PREC_FP64, block=200)
    ii, jj = _all_cells(w.m, w.t)
    rb, rse, rfl = oracle_cells(w, ii, jj)
    assert (fl == 0).all()
    eb, es = errors(b.ravel(), se.ravel(), rb[:, -1], rse)
    print(f"eps_b={eb:.3e} eps_se={es:.3e}")
    assert eb < TOL and es < TOL


def test_full_vector_paper_variance_f32_f16_padded():
    """CLAK_OUT_FULL | CLAK_VAR_PAPER, FP32 outputs, FP16 genotypes, padded
    leading dimensions."""
    from paper_1207_2169_amd import clak
    w = make_workload(2, n=200, m=70, t=5, kin_cols=400)
    flags = clak.CLAK_OUT_FULL | clak.CLAK_VAR_PAPER
    print("full vector / paper variance FP64 path", flush=True)
    b, se, fl = gpu_run(w, clak.CLAK_PREC_FP64, flags=flags, block=70, g_dtype="f16", out_dtype="f32",
                        ldg_pad=24, ldo_pad=3)
    ii, jj = _all_cells(w.m, w.t)
    rb, rse, rfl = oracle_cells(w, ii, jj, var_paper=True)
    bf = b.reshape(-1, w.pL + 1)
    # FP32 storage of the outputs bounds the agreement at ~1e-7 relative
    scale = np.abs(rb).max(axis=1, keepdims=True) + rse[:, None]
    assert np.max(np.abs(bf - rb) / scale) < 1e-6
    assert np.max(np.abs(se.ravel() - rse) / rse) < 1e-6
    # the full vector in FP64 as well
    b64, se64, _ = gpu_run(w, clak.CLAK_PREC_FP64, flags=flags, block=70)
    scale = np.abs(rb).max(axis=1, keepdims=True) + rse[:, None]
    assert np.max(np.abs(b64.reshape(-1, w.pL + 1) - rb) / scale) < TOL


def test_eigenbasis_invariance():
    """set_eigen with sign-flipped eigenvectors gives the same b and SE."""
    from paper_1207_2169_amd import clak
    w = make_workload(2, n=160, m=40, t=6, kin_cols=320)
    ev, Z = np.linalg.eigh(w.Phi)
    flip = np.where(np.arange(w.n) % 3 == 0, -1.0, 1.0)
    print("eigenbasis invariance FP64", flush=True)
    b0, se0, _ = gpu_run(w, clak.CLAK_PREC_FP64, block=40)
    b1, se1, _ = gpu_run(w, clak.CLAK_PREC_FP64, block=40, eigen=(Z * flip, ev))
    eb, es = errors(b1.ravel(), se1.ravel(), b0.ravel(), se0.ravel())
    assert eb < TOL and es < TOL


@pytest.mark.parametrize("kw,block", [(dict(n=600, m=300, t=1, kin_cols=1200), 128),
                                      (dict(n=700, m=200, t=40, kin_cols=1400), 200)])
def test_eight_covariates(kw, block):
    """p_L = 8 (intercept, sex, age, five principal components of Phi)."""
    from paper_1207_2169_amd import clak
    w = make_workload(4, **kw)
    print(f"FP64 p_L=8 n={w.n} m={w.m} t={w.t}", flush=True)
    b, se, fl = gpu_run(w, clak.CLAK_PREC_FP64, block=block)
    ii, jj = _all_cells(w.m, w.t)
    rb, rse, rfl = oracle_cells(w, ii, jj)
    assert (fl == 0).all()
    eb, es = errors(b.ravel(), se.ravel(), rb[:, -1], rse)
    print(f"eps_b={eb:.3e} eps_se={es:.3e}")
    assert eb < TOL and es < TOL
