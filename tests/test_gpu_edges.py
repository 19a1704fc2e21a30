"""Edge sizes of the HIP path against the oracle: the smallest systems (n just
above p_L, one SNP, one trait), sizes on either side of the paddings of the
individuals (128), the SNP blocks (256) and the traits (128), and p_L at both
ends of each precision's range."""
import numpy as np
import pytest

from synth import make_workload

from _helpers import errors, gpu_run, oracle_cells

pytestmark = pytest.mark.gpu


def _check(w, prec, block, tol=None, **kw):
    b, se, fl = gpu_run(w, prec, block=block, **kw)
    ii, jj = np.meshgrid(np.arange(w.m), np.arange(w.t), indexing="ij")
    rb, rse, rfl = oracle_cells(w, ii.ravel(), jj.ravel())
    ok = (fl.ravel() == 0)
    assert np.array_equal(ok, rfl == 0), "degeneracy flags differ"
    eb, es = errors(b.ravel()[ok], se.ravel()[ok], rb[ok, -1], rse[ok])
    tol = tol or (1e-9 if prec == 0 else 1e-6)
    print(f"n={w.n} m={w.m} t={w.t} pL={w.pL} block={block} prec={prec}: eps_b={eb:.3e} eps_se={es:.3e}")
    assert eb < tol and es < tol


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("n,m,t,block", [(6, 1, 1, 1), (7, 3, 2, 2), (12, 5, 1, 5)])
def test_smallest_systems(prec, n, m, t, block):
    w = make_workload(2 if t > 1 else 1, n=n, m=m, t=t, kin_cols=4 * n)
    print(f"smallest n={n} m={m} t={t}", flush=True)
    _check(w, prec, block)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("n", [127, 128, 129])
def test_individual_padding(prec, n):
    w = make_workload(2, n=n, m=300, t=5, kin_cols=2 * n)
    print(f"padding n={n}", flush=True)
    _check(w, prec, 300)


# Single trait, mixed path: the p_L + 1 rows U^T of the rotation sit in the
# zero padding rows n .. n + p_L when n + p_L + 1 <= n_pad, else in one more
# row tile; both sides of that boundary for p_L = 3 (workload 1) and p_L = 8
# (workload 4), by CLAK-Eig and by CLAK-Chol.
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("n,config,chol", [(124, 1, False), (125, 1, False), (128, 1, False), (129, 1, False),
                                           (119, 4, False), (120, 4, False), (124, 1, True), (128, 1, True)])
def test_individual_padding_single_trait(prec, n, config, chol):
    from paper_1207_2169_amd import clak
    w = make_workload(config, n=n, m=300, t=1, kin_cols=2 * n)
    print(f"single-trait padding n={n} p_L={w.pL} chol={chol}", flush=True)
    _check(w, prec, 300, flags=clak.CLAK_CHOL if chol else 0)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("m,block", [(257, 255), (513, 256), (520, 257)])
def test_block_padding_single_trait(prec, m, block):
    w = make_workload(1, n=200, m=m, kin_cols=400)
    print(f"blocks m={m} block={block}", flush=True)
    _check(w, prec, block)


@pytest.mark.parametrize("t", [127, 128, 129])
def test_trait_padding(t):
    w = make_workload(2, n=160, m=130, t=t, kin_cols=320)
    print(f"traits t={t}", flush=True)
    _check(w, 1, 130)


@pytest.mark.parametrize("prec,pL", [(0, 1), (1, 1), (1, 8), (0, 16)])
def test_covariate_count_limits(prec, pL):
    w = make_workload(2, n=220, m=140, t=9, kin_cols=440)
    rng = np.random.default_rng(pL)
    XL = np.ones((w.n, pL))
    if pL > 1:
        XL[:, 1:] = rng.standard_normal((w.n, pL - 1))
    w.XL = XL
    w.pL = pL
    print(f"p_L={pL} prec={prec}", flush=True)
    _check(w, prec, 140)
