"""Parity of the GPU variance-component estimates (clak_estimate_vc) with the
oracle's (oracle/vc.py): ML and REML, several covariate counts, a ragged n,
the t = 1000, n = 1000 multi-trait shape on sampled traits, the error paths,
and the hand-over of the estimates to clak_set_traits.

Both sides run the same search (grid, then golden section), so h2 agrees to
about the resolution of the search; the log-likelihood at the two maximisers
agrees to rounding (the maximum is flat), and the GPU's (s2, l) must equal the
oracle's profile values at the GPU's own h2 to rounding."""
import math

import numpy as np
import pytest

from oracle import vc
from synth import make_workload

pytestmark = pytest.mark.gpu

H2_TOL = 2e-5      # search resolution (bracket width 1e-7, flat maximum)
LL_TOL = 1e-10     # relative, maximised log-likelihood
PROF_TOL = 1e-9    # relative, (s2, l) at the same h2


def _covariates(n, pL, seed):
    rng = np.random.default_rng(seed)
    X = np.ones((n, pL))
    if pL > 1:
        X[:, 1:] = rng.standard_normal((n, pL - 1)) * np.linspace(0.5, 3.0, pL - 1)
    return X


def _gpu_vc(Phi, XL, Y, method, precision=0, outs=None):
    import torch

    from paper_1207_2169_amd import clak

    dev = torch.device("cuda")
    n, pL = XL.shape
    t = Y.shape[1]
    with clak.Plan(n, pL, t, 64, precision) as plan:
        clak.clak_set_kinship(plan.handle, torch.from_numpy(np.ascontiguousarray(Phi)).to(dev))
        clak.clak_set_covariates(plan.handle, torch.from_numpy(np.ascontiguousarray(XL.T)).to(dev).t())
        Yd = torch.from_numpy(np.ascontiguousarray(Y.T)).to(dev).t()
        h2, s2, ll = clak.clak_estimate_vc(plan.handle, Yd, method, *(outs or (None, None, None)))
        torch.cuda.synchronize()
        return h2.cpu().numpy(), s2.cpu().numpy(), ll.cpu().numpy()


def _compare(Phi, XL, Y, method, h2, s2, ll, traits):
    worst = [0.0, 0.0, 0.0]
    for j in traits:
        oh2, os2, oll = vc.estimate(Phi, XL, Y[:, j], method)
        assert abs(h2[j] - oh2) < H2_TOL, (j, h2[j], oh2)
        assert abs(ll[j] - oll) < LL_TOL * abs(oll), (j, ll[j], oll)
        pll, ps2 = vc.loglik(Phi, XL, Y[:, j], float(h2[j]), method)
        assert abs(ll[j] - pll) < PROF_TOL * abs(pll) and abs(s2[j] - ps2) < PROF_TOL * ps2, (j, ll[j], pll, s2[j], ps2)
        worst = [max(worst[0], abs(h2[j] - oh2)), max(worst[1], abs(ll[j] - oll) / abs(oll)),
                 max(worst[2], abs(s2[j] - ps2) / ps2)]
    print(f"max |dh2| = {worst[0]:.2e}, max rel dl = {worst[1]:.2e}, max rel ds2 at same h2 = {worst[2]:.2e}")


@pytest.mark.parametrize("method", [vc.ML, vc.REML])
@pytest.mark.parametrize("n,pL", [(300, 3), (257, 1), (333, 6)])
def test_vc_parity(method, n, pL):
    w = make_workload(2, n=n, m=4, t=8, kin_cols=2 * n)
    XL = w.XL if pL == w.pL else _covariates(n, pL, 11)
    print(f"vc parity method={method} n={n} pL={pL}", flush=True)
    h2, s2, ll = _gpu_vc(w.Phi, XL, w.Y, method)
    assert np.all((h2 >= 0) & (h2 <= 1)) and np.all(s2 > 0)
    _compare(w.Phi, XL, w.Y, method, h2, s2, ll, range(w.t))


def test_vc_boundary_maxima_and_mixed_plan():
    """Traits whose maximum sits at h2 = 0 (pure noise) or near 1 come out on the same side as the oracle;
    a MIXED-precision plan gives bitwise the same estimates (the set-up is FP64 in both)."""
    n = 280
    w = make_workload(2, n=n, m=4, t=2, kin_cols=2 * n)
    rng = np.random.default_rng(4)
    L = np.linalg.cholesky(w.Phi)
    Y = np.column_stack([rng.standard_normal(n), rng.standard_normal(n) * 0.05 + L @ rng.standard_normal(n),
                         w.Y[:, 0], w.Y[:, 1]]) + 2.0
    print("vc boundary", flush=True)
    res = _gpu_vc(w.Phi, w.XL, Y, vc.REML)
    _compare(w.Phi, w.XL, Y, vc.REML, *res, range(Y.shape[1]))
    res2 = _gpu_vc(w.Phi, w.XL, Y, vc.REML, precision=1)
    for a, b in zip(res, res2):
        assert np.array_equal(a, b)


def test_vc_multitrait_shape_sampled():
    """n = 1000, t = 1000 (the many-trait shape): all traits on the GPU, sampled traits against the oracle."""
    w = make_workload(2, n=1000, m=4, t=1000, kin_cols=2000)
    for method in (vc.ML, vc.REML):
        print(f"vc n=1000 t=1000 method={method}", flush=True)
        h2, s2, ll = _gpu_vc(w.Phi, w.XL, w.Y, method)
        assert np.all(np.isfinite(h2)) and np.all(np.isfinite(ll)) and np.all(s2 > 0)
        _compare(w.Phi, w.XL, w.Y, method, h2, s2, ll, [0, 577])
    # the estimates track the heritabilities the phenotypes were drawn with
    assert np.corrcoef(h2, w.h2)[0, 1] > 0.7


def test_vc_errors_and_nonfinite_trait():
    import torch

    from paper_1207_2169_amd import clak

    dev = torch.device("cuda")
    w = make_workload(2, n=200, m=4, t=3, kin_cols=400)
    Y = np.ascontiguousarray(w.Y.T).copy()
    Y[1, 17] = math.nan
    with clak.Plan(w.n, w.pL, w.t, 64, 0) as plan:
        Yd = torch.from_numpy(Y).to(dev).t()
        with pytest.raises(clak.ClakError) as e:
            clak.clak_estimate_vc(plan.handle, Yd)
        assert e.value.status == clak.CLAK_E_STATE
        clak.clak_set_kinship(plan.handle, torch.from_numpy(np.ascontiguousarray(w.Phi)).to(dev))
        clak.clak_set_covariates(plan.handle, torch.from_numpy(np.ascontiguousarray(w.XL.T)).to(dev).t())
        with pytest.raises(clak.ClakError) as e:
            clak.clak_estimate_vc(plan.handle, Yd, 7)
        assert e.value.status == clak.CLAK_E_ARG
        outs = [torch.full((w.t,), -1.0, dtype=torch.float64, device=dev) for _ in range(3)]
        with pytest.raises(clak.ClakError) as e:
            clak.clak_estimate_vc(plan.handle, Yd, clak.CLAK_VC_REML, *outs)
        assert e.value.status == clak.CLAK_E_ARG
        h2, s2, ll = (x.cpu().numpy() for x in outs)
    assert np.isnan(h2[1]) and np.isnan(s2[1]) and np.isnan(ll[1])
    for j in (0, 2):
        oh2, _, oll = vc.estimate(w.Phi, w.XL, w.Y[:, j], vc.REML)
        assert abs(h2[j] - oh2) < H2_TOL and abs(ll[j] - oll) < LL_TOL * abs(oll)


def test_vc_feeds_set_traits():
    """estimate -> set_traits -> run_block equals run_block with the oracle's estimates handed in,
    and a later estimate_vc call leaves the ready traits untouched."""
    import torch

    from paper_1207_2169_amd import clak

    dev = torch.device("cuda")
    w = make_workload(2, n=240, m=96, t=4, kin_cols=480)
    G = torch.from_numpy(w.genotypes(0, w.m)).to(dev)

    def scan(plan):
        b = torch.empty((w.t, w.m), dtype=torch.float64, device=dev)
        se = torch.empty_like(b)
        clak.clak_run_block(plan.handle, G, b, se)
        torch.cuda.synchronize()
        return b.cpu().numpy(), se.cpu().numpy()

    print("vc -> set_traits", flush=True)
    with clak.Plan(w.n, w.pL, w.t, w.m, 0) as plan:
        clak.clak_set_kinship(plan.handle, torch.from_numpy(np.ascontiguousarray(w.Phi)).to(dev))
        clak.clak_set_covariates(plan.handle, torch.from_numpy(np.ascontiguousarray(w.XL.T)).to(dev).t())
        Yd = torch.from_numpy(np.ascontiguousarray(w.Y.T)).to(dev).t()
        h2, s2, _ = clak.clak_estimate_vc(plan.handle, Yd, clak.CLAK_VC_REML)
        clak.clak_set_traits(plan.handle, Yd, h2, s2)
        b1, se1 = scan(plan)
        clak.clak_estimate_vc(plan.handle, torch.zeros_like(Yd) + 1.0 + torch.arange(w.n, device=dev)[:, None] * 1e-3,
                              clak.CLAK_VC_ML)
        b2, se2 = scan(plan)
        oh2, os2, _ = vc.estimate_all(w.Phi, w.XL, w.Y, vc.REML)
        clak.clak_set_traits(plan.handle, Yd, torch.from_numpy(oh2).to(dev), torch.from_numpy(os2).to(dev))
        b3, se3 = scan(plan)
    assert np.array_equal(b1, b2) and np.array_equal(se1, se2)
    # the two estimates differ by the search resolution only: effects agree far below their SE
    assert np.max(np.abs(b1 - b3) / se3) < 1e-3 and np.max(np.abs(se1 - se3) / se3) < 1e-3
