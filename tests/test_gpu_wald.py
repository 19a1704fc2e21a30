"""p-values of the SNP effect written by the Schur epilogue (d_pval of
clak_run_block): parity with the oracle's Wald test on the oracle's own (b,
SE), on every epilogue (FP64 grid, mixed grid of up to eleven covariates, the
OUT_FULL mixed grid with p_L > 3, the fused single-trait finish of both
precisions), both output types and padded leading dimensions; NaN exactly on
flagged cells; the pipeline writes the same p-values as the eager path.

Bar.  The p-value moves with z = b / SE: |dz| <= tol (1 + |z|) when b and SE
meet eps_b, eps_SE <= tol, so |dp| <= 2 phi(z) tol (1 + |z|), plus the
rounding of the stored value.  On the GPU's own outputs p must also equal
erfc(|b / SE| / sqrt 2) evaluated on the host to a few ulps (F64 output)."""
import math

import numpy as np
import pytest

from oracle.wald import wald
from synth import make_workload

from _helpers import gpu_run, oracle_cells

pytestmark = pytest.mark.gpu

CASES = [  # (precision, workload kwargs, plan flags, out dtype, block, ldo pad)
    (0, dict(cfg=2, n=300, m=150, t=20, kin_cols=600), 0, "f64", 64, 0),
    (0, dict(cfg=4, n=400, m=130, t=1, kin_cols=800), 0, "f32", 128, 3),
    (1, dict(cfg=2, n=300, m=333, t=37, kin_cols=600), 0, "f32", 200, 0),
    (1, dict(cfg=2, n=300, m=160, t=70, kin_cols=600), 0, "f64", 160, 5),
    (1, dict(cfg=4, n=600, m=300, t=1, kin_cols=1200), 0, "f64", 128, 0),
    (1, dict(cfg=4, n=500, m=128, t=20, kin_cols=1000), 0, "f32", 128, 0),  # p_L = 8: partial-sum epilogue
    (1, dict(cfg=4, n=500, m=128, t=20, kin_cols=1000), 2, "f64", 128, 0),  # OUT_FULL, p_L = 8
]


def _phi(z):
    return np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


@pytest.mark.parametrize("prec,kw,flags,odt,block,pad", CASES)
def test_pvalues_vs_oracle(prec, kw, flags, odt, block, pad):
    kw = dict(kw)
    w = make_workload(kw.pop("cfg"), **kw)
    print(f"wald prec={prec} n={w.n} m={w.m} t={w.t} pL={w.pL} flags={flags} out={odt}", flush=True)
    b, se, fl, pv = gpu_run(w, prec, flags=flags, block=block, out_dtype=odt, ldo_pad=pad, want_pval=True)
    bsnp = b[..., -1] if b.ndim == 3 else b
    assert (fl == 0).all() and np.isfinite(pv).all() and ((pv >= 0) & (pv <= 1)).all()
    ii, jj = np.meshgrid(np.arange(w.m), np.arange(w.t), indexing="ij")
    rb, rse, _ = oracle_cells(w, ii.ravel(), jj.ravel())
    zr, pr = wald(rb[:, -1], rse)
    tol = 1e-9 if prec == 0 else 1e-6
    eps_out = 2.0 ** -24 if odt == "f32" else 2.0 ** -53
    bound = 3.0 * 2.0 * _phi(zr) * tol * (1.0 + np.abs(zr)) + 2.0 * eps_out * pr + 1e-300
    err = np.abs(pv.ravel() - pr)
    print(f"max |p - p_ref| / bound = {np.max(err / bound):.3e}; min p = {pr.min():.3e}")
    assert np.all(err <= bound)
    if odt == "f64":
        _, pself = wald(bsnp, se)
        rel = np.abs(pv - pself) / pself
        print(f"max rel |p - erfc(|b/SE|/sqrt2)| on the GPU's own b, SE = {rel.max():.3e}")
        assert rel.max() < 1e-13


def test_pvalues_nan_on_flagged_cells():
    import torch

    from paper_1207_2169_amd import clak
    w = make_workload(2, n=200, m=8, t=3, kin_cols=400)
    g = w.genotypes(0, 8).astype(np.uint8)
    g[0] = 2
    g[2] = w.XL[:, 1].astype(np.uint8)
    g[3, 5] = 3
    print("wald flagged cells", flush=True)
    for prec in (0, 1):
        with clak.Plan(w.n, w.pL, w.t, 8, prec) as plan:
            clak.clak_set_kinship(plan.handle, torch.from_numpy(np.ascontiguousarray(w.Phi)).cuda())
            clak.clak_set_covariates(plan.handle, torch.from_numpy(np.ascontiguousarray(w.XL.T)).cuda().t())
            clak.clak_set_traits(plan.handle, torch.from_numpy(np.ascontiguousarray(w.Y.T)).cuda().t(),
                                 torch.from_numpy(w.h2).cuda(), torch.from_numpy(w.s2).cuda())
            b = torch.empty((w.t, 8), dtype=torch.float32, device="cuda")
            se, pv = torch.empty_like(b), torch.full_like(b, -1.0)
            fl = torch.empty((w.t, 8), dtype=torch.uint8, device="cuda")
            clak.clak_run_block(plan.handle, torch.from_numpy(g).cuda(), b, se, fl, pv)
            torch.cuda.synchronize()
            fl, pv = fl.cpu().numpy(), pv.cpu().numpy()
        assert (fl[:, [0, 2, 3]] != 0).all() and (fl[:, [1, 4, 5, 6, 7]] == 0).all()
        assert np.isnan(pv[fl != 0]).all() and np.isfinite(pv[fl == 0]).all()


def test_pvalues_through_the_pipeline_and_argument_checks():
    import torch

    from paper_1207_2169_amd import clak
    w = make_workload(2, n=300, m=700, t=9, kin_cols=600)
    block = 256
    print("wald pipeline", flush=True)
    with clak.Plan(w.n, w.pL, w.t, block, 1) as plan:
        clak.clak_set_kinship(plan.handle, torch.from_numpy(np.ascontiguousarray(w.Phi)).cuda())
        clak.clak_set_covariates(plan.handle, torch.from_numpy(np.ascontiguousarray(w.XL.T)).cuda().t())
        clak.clak_set_traits(plan.handle, torch.from_numpy(np.ascontiguousarray(w.Y.T)).cuda().t(),
                             torch.from_numpy(w.h2).cuda(), torch.from_numpy(w.s2).cuda())
        G = torch.from_numpy(w.genotypes(0, w.m)).cuda()
        outs = [torch.full((w.t, w.m), float("nan"), dtype=torch.float64, device="cuda") for _ in range(3)]
        for s in range(0, w.m, block):
            clak.clak_run_block(plan.handle, G[s:s + block], *(o[:, s:s + block] for o in outs[:2]), None,
                                outs[2][:, s:s + block])
        torch.cuda.synchronize()
        ref = [o.clone() for o in outs]
        for o in outs:
            o.fill_(float("nan"))
        blocks = [(G[s:s + block], outs[0][:, s:s + block], outs[1][:, s:s + block], None, outs[2][:, s:s + block])
                  for s in range(0, w.m, block)]
        pipe = clak.clak_pipeline_create(plan.handle, blocks)
        try:
            clak.clak_pipeline_launch(pipe)
            torch.cuda.synchronize()
        finally:
            clak.clak_pipeline_destroy(pipe)
        for o, r in zip(outs, ref):
            assert torch.equal(o, r)
        # a p-value buffer of another type than b and SE is refused by the binding, a misaligned one by the library
        with pytest.raises(ValueError):
            clak.clak_run_block(plan.handle, G[:block], outs[0][:, :block], outs[1][:, :block], None,
                                outs[2][:, :block].float())
        raw = torch.empty(w.t * block * 8 + 8, dtype=torch.uint8, device="cuda")
        st = clak.lib().clak_run_block(plan.handle, block, G.data_ptr(), clak.CLAK_G_U8, G.stride(0),
                                       outs[0].data_ptr(), outs[1].data_ptr(), clak.CLAK_OUT_F64, w.m, None,
                                       raw.data_ptr() + 4)
        assert st == clak.CLAK_E_ARG and b"misaligned" in clak.lib().clak_last_error()
