"""Parity at the full workload sizes in the launch configuration the benchmark
times (the block pipeline over every SNP block, FP32 outputs), on cells
sampled uniformly and at block edges and checked one by one against the
oracle; and the large configuration (n = 10^4, p_L = 8 with five principal
components) on one block.

FP32 outputs add a relative rounding of at most 2^-24 to b and SE, i.e. at
most 6e-8 |b| / SE to eps_b; the sampled z-scores stay far below 10, so the
bar stays 1e-6."""
import numpy as np
import pytest

from synth import make_workload

from _helpers import errors, oracle_cells

pytestmark = pytest.mark.gpu
TOL = 1e-6


def _plan(w, block):
    import torch

    from paper_1207_2169_amd import clak
    plan = clak.Plan(w.n, w.pL, w.t, block, clak.CLAK_PREC_MIXED)
    clak.clak_set_kinship(plan.handle, torch.from_numpy(np.ascontiguousarray(w.Phi)).cuda())
    clak.clak_set_covariates(plan.handle, torch.from_numpy(np.ascontiguousarray(w.XL.T)).cuda().t())
    clak.clak_set_traits(plan.handle, torch.from_numpy(np.ascontiguousarray(w.Y.T)).cuda().t(),
                         torch.from_numpy(w.h2).cuda(), torch.from_numpy(w.s2).cuda())
    return plan


def _pipeline(w, block):
    """b, se (t, m) FP32 and flags (t, m) on the device, through the pipeline."""
    import torch

    from paper_1207_2169_amd import clak
    with _plan(w, block) as plan:
        G = torch.from_numpy(w.genotypes(0, w.m)).cuda()
        b = torch.full((w.t, w.m), float("nan"), dtype=torch.float32, device="cuda")
        se = torch.full_like(b, float("nan"))
        fl = torch.full((w.t, w.m), 255, dtype=torch.uint8, device="cuda")
        blocks = [(G[s:s + block], b[:, s:s + block], se[:, s:s + block], fl[:, s:s + block])
                  for s in range(0, w.m, block)]
        pipe = clak.clak_pipeline_create(plan.handle, blocks)
        try:
            clak.clak_pipeline_launch(pipe)
            torch.cuda.synchronize()
        finally:
            clak.clak_pipeline_destroy(pipe)
        del G
    return b, se, fl


def _check(w, b, se, fl, ii, jj, label):
    import torch
    assert bool((fl == 0).all()), "unexpected flagged cells"
    assert bool(torch.isfinite(b).all()) and bool(torch.isfinite(se).all())
    it = torch.from_numpy(ii).cuda()
    jt = torch.from_numpy(jj).cuda()
    bs = b[jt, it].double().cpu().numpy()
    ss = se[jt, it].double().cpu().numpy()
    rb, rse, rfl = oracle_cells(w, ii, jj)
    assert (rfl == 0).all()
    eb, es = errors(bs, ss, rb[:, -1], rse)
    print(f"{label}: cells={ii.size} eps_b={eb:.3e} eps_se={es:.3e}", flush=True)
    assert eb < TOL and es < TOL


def test_single_trait_full_size_pipeline():
    """n = 1000, m = 10^6 in 100 blocks of 10^4, t = 1."""
    w = make_workload(1)
    print(f"full size n={w.n} m={w.m} t={w.t} block={w.block}", flush=True)
    b, se, fl = _pipeline(w, w.block)
    rng = np.random.default_rng(11)
    edges = np.concatenate([[s, s + 1, s + w.block - 1] for s in range(0, w.m, w.block)])
    ii = np.unique(np.concatenate([rng.integers(0, w.m, 3000), edges]))
    _check(w, b, se, fl, ii, np.zeros_like(ii), "single trait")


def test_multi_trait_full_size_pipeline():
    """n = 1000, m = 10^5 in 10 blocks of 10^4, t = 1000."""
    w = make_workload(2)
    print(f"full size n={w.n} m={w.m} t={w.t} block={w.block}", flush=True)
    b, se, fl = _pipeline(w, w.block)
    rng = np.random.default_rng(12)
    traits = np.unique(np.concatenate([rng.choice(w.t, 150, replace=False), [0, 63, 64, 999]]))
    ii = rng.integers(0, w.m, 20 * traits.size)
    jj = np.repeat(traits, 20)
    e_i = np.array([0, 9999, 10000, 99999])
    ii = np.concatenate([ii, np.repeat(e_i, 4)])
    jj = np.concatenate([jj, np.tile([0, 63, 64, 999], e_i.size)])
    _check(w, b, se, fl, ii, jj, "multi trait")


@pytest.mark.timeout(900)
def test_large_configuration_full_block():
    """n = 10^4, p_L = 8 (intercept, sex, age, five principal components),
    kinship from 2 10^4 columns, t = 1000 traits: one full block of 2 10^4 SNPs
    through the pipeline, FP32 outputs.  The oracle takes minutes per trait at
    this n, so its values for 20 random traits x 500 random SNPs (every pair)
    were written by tests/golden/make_c4_sample.py (oracle and input generators
    only); the regenerated inputs are first checked against the fingerprints
    stored with them.  Every cell of the block must be finite and unflagged."""
    import os

    import torch
    golden = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c4_sample.npz"))
    w = make_workload(4, m=20_000)
    print(f"large n={w.n} p_L={w.pL} m={w.m} t={w.t}", flush=True)
    traits = golden["traits"]
    idx = np.array([0, 1, 17, 4321, w.n - 1])
    fp = {"phi_trace": np.trace(w.Phi), "phi_entries": w.Phi[idx, idx[::-1]], "xl_colsum": w.XL.sum(0),
          "y_colsum": w.Y[:, traits].sum(0), "h2": w.h2[traits], "s2": w.s2[traits]}
    for k, v in fp.items():
        ref = golden["fp_" + k]
        # principal components may come out with either sign (b_snp and SE do not depend on it)
        v, ref = (np.abs(v), np.abs(ref)) if k == "xl_colsum" else (v, ref)
        assert np.allclose(v, ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max()), k
    b, se, fl = _pipeline(w, 20_000)
    assert bool((fl == 0).all()) and bool(torch.isfinite(b).all()) and bool(torch.isfinite(se).all())
    it = torch.from_numpy(golden["snp"]).cuda()
    jt = torch.from_numpy(golden["trait"]).cuda()
    gb = b[jt, it].double().cpu().numpy()
    gs = se[jt, it].double().cpu().numpy()
    assert (golden["flag"] == 0).all()
    eb, es = errors(gb, gs, golden["b"], golden["se"])
    print(f"large: cells={gb.size} eps_b={eb:.3e} eps_se={es:.3e}", flush=True)
    assert eb < TOL and es < TOL
