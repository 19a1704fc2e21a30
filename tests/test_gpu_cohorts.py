"""The batched configuration at its real shapes: eight cohorts with
n = 500 .. 4000 individuals, each with its own kinship (from 2 n genotype
columns) and covariates, t between 10 and 2000 traits (log-uniform), 5 10^4
SNPs each in blocks of 10^4, submitted as one clak_batch launch (the SNP
blocks of section 3 streamed for every cohort in one submission): five rounds,
each one launch per kernel over all eight cohorts, on three streams.  Every
cohort is checked against the oracle on a stratified sample: six traits (the
first, the last and four random ones) x 200 SNPs (block edges and random
ones), 1200 cells per cohort; every cell of every cohort must be finite and
unflagged."""
import numpy as np
import pytest

from synth import cohort_workloads

from _helpers import errors, oracle_cells

pytestmark = pytest.mark.gpu
TOL = 1e-6
BLOCK = 10_000


@pytest.mark.timeout(900)
def test_batched_cohorts_against_the_oracle():
    import torch

    from paper_1207_2169_amd import clak
    ws = cohort_workloads(m=50_000)
    print("cohorts " + ", ".join(f"(n={w.n}, t={w.t})" for w in ws), flush=True)
    plans, outs, blocks = [], [], []
    try:
        for w in ws:
            plan = clak.Plan(w.n, w.pL, w.t, BLOCK, clak.CLAK_PREC_MIXED)
            plans.append(plan)
            clak.clak_set_kinship(plan.handle, torch.from_numpy(np.ascontiguousarray(w.Phi)).cuda())
            clak.clak_set_covariates(plan.handle, torch.from_numpy(np.ascontiguousarray(w.XL.T)).cuda().t())
            clak.clak_set_traits(plan.handle, torch.from_numpy(np.ascontiguousarray(w.Y.T)).cuda().t(),
                                 torch.from_numpy(w.h2).cuda(), torch.from_numpy(w.s2).cuda())
            G = torch.from_numpy(w.genotypes(0, w.m)).cuda()
            b = torch.full((w.t, w.m), float("nan"), dtype=torch.float32, device="cuda")
            se = torch.full_like(b, float("nan"))
            fl = torch.full((w.t, w.m), 255, dtype=torch.uint8, device="cuda")
            outs.append((G, b, se, fl))
            blocks.append([(G[s:s + BLOCK], b[:, s:s + BLOCK], se[:, s:s + BLOCK], fl[:, s:s + BLOCK])
                           for s in range(0, w.m, BLOCK)])
        batch = clak.clak_batch_create([p.handle for p in plans], blocks)
        try:
            batched, rounds, streams = clak.clak_batch_get_info(batch)
            assert batched and rounds == 5 and streams == 3  # one launch per kernel and round, three streams
            clak.clak_batch_launch(batch)
            torch.cuda.synchronize()
        finally:
            clak.clak_batch_destroy(batch)
        print("batch done", flush=True)
        rng = np.random.default_rng(33)
        worst = 0.0
        for c, (w, (G, b, se, fl)) in enumerate(zip(ws, outs)):
            assert bool((fl == 0).all()), f"cohort {c}: flagged cells"
            assert bool(torch.isfinite(b).all()) and bool(torch.isfinite(se).all()), f"cohort {c}: non-finite"
            traits = np.unique(np.r_[0, w.t - 1, rng.choice(w.t, 4, replace=False)])
            edges = np.array([0, BLOCK - 1, BLOCK, 2 * BLOCK + 127, w.m - 1])
            snps = np.unique(np.r_[edges, rng.choice(w.m, 200 - edges.size, replace=False)])
            ii, jj = np.meshgrid(snps, traits, indexing="ij")
            ii, jj = ii.ravel(), jj.ravel()
            it, jt = torch.from_numpy(ii).cuda(), torch.from_numpy(jj).cuda()
            gb = b[jt, it].double().cpu().numpy()
            gs = se[jt, it].double().cpu().numpy()
            rb, rse, rfl = oracle_cells(w, ii, jj)
            assert (rfl == 0).all()
            eb, es = errors(gb, gs, rb[:, -1], rse)
            worst = max(worst, eb, es)
            print(f"cohort {c} n={w.n} t={w.t}: cells={ii.size} eps_b={eb:.3e} eps_se={es:.3e}", flush=True)
            assert eb < TOL and es < TOL
        print(f"worst over cohorts {worst:.3e}", flush=True)
    finally:
        for p in plans:
            p.close()
