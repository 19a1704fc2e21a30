"""The launch-parameter tuner: every tunable choice leaves the results bitwise
unchanged, clak_autotune computes the block like clak_run_block, writes its
choice to the cache file and reads it back on the next call."""
import numpy as np
import pytest

from synth import make_workload

pytestmark = pytest.mark.gpu


def _plan(w, block, flags=0):
    import torch

    from paper_1207_2169_amd import clak
    plan = clak.Plan(w.n, w.pL, w.t, block, clak.CLAK_PREC_MIXED, flags)
    clak.clak_set_kinship(plan.handle, torch.from_numpy(np.ascontiguousarray(w.Phi)).cuda())
    clak.clak_set_covariates(plan.handle, torch.from_numpy(np.ascontiguousarray(w.XL.T)).cuda().t())
    clak.clak_set_traits(plan.handle, torch.from_numpy(np.ascontiguousarray(w.Y.T)).cuda().t(),
                         torch.from_numpy(w.h2).cuda(), torch.from_numpy(w.s2).cuda())
    return plan


def _outputs(w):
    import torch
    b = torch.full((w.t, w.m), float("nan"), dtype=torch.float64, device="cuda")
    return b, torch.full_like(b, float("nan")), torch.full((w.t, w.m), 255, dtype=torch.uint8, device="cuda")


# n_pad = 256, 384, 512: 4, 6 and 8 K slices of 64 (every remainder of the
# three- and four-slot rings of the direct-load rotations); CLAK-Chol rotates
# triangular tiles of 1 to n_pad / 64 slices; p_L = 8 (workload 4) gives the
# single-trait epilogue its largest per-wave-row partials
@pytest.mark.parametrize("t,n,chol,config", [(1, 300, False, 2), (150, 300, False, 2), (1, 200, False, 2),
                                             (1, 450, False, 2), (1, 450, True, 2), (1, 450, False, 4)])
def test_every_tuning_is_bitwise_identical(t, n, chol, config):
    import torch

    from paper_1207_2169_amd import clak
    w = make_workload(config, n=n, m=700, t=t, kin_cols=2 * n)
    print(f"tuning sweep t={t} n={n} chol={chol} p_L={w.pL}", flush=True)
    G = torch.from_numpy(w.genotypes(0, w.m)).cuda()
    with _plan(w, w.m, clak.CLAK_CHOL if chol else 0) as plan:
        ref = _outputs(w)
        clak.clak_run_block(plan.handle, G, *ref)
        torch.cuda.synchronize()
        assert bool(torch.isfinite(ref[0]).all()) and bool((ref[2] == 0).all())
        for cfg in range(11):
            for rg in (1, 2, 4, 8):
                for tt in ((0, 32, 64) if t > 1 else (0,)):
                    for xt in ((1, 2, 4, 8) if t > 1 else (0,)):
                        clak.clak_plan_set_tuning(plan.handle, cfg, rg, tt, xt)
                        out = _outputs(w)
                        clak.clak_run_block(plan.handle, G, *out)
                        torch.cuda.synchronize()
                        for a, r in zip(out, ref):
                            assert torch.equal(a, r), (cfg, rg, tt, xt)


def test_autotune_matches_run_block_and_uses_cache(tmp_path):
    import torch

    from paper_1207_2169_amd import clak
    w = make_workload(2, n=300, m=1000, t=100, kin_cols=600)
    print("autotune", flush=True)
    G = torch.from_numpy(w.genotypes(0, w.m)).cuda()
    cache = tmp_path / "clak_tune.txt"
    with _plan(w, w.m) as plan:
        ref = _outputs(w)
        clak.clak_run_block(plan.handle, G, *ref)
        out = _outputs(w)
        clak.clak_autotune(plan.handle, G, *out, cache_path=str(cache))
        torch.cuda.synchronize()
        for a, r in zip(out, ref):
            assert torch.equal(a, r)
        tuned = clak.clak_plan_get_tuning(plan.handle)
        # 0 keeps the built-in choice (no candidate more than 2 % faster)
        assert tuned[0] in range(11) and tuned[1] in (0, 1, 2, 4, 8) and tuned[2] in (0, 32, 64)
        assert tuned[3] in (0, 1, 2, 4, 8)
        lines = cache.read_text().splitlines()
        assert len(lines) == 1 and lines[0].startswith("gfx950")
        assert " n_pad=384 p_L=3 t=100 m_blk=1000 blocks=1 flags=0x0 " in lines[0]
    with _plan(w, w.m) as plan2:  # a new plan takes the cached choice without timing
        out2 = _outputs(w)
        clak.clak_autotune(plan2.handle, G, *out2, cache_path=str(cache))
        torch.cuda.synchronize()
        assert clak.clak_plan_get_tuning(plan2.handle) == tuned
        assert cache.read_text().splitlines() == lines
        for a, r in zip(out2, ref):
            assert torch.equal(a, r)


@pytest.mark.parametrize("t", [1, 40])
def test_pipelined_autotune(tmp_path, t):
    """clak_autotune_pipeline times pipelined passes over four blocks: the
    outputs equal the eager blocks' bitwise, the choice is cached per shape
    (with the number of blocks) and taken back by a new plan."""
    import torch

    from paper_1207_2169_amd import clak
    w = make_workload(2, n=300, m=1024, t=t, kin_cols=600)
    print(f"pipelined autotune t={t}", flush=True)
    G = torch.from_numpy(w.genotypes(0, w.m)).cuda()
    cache = tmp_path / "clak_tune.txt"
    block = 256

    def blocks(out):
        return [(G[s:s + block],) + tuple(o[:, s:s + block] for o in out) for s in range(0, w.m, block)]

    with _plan(w, block) as plan:
        ref = _outputs(w)
        for blk in blocks(ref):
            clak.clak_run_block(plan.handle, *blk)
        out = _outputs(w)
        clak.clak_autotune_pipeline(plan.handle, blocks(out), cache_path=str(cache))
        torch.cuda.synchronize()
        for a, r in zip(out, ref):
            assert torch.equal(a, r)
        tuned = clak.clak_plan_get_tuning(plan.handle)
        lines = cache.read_text().splitlines()
        assert len(lines) == 1 and f" m_blk={block} blocks=4 " in lines[0]
    with _plan(w, block) as plan2:
        out2 = _outputs(w)
        clak.clak_autotune_pipeline(plan2.handle, blocks(out2), cache_path=str(cache))
        torch.cuda.synchronize()
        assert clak.clak_plan_get_tuning(plan2.handle) == tuned and cache.read_text().splitlines() == lines
        for a, r in zip(out2, ref):
            assert torch.equal(a, r)


# Single-trait plans over blocks of at least 8192 SNPs take 64 x 256 rotation
# tiles by default (CLAK-Chol's triangular ones with one XCD row group).  n = 126 (p_L = 3) and n = 1020 (p_L = 8) put the
# U^T rows in the extra 64-row tile; n = 1000 keeps them in the padding rows.
# The default must equal, bitwise, the 64 x 128 configurations (the
# register-staged one and the four-slot ring) and a 64 x 64 one, over a full
# block and a ragged one.
@pytest.mark.parametrize("n,config,chol", [(126, 2, False), (1000, 2, False), (1000, 4, False), (1020, 4, False),
                                          (126, 2, True), (1000, 2, True)])
def test_wide_default_rotation_is_bitwise_identical(n, config, chol):
    import torch

    from paper_1207_2169_amd import clak
    block = 8192
    w = make_workload(config, n=n, m=block + 300, t=1, kin_cols=2 * n)
    print(f"wide default rotation n={n} p_L={w.pL} chol={chol}", flush=True)
    G = torch.from_numpy(w.genotypes(0, w.m)).cuda()

    def run(plan):
        out = _outputs(w)
        for s in range(0, w.m, block):
            clak.clak_run_block(plan.handle, G[s:s + block], *(o[:, s:s + block] for o in out))
        torch.cuda.synchronize()
        return out

    with _plan(w, block, clak.CLAK_CHOL if chol else 0) as plan:
        ref = run(plan)
        assert bool(torch.isfinite(ref[0]).all()) and bool((ref[2] == 0).all())
        for cfg in (5, 9, 7, 10):
            clak.clak_plan_set_tuning(plan.handle, cfg, 2, 0, 0)
            out = run(plan)
            for a, r in zip(out, ref):
                assert torch.equal(a, r), cfg
