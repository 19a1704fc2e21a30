"""Pipelines and cohort batches against the eager per-block
path, determinism, and independence of the block split."""
import numpy as np
import pytest

from synth import make_workload

pytestmark = pytest.mark.gpu


def _setup(w, prec, block, flags=0):
    import torch

    from paper_1207_2169_amd import clak
    plan = clak.Plan(w.n, w.pL, w.t, block, prec, flags)
    clak.clak_set_kinship(plan.handle, torch.from_numpy(np.ascontiguousarray(w.Phi)).cuda())
    clak.clak_set_covariates(plan.handle, torch.from_numpy(np.ascontiguousarray(w.XL.T)).cuda().t())
    clak.clak_set_traits(plan.handle, torch.from_numpy(np.ascontiguousarray(w.Y.T)).cuda().t(),
                         torch.from_numpy(w.h2).cuda(), torch.from_numpy(w.s2).cuda())
    return plan


def _blocks(w, block, dtype):
    import torch
    G = torch.from_numpy(w.genotypes(0, w.m)).cuda()
    b = torch.full((w.t, w.m), float("nan"), dtype=dtype, device="cuda")
    se = torch.full_like(b, float("nan"))
    fl = torch.full((w.t, w.m), 255, dtype=torch.uint8, device="cuda")
    blocks = [(G[s:s + block], b[:, s:s + block], se[:, s:s + block], fl[:, s:s + block])
              for s in range(0, w.m, block)]
    return G, b, se, fl, blocks


def _eager(plan, blocks):
    import torch

    from paper_1207_2169_amd import clak
    for G, b, se, fl in blocks:
        clak.clak_run_block(plan.handle, G, b, se, fl)
    torch.cuda.synchronize()


@pytest.mark.skip(reason="graph capture of the pipeline ended in a host segmentation fault in two independent "
                         "implementations (inside clak_pipeline_create, then inside the first capturing "
                         "clak_pipeline_launch); the cause was not found, the capture path was removed and the "
                         "pipeline enqueues eagerly on three streams (see test_two_stream_pipeline_matches_eager)")
@pytest.mark.parametrize("prec,t", [(1, 1), (1, 7), (0, 1), (0, 7)])
def test_pipeline_matches_eager_over_replays(prec, t):
    import torch

    from paper_1207_2169_amd import clak
    w = make_workload(2, n=300, m=900, t=t, kin_cols=600)
    block = 256  # 4 blocks, the last ragged
    print(f"pipeline prec={prec} t={t}", flush=True)
    with _setup(w, prec, block) as plan:
        G, b, se, fl, blocks = _blocks(w, block, torch.float64)
        _eager(plan, blocks)
        ref = (b.clone(), se.clone(), fl.clone())
        assert torch.isfinite(ref[0]).all() and (ref[2] == 0).all()
        pipe = clak.clak_pipeline_create(plan.handle, blocks)
        try:
            for rep in range(3):
                b.fill_(float("nan"))
                se.fill_(float("nan"))
                fl.fill_(255)
                torch.cuda.synchronize()
                clak.clak_pipeline_launch(pipe)
                torch.cuda.synchronize()
                assert torch.equal(b, ref[0]) and torch.equal(se, ref[1]) and torch.equal(fl, ref[2]), rep
                # eager work between replays
                _eager(plan, blocks[:1])
        finally:
            clak.clak_pipeline_destroy(pipe)


def test_block_split_and_run_to_run_bitwise():
    import torch
    w = make_workload(2, n=300, m=700, t=5, kin_cols=600)
    outs = []
    for block in (700, 256, 100):
        with _setup(w, 1, block) as plan:
            G, b, se, fl, blocks = _blocks(w, block, torch.float64)
            _eager(plan, blocks)
            outs.append((b.cpu(), se.cpu()))
            if block == 256:
                b.fill_(0)
                _eager(plan, blocks)
                assert torch.equal(b.cpu(), outs[-1][0])
    for o in outs[1:]:
        assert torch.equal(o[0], outs[0][0]) and torch.equal(o[1], outs[0][1])


def test_batch_of_uneven_cohorts_matches_per_plan():
    import torch

    from paper_1207_2169_amd import clak
    sizes = [(300, 3, 512), (200, 20, 256), (450, 1, 300)]
    plans, data, refs = [], [], []
    try:
        for k, (n, t, m) in enumerate(sizes):
            w = make_workload(2, n=n, m=m, t=t, kin_cols=2 * n, seed=777 + k)
            plan = _setup(w, 1, 256)
            G, b, se, fl, blocks = _blocks(w, 256, torch.float32)
            _eager(plan, blocks)
            refs.append((b.clone(), se.clone()))
            b.fill_(float("nan"))
            se.fill_(float("nan"))
            plans.append(plan)
            data.append((b, se, blocks))
        torch.cuda.synchronize()
        batch = clak.clak_batch_create([p.handle for p in plans], [d[2] for d in data])
        try:
            for rep in range(2):
                for b, se, _ in data:
                    b.fill_(float("nan"))
                    se.fill_(float("nan"))
                torch.cuda.synchronize()
                clak.clak_batch_launch(batch)
                torch.cuda.synchronize()
                for (b, se, _), (rb, rse) in zip(data, refs):
                    assert torch.equal(b, rb) and torch.equal(se, rse)
        finally:
            clak.clak_batch_destroy(batch)
    finally:
        for p in plans:
            p.close()


@pytest.mark.parametrize("prec", [1, 0])
def test_batched_rounds_match_per_plan(prec):
    """Cohorts whose kernels agree (mixed, several traits, p_L = 3) run as one
    launch per kernel and round on three streams; the outputs are bitwise
    those of each plan's own eager blocks.  Uneven block counts (3, 2, 4
    blocks of 256) leave plans out of later rounds.  FP64 plans run their
    per-block launches in the same rounds (not batched), equally bitwise."""
    import torch

    from paper_1207_2169_amd import clak
    sizes = [(300, 7, 700), (200, 40, 300), (450, 33, 1000)]
    plans, data, refs = [], [], []
    try:
        for k, (n, t, m) in enumerate(sizes):
            w = make_workload(2, n=n, m=m, t=t, kin_cols=2 * n, seed=991 + k)
            plan = _setup(w, prec, 256)
            G, b, se, fl, blocks = _blocks(w, 256, torch.float32)
            _eager(plan, blocks)
            refs.append((b.clone(), se.clone(), fl.clone()))
            plans.append(plan)
            data.append((b, se, fl, blocks))
        batch = clak.clak_batch_create([p.handle for p in plans], [d[3] for d in data])
        try:
            batched, rounds, streams = clak.clak_batch_get_info(batch)
            print(f"batch prec={prec}: batched={batched} rounds={rounds} streams={streams}", flush=True)
            assert batched == (prec == 1) and rounds == 4 and streams == 3
            for rep in range(3):
                for b, se, fl, _ in data:
                    b.fill_(float("nan"))
                    se.fill_(float("nan"))
                    fl.fill_(255)
                torch.cuda.synchronize()
                clak.clak_batch_launch(batch)
                torch.cuda.synchronize()
                for (b, se, fl, _), (rb, rse, rfl) in zip(data, refs):
                    assert torch.equal(b, rb) and torch.equal(se, rse) and torch.equal(fl, rfl), rep
        finally:
            clak.clak_batch_destroy(batch)
    finally:
        for p in plans:
            p.close()


@pytest.mark.parametrize("prec,t,m", [(1, 1, 900), (1, 7, 900), (0, 1, 900), (0, 7, 900), (1, 1, 3000),
                                      (1, 7, 3000), (0, 1, 3000)])
def test_two_stream_pipeline_matches_eager(prec, t, m):
    """The pipeline (blocks round the workspace slots, alternating between two
    compute streams, ingest overlapped) gives bitwise the outputs of eager
    clak_run_block calls, over repeated launches with eager work in between.
    m = 3000 makes 12 blocks of 256 (the last ragged): every slot is reused
    several times, by either compute stream."""
    import torch

    from paper_1207_2169_amd import clak
    w = make_workload(2, n=300, m=m, t=t, kin_cols=600)
    block = 256
    print(f"two-stream pipeline prec={prec} t={t} m={m}", flush=True)
    with _setup(w, prec, block) as plan:
        G, b, se, fl, blocks = _blocks(w, block, torch.float64)
        _eager(plan, blocks)
        ref = (b.clone(), se.clone(), fl.clone())
        assert torch.isfinite(ref[0]).all() and (ref[2] == 0).all()
        pipe = clak.clak_pipeline_create(plan.handle, blocks)
        try:
            for rep in range(3):
                b.fill_(float("nan"))
                se.fill_(float("nan"))
                fl.fill_(255)
                torch.cuda.synchronize()
                clak.clak_pipeline_launch(pipe)
                torch.cuda.synchronize()
                assert torch.equal(b, ref[0]) and torch.equal(se, ref[1]) and torch.equal(fl, ref[2]), rep
                _eager(plan, blocks[:1])
        finally:
            clak.clak_pipeline_destroy(pipe)
