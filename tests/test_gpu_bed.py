"""2-bit genotype input (CLAK_G_P2) and the out-of-core file scan: the ingest
decodes the PLINK 1 binary codes exactly (results bitwise equal to the u8
path on the same genotypes, missing codes flagged, parity with the oracle's
decoding of the file), from device memory, pinned host memory and through the
copy-engine staging; clak_bed_scan over a file equals per-block runs bitwise."""
import numpy as np
import pytest

import oracle
from oracle import bed as obed
from synth import make_workload, pack_rows, write_bed

from _helpers import errors

pytestmark = pytest.mark.gpu


def _plan(w, prec, block, flags=0):
    import torch

    from paper_1207_2169_amd import clak
    plan = clak.Plan(w.n, w.pL, w.t, block, prec, flags)
    clak.clak_set_kinship(plan.handle, torch.from_numpy(np.ascontiguousarray(w.Phi)).cuda())
    clak.clak_set_covariates(plan.handle, torch.from_numpy(np.ascontiguousarray(w.XL.T)).cuda().t())
    clak.clak_set_traits(plan.handle, torch.from_numpy(np.ascontiguousarray(w.Y.T)).cuda().t(),
                         torch.from_numpy(w.h2).cuda(), torch.from_numpy(w.s2).cuda())
    return plan


def _outs(w, m, dtype, full=False):
    import torch
    p = w.pL + 1
    b = torch.full((w.t, m, p) if full else (w.t, m), float("inf"), dtype=dtype, device="cuda")
    se = torch.full((w.t, m), float("inf"), dtype=dtype, device="cuda")
    fl = torch.full((w.t, m), 255, dtype=torch.uint8, device="cuda")
    pv = torch.full((w.t, m), float("inf"), dtype=dtype, device="cuda")
    return b, se, fl, pv


def _same(x, y):
    return np.array_equal(x.cpu().numpy(), y.cpu().numpy(), equal_nan=True)


@pytest.mark.parametrize("prec,n,pad", [(1, 300, 0), (1, 301, 1), (0, 257, 3), (1, 1000, 2)])
def test_packed_rows_equal_u8_rows(prec, n, pad):
    """Row pitches with and without 4-byte words, device and pinned host rows, staging."""
    import torch

    from paper_1207_2169_amd import clak
    w = make_workload(2, n=n, m=200, t=5, kin_cols=2 * n)
    g = w.genotypes(0, w.m)
    g[17, 5] = 7  # out of range in u8 ...
    packed = pack_rows(np.minimum(g, 3))  # ... missing in 2-bit
    row = packed.shape[1]
    P = np.zeros((w.m, row + pad), np.uint8)
    P[:, :row] = packed
    print(f"packed rows prec={prec} n={n} row={row} ldg={row + pad}", flush=True)
    for flags in (0, clak.CLAK_STAGE_GENOTYPES):
        with _plan(w, prec, w.m, flags) as plan:
            ref = _outs(w, w.m, torch.float64)
            clak.clak_run_block(plan.handle, torch.from_numpy(g).cuda(), *ref)
            torch.cuda.synchronize()
            assert int(ref[2][:, 17].min()) == 2 and int((ref[2] == 0).sum()) == w.t * (w.m - 1)
            for G in (torch.from_numpy(P).cuda(), torch.from_numpy(P).pin_memory()):
                out = _outs(w, w.m, torch.float64)
                clak.clak_run_block(plan.handle, G, *out, g_dtype=clak.CLAK_G_P2)
                torch.cuda.synchronize()
                for a, r in zip(out, ref):
                    assert _same(a, r)


@pytest.mark.parametrize("prec,full,depth", [(1, False, 2), (1, True, 3), (0, False, 4)])
def test_bed_scan_matches_blocks_and_oracle(tmp_path, prec, full, depth):
    import torch

    from paper_1207_2169_amd import clak
    w = make_workload(2, n=300, m=1100, t=7, kin_cols=600)
    block = 256  # 5 blocks, the last ragged
    path = tmp_path / "w.bed"
    write_bed(path, w)
    print(f"bed scan prec={prec} full={full} depth={depth}", flush=True)
    flags = clak.CLAK_OUT_FULL if full else 0
    with _plan(w, prec, block, flags) as plan:
        ref = _outs(w, w.m, torch.float32, full)
        G = torch.from_numpy(w.genotypes(0, w.m)).cuda()
        for s in range(0, w.m, block):
            clak.clak_run_block(plan.handle, G[s:s + block], *(x[:, s:s + block] for x in ref))
        torch.cuda.synchronize()
        out = _outs(w, w.m, torch.float32, full)
        h = clak.clak_bed_open(str(path), w.n, w.m, block, depth)
        try:
            clak.clak_bed_scan(h, plan.handle, *out)
            again = _outs(w, w.m, torch.float32, full)  # a finished scan rewinds the reader
            clak.clak_bed_scan(h, plan.handle, *again)
        finally:
            clak.clak_bed_close(h)
        for a, a2, r in zip(out, again, ref):
            assert _same(a, r) and _same(a2, r)
    # parity of the scanned genotypes with the oracle's own reading of the file, on sampled cells
    gf = obed.read_bed(path, w.n, w.m)
    rng = np.random.default_rng(3)
    snp, tr = rng.integers(0, w.m, 300), rng.integers(0, w.t, 300)
    uniq, inv = np.unique(snp, return_inverse=True)
    rb, rv, _ = oracle.gls_cells(w.Phi, w.XL, gf[uniq].T.astype(float), w.Y, w.h2, w.s2, inv, tr)
    b = out[0].cpu().numpy().astype(np.float64)
    bs = b[tr, snp, -1] if full else b[tr, snp]
    eb, es = errors(bs, out[1].cpu().numpy()[tr, snp], rb[:, -1], np.sqrt(rv[:, -1, -1]))
    print(f"eps_b={eb:.3e} eps_se={es:.3e}")
    assert eb < 1e-6 and es < 1e-6


def test_bed_scan_argument_errors(tmp_path):
    import torch

    from paper_1207_2169_amd import clak
    w = make_workload(2, n=200, m=300, t=2, kin_cols=400)
    path = tmp_path / "w.bed"
    write_bed(path, w)
    with _plan(w, 1, 128) as plan:
        b, se, fl, pv = _outs(w, w.m, torch.float32)
        h = clak.clak_bed_open(str(path), w.n, w.m, 256, 2)
        try:
            with pytest.raises(clak.ClakError) as e:  # block larger than the plan's max_block
                clak.clak_bed_scan(h, plan.handle, b, se)
            assert e.value.status == clak.CLAK_E_ARG
        finally:
            clak.clak_bed_close(h)
        h = clak.clak_bed_open(str(path), w.n, w.m, 128, 2)
        try:
            small = torch.empty((w.t, 100), dtype=torch.float32, device="cuda")
            with pytest.raises(ValueError):  # fewer output columns than SNPs: the binding refuses
                clak.clak_bed_scan(h, plan.handle, small, small.clone())
            small2 = small.clone()
            assert clak.lib().clak_bed_scan(h, plan.handle, small.data_ptr(), small2.data_ptr(), clak.CLAK_OUT_F32,
                                            100, None, None) == clak.CLAK_E_ARG  # ldo < m: so does the library
            clak.clak_bed_scan(h, plan.handle, b, se, fl, pv)
            torch.cuda.synchronize()
            assert bool(torch.isfinite(pv).all()) and int(fl.max()) == 0
        finally:
            clak.clak_bed_close(h)


def test_staging_contiguous_and_wide_rows():
    """CLAK_STAGE_GENOTYPES moves rows that fit the staging pitch as one contiguous copy and re-pitches
    wider ones; both give the unstaged results bitwise (u8 rows 3n + 5 wide, f16 rows, 2-bit rows)."""
    import torch

    from paper_1207_2169_amd import clak
    w = make_workload(2, n=250, m=300, t=3, kin_cols=500)
    g = w.genotypes(0, w.m)
    wide = np.zeros((w.m, 3 * w.n + 5), np.uint8)
    wide[:, :w.n] = g
    print("staging wide rows", flush=True)
    with _plan(w, 1, w.m) as plan:
        ref = _outs(w, w.m, torch.float64)
        clak.clak_run_block(plan.handle, torch.from_numpy(g).cuda(), *ref)
        torch.cuda.synchronize()
    cases = [(torch.from_numpy(wide).cuda(), None), (torch.from_numpy(wide).pin_memory(), None),
             (torch.from_numpy(g).half().cuda(), None), (torch.from_numpy(pack_rows(g)).pin_memory(), clak.CLAK_G_P2)]
    with _plan(w, 1, w.m, clak.CLAK_STAGE_GENOTYPES) as plan:
        for G, gdt in cases:
            out = _outs(w, w.m, torch.float64)
            clak.clak_run_block(plan.handle, G, *out, g_dtype=gdt)
            torch.cuda.synchronize()
            for a, r in zip(out, ref):
                assert _same(a, r)
