"""Host-side model of the mixed rotation's work decomposition (k_rot_i8): for
every tile configuration, XCD grouping (rg), plain and triangular (CLAK-Chol)
operands, and both placements of the single-trait U^T rows (padding rows or
one more row tile), at test and bench shapes:

* the work-group -> (row tile, SNP tile) map covers every tile exactly once;
* every K slice a tile loads (including the clamped prefetches past its last
  slice) lies in [0, KT), KT = n_pad / 64, or the triangular bound;
* every direct-load fragment address (Z^T digit planes, genotype panel) lies
  inside its buffer.

The formulas restate the kernel's index arithmetic (its launch grid, tile map
and fragment offsets); a change there must be mirrored here."""
import numpy as np
import pytest

ROT_BM, BK, SNP_PAD, KPAD, ZEXT = 64, 64, 256, 128, 64
# (CT, WR, WC) of the ten configurations; all have 64-row tiles
CONFIGS = [(2, 2, 2), (4, 2, 1), (2, 2, 4), (4, 2, 2), (1, 2, 2), (2, 2, 2), (2, 2, 4), (1, 2, 2), (2, 2, 4),
           (2, 2, 2)]


def rnd(a, b):
    return (a + b - 1) // b * b


def rows_of(n, pL, single_trait_mixed):
    """(n_pad, zrows, zlin) as the plan sets them."""
    np_ = rnd(n, KPAD)
    if not single_trait_mixed:
        return np_, np_, np_
    zlin = n if n + pL + 1 <= np_ else np_
    return np_, np_ + (ZEXT if zlin == np_ else 0), zlin


def decompose(n, pL, m_blk, max_block, cfg, rg, tri, single):
    CT, WR, WC = CONFIGS[cfg]
    BM, BN = 32 * WR, 32 * CT * WC
    np_, nz, _ = rows_of(n, pL, single)
    mbp = rnd(max_block, SNP_PAD)
    ntn, ntm = rnd(m_blk, SNP_PAD) // BN, nz // ROT_BM
    sg = 8 // rg
    gm, gn = (ntm + rg - 1) // rg, (ntn + sg - 1) // sg
    bid = np.arange(8 * gm * gn)
    xcd, idx = bid % 8, bid // 8
    tm = ntm - 1 - ((idx % gm) * rg + xcd % rg) if tri else (xcd % rg) * gm + idx % gm
    tn = (xcd // rg) * gn + idx // gm
    live = (tm >= 0) & (tm < ntm) & (tn < ntn) & (idx < gm * gn)
    return dict(CT=CT, WR=WR, WC=WC, BM=BM, BN=BN, np=np_, nz=nz, mbp=mbp, ntm=ntm, ntn=ntn,
                tm=tm[live], tn=tn[live])


SHAPES = [  # n, pL, m_blk, max_block
    (300, 3, 700, 700), (200, 3, 700, 700), (450, 3, 700, 700), (124, 3, 300, 300), (125, 3, 300, 300),
    (128, 3, 300, 300), (119, 8, 300, 300), (100, 3, 1, 64), (129, 3, 257, 300), (1000, 3, 10000, 10000),
    (1000, 3, 476, 1024), (333, 3, 128, 128), (600, 3, 44, 256)]


@pytest.mark.parametrize("n,pL,m_blk,max_block", SHAPES)
def test_rotation_tiles_and_addresses(n, pL, m_blk, max_block):
    for single in (False, True):
        for tri in (0, 1):
            for cfg in range(len(CONFIGS)):
                for rg in (1, 2, 4, 8):
                    d = decompose(n, pL, m_blk, max_block, cfg, rg, tri, single)
                    tm, tn = d["tm"], d["tn"]
                    # every tile exactly once
                    key = tm * d["ntn"] + tn
                    assert len(key) == d["ntm"] * d["ntn"], (cfg, rg, tri, single)
                    assert len(np.unique(key)) == len(key)
                    # K slices: the loop runs KT slices and its prefetches are clamped to KT - 1
                    m0, n0 = tm * d["BM"], tn * d["BN"]
                    kt = (np.minimum(d["np"], m0 + d["BM"]) if tri else np.full_like(m0, d["np"])) // BK
                    assert (kt >= 1).all() and (kt <= d["np"] // BK).all()
                    last = 2 * (kt - 1) + 1  # last 32-byte K slice touched
                    # Z^T digit planes: 4 x nz rows x n_pad bytes, kt32 layout over nz rows
                    WR, CT, WC = d["WR"], d["CT"], d["WC"]
                    a_end = 3 * d["nz"] * d["np"] + (last * d["nz"] + m0 + 32 * (WR - 1) + 32) * 32
                    assert (a_end <= 4 * d["nz"] * d["np"]).all()
                    assert (m0 + d["BM"] <= d["nz"]).all()
                    # genotype panel: mb_pad rows x n_pad bytes, kt32 layout over mb_pad rows
                    b_end = (last * d["mbp"] + n0 + 32 * (CT * WC - 1) + 32) * 32
                    assert (b_end <= d["mbp"] * d["np"]).all()
                    assert (n0 + d["BN"] <= d["mbp"]).all()


@pytest.mark.parametrize("n,pL", [(124, 3), (125, 3), (128, 3), (1000, 3), (119, 8), (120, 8), (256, 3)])
def test_single_trait_rows_placement(n, pL):
    np_, nz, zlin = rows_of(n, pL, True)
    # the p_L + 1 rows of U^T lie past the n eigen rows and inside the operand
    assert zlin >= n and zlin + pL + 1 <= nz and nz % ROT_BM == 0
    # padding rows are used exactly when they can hold them
    assert (nz == np_) == (n + pL + 1 <= np_)


# Z-resident rotation (configuration 10, k_rotz.hip): n_pad <= 1024, plain operand
ZR_KS, ZR_D, ZR_WAVES = 32, 4, 8


def zs_decompose(n, pL, m_blk, max_block, single):
    """Per (work-group, wave, item, tile): the slice, the tile (clamped as the
    kernel clamps it), and whether its results are kept; the kernel's launch
    grid and index arithmetic restated."""
    np_, nz, zlin = rows_of(n, pL, single)
    mbp = rnd(max_block, SNP_PAD)
    S = nz // 32
    q = 1 if S >= 32 else (32 + S // 2) // S
    ntl = rnd(m_blk, SNP_PAD) // 32
    out = []
    for bid in range(8 * S * q):
        xcd, idx = bid % 8, bid // 8
        s, j = idx % S, idx // S
        T8 = (ntl + 7) // 8
        xb = xcd * T8
        xe = min(ntl, xb + T8)
        Tq = (T8 + q - 1) // q
        tb = xb + j * Tq
        te = min(xe, tb + Tq)
        if j >= q or tb >= te:
            continue
        P = (te - tb + 1) // 2
        for w in range(ZR_WAVES):
            NI = (P - w + ZR_WAVES - 1) // ZR_WAVES if P > w else 0
            for i in range(NI):
                for ct in range(2):
                    t = tb + 2 * (w + ZR_WAVES * i) + ct
                    out.append((s, min(t, te - 1), t < te, i, NI, w))
    return dict(np=np_, nz=nz, mbp=mbp, S=S, ntl=ntl, items=out)


@pytest.mark.parametrize("n,pL,m_blk,max_block", [s for s in SHAPES if rnd(s[0], KPAD) <= 32 * ZR_KS])
def test_z_resident_rotation_map_and_addresses(n, pL, m_blk, max_block):
    for single in (False, True):
        d = zs_decompose(n, pL, m_blk, max_block, single)
        np_, nz, mbp = d["np"], d["nz"], d["mbp"]
        KS = np_ // 32
        assert KS % ZR_D == 0 and KS >= ZR_D and KS <= ZR_KS
        items = d["items"]
        kept = [(s, t) for s, t, k, *_ in items if k]
        # every (slice, 32-SNP tile) of the block exactly once
        assert len(kept) == d["S"] * d["ntl"] and len(set(kept)) == len(kept)
        # fragment sources: every K step of every item, the prefetch clamped
        # to the wave's last item and step
        loff_max = 32 * 31 + 16
        zplane = nz * np_
        for s, t, _, i, NI, w in items:
            assert 0 <= t < mbp // 32
            b_last = ((KS - 1) * mbp + 32 * t) * 32 + loff_max + 16
            assert b_last <= mbp * np_
            a_last = 3 * zplane + (KS - 1) * nz * 32 + 32 * s * 32 + loff_max + 16
            assert a_last <= 4 * zplane
            # outputs: x~ rows (EPI 0), the slice partial (EPI 1), the SNP's statistics
            col = 32 * t + 31
            assert col * np_ + 32 * s + 28 + 4 <= mbp * np_ or single
            assert s * mbp + col < (np_ // 64) * mbp * (pL + 2)
            assert col < mbp
        # the prefetch pointer starts D steps in and never passes the wave's last (item, step)
        assert (ZR_D // KS, ZR_D % KS) in ((0, ZR_D), (1, 0))
