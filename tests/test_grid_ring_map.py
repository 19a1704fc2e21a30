"""Host-side model of the one-pass grid kernel's work decomposition and
direct loads (k_grid_ring, p_L <= 3), at test and bench shapes and for every
XCD grouping sg:

* the work-group -> (SNP tile, trait group) map covers every (128-SNP tile,
  32-trait group) pair of the block exactly once, and the SNP tiles of one
  XCD are a contiguous range;
* every fragment the ring loads (the trait operand and d planes into LDS,
  the x and x o x digit planes into registers), for every K slice including
  the clamped loads past the last slice, lies inside its buffer, and every LDS
  destination inside its ring slot;
* the per-wave epilogue stages and the SNP tables fit their LDS slots.

The formulas restate the kernel's index arithmetic (launch grid, tile map,
fragment offsets); a change there must be mirrored here."""
import numpy as np
import pytest

KPAD, SNP_PAD, TRAIT_PAD = 128, 256, 128
GR_SLOT, GR_STAGE = 52 * 1024, 32 * 33


def rnd(a, b):
    return (a + b - 1) // b * b


def work_map(m_blk, t, sg):
    """(SNP tile, trait group, XCD) of every live work-group."""
    ns, ng = (m_blk + 127) // 128, (t + 31) // 32
    gs = (ns + 7) // 8
    bid = np.arange(8 * gs * ng)
    xcd, idx = bid % 8, bid // 8
    c = idx // (sg * ng)
    base = c * sg * ng
    cs = np.minimum(sg, gs - c * sg)
    ok = cs > 0
    cs1 = np.where(ok, cs, 1)
    rem = idx - base
    tg, sl = rem // cs1, c * sg + rem % cs1
    st = xcd * gs + sl
    live = ok & (tg < ng) & (sl < gs) & (st < ns)
    return st[live], tg[live], xcd[live], ns, ng


SHAPES = [  # n, p_L, t, m_blk, max_block
    (1000, 3, 1000, 10000, 10000), (1000, 3, 1000, 476, 10000), (300, 3, 37, 200, 333), (300, 3, 37, 133, 333),
    (160, 3, 127, 130, 130), (160, 3, 129, 130, 130), (128, 1, 5, 300, 300), (4000, 3, 16, 10000, 10000),
    (2000, 3, 1754, 10000, 10000), (200, 2, 70, 1, 64), (256, 3, 1000, 2048, 2048), (129, 3, 3, 257, 300)]


@pytest.mark.parametrize("n,pL,t,m_blk,max_block", SHAPES)
@pytest.mark.parametrize("sg", [1, 2, 4, 8])
def test_ring_grid_tiles_and_addresses(n, pL, t, m_blk, max_block, sg):
    np_, mbp, tp = rnd(n, KPAD), rnd(max_block, SNP_PAD), rnd(t, TRAIT_PAD)
    NV, NT = pL + 1, pL + 2
    two = NT * 64 > 256  # p_L = 3: the quadratic sums in a pass of their own
    st, tg, xcd, ns, ng = work_map(m_blk, t, sg)
    key = st * ng + tg
    assert len(key) == ns * ng and len(np.unique(key)) == len(key)
    for x in range(8):  # contiguous SNP range per XCD
        s = np.unique(st[xcd == x])
        if s.size:
            assert s.max() - s.min() + 1 == s.size
    KT = np_ // 32
    slices = np.unique(np.minimum(np.arange(KT + 2), KT - 1))  # clamped ring loads included
    assert slices.min() == 0 and slices.max() == KT - 1
    i0, j0 = st * 128, tg * 32
    xplane, vplane, dplane = mbp * np_, tp * NV * np_, tp * np_
    vgrp = (j0 // 32) * 32 * NV
    s = slices.max()

    def x_end(p, w):  # digit plane p of x (p < 4) or x o x (p >= 4), SNP tile w
        return p * xplane + (s * mbp + i0 + 32 * w) * 32 + 1024

    def t_end(e, w):  # plane w of operand entry e (d for e = p_L + 1)
        if e <= pL:
            return w * vplane + (s * tp * NV + vgrp + 32 * e) * 32 + 1024, 4 * vplane
        return w * dplane + (s * tp + j0) * 32 + 1024, 4 * dplane

    # the passes as the kernel issues them: (LDS loads per wave per slice,
    # register loads per wave per slice, slices per ring step, operand entry
    # of LDS load q, digit plane of register load q, LDS bound); the second
    # pass of the two-pass kernel stays below the sums parked after the first
    ASAVE_OFF = 36 * 1024
    if two:
        passes = [(1, 4, 2, lambda q: pL + 1, lambda q: 4 + q, GR_SLOT),
                  (NV, 4, 1, lambda q: q, lambda q: q, ASAVE_OFF)]
    else:
        passes = [(NT, 8, 1, lambda q: q, lambda q: q, GR_SLOT)]
    for lpw, xpw, sps, ent, plane, bound in passes:
        assert KT % sps == 0
        for w in range(4):
            for h in range(sps):
                for q in range(lpw):
                    end, size = t_end(ent(q), w)
                    assert (end <= size).all(), ("operand", ent(q), w)
                    assert ((h * lpw + q) * 4 + w) * 1024 + 1024 <= bound
                for q in range(xpw):
                    assert (x_end(plane(q), w) <= 8 * xplane).all(), ("x digits", plane(q), w)
    # epilogue LDS: four waves' [32][33] double stages, then the SNP tables
    assert 4 * GR_STAGE * 8 + 128 * (2 + pL) * 8 <= GR_SLOT
    assert 4 * GR_STAGE <= GR_SLOT
    if two:  # parked sums of two waves per slot after the stages, inside the slot
        assert 4 * GR_STAGE * 8 <= ASAVE_OFF and ASAVE_OFF + 2 * 16 * 64 * 8 <= GR_SLOT


def test_trait_operand_rows_of_a_group():
    """The rows vrow(j, q, p_L + 1) of a 32-trait group are entry-major:
    entry q of the group's 32 traits is rows vgrp + 32 q .. + 31."""
    for NV in (2, 3, 4):
        for j in (0, 5, 31, 32, 70, 999):
            for q in range(NV):
                vrow = (j >> 5) * 32 * NV + q * 32 + (j & 31)
                assert vrow == (j // 32) * 32 * NV + 32 * q + j % 32
