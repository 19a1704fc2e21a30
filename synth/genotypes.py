"""Counter-based SNP genotype generator.

Every genotype is a pure function of (seed, SNP index, individual index), so a
block of SNPs can be regenerated anywhere (a streamed block, a sampled column
for the oracle) without storing the full n x m matrix, and the result does not
depend on how the SNP axis is split into blocks.

Definition (all arithmetic modulo 2**64):
    mix(x)      = SplitMix64 finaliser: x ^= x>>30; x *= 0xBF58476D1CE4E5B9;
                  x ^= x>>27; x *= 0x94D049BB133111EB; x ^= x>>31
    c           = mix(seed + 0x9E3779B97F4A7C15 * (snp + 1))
    F(snp)      = 838861 + (c >> 40) mod 7549747          (= f * 2**24, f in [0.05, 0.5))
    h           = mix(c ^ (0xD1B54A32D192ED03 * (ind + 1)))
    u1, u2      = h & 0xFFFFFF, (h >> 24) & 0xFFFFFF      (two 24-bit uniforms)
    g(snp, ind) = [u1 < F] + [u2 < F]                      (Binomial(2, f) in {0, 1, 2})
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_GOLD = np.uint64(0x9E3779B97F4A7C15)
_GOLD2 = np.uint64(0xD1B54A32D192ED03)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_F_LO = 838861          # 0.05 * 2**24
_F_SPAN = 7549747       # (0.5 - 0.05) * 2**24


def _mix(x: np.ndarray) -> np.ndarray:
    x = x ^ (x >> np.uint64(30))
    x = x * _M1
    x = x ^ (x >> np.uint64(27))
    x = x * _M2
    return x ^ (x >> np.uint64(31))


def _col_keys(seed: int, snps: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        return _mix(np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + _GOLD * (snps.astype(np.uint64) + np.uint64(1)))


def allele_thresholds(seed: int, start: int, count: int) -> np.ndarray:
    """Per-SNP threshold F = f * 2**24 (int64) for SNPs [start, start+count)."""
    c = _col_keys(seed, np.arange(start, start + count, dtype=np.uint64))
    return (np.int64(_F_LO) + ((c >> np.uint64(40)) % np.uint64(_F_SPAN)).astype(np.int64))


def _block(seed: int, n: int, start: int, count: int) -> np.ndarray:
    snps = np.arange(start, start + count, dtype=np.uint64)
    c = _col_keys(seed, snps)
    F = (np.uint64(_F_LO) + (c >> np.uint64(40)) % np.uint64(_F_SPAN))[:, None]
    with np.errstate(over="ignore"):
        rowk = _GOLD2 * (np.arange(n, dtype=np.uint64) + np.uint64(1))
        h = _mix(c[:, None] ^ rowk[None, :])
    u1 = h & np.uint64(0xFFFFFF)
    u2 = (h >> np.uint64(24)) & np.uint64(0xFFFFFF)
    return ((u1 < F).astype(np.uint8) + (u2 < F).astype(np.uint8))


def snp_genotypes(seed: int, n: int, start: int, count: int, out: np.ndarray | None = None,
                  ld: int | None = None, threads: int | None = None) -> np.ndarray:
    """Genotypes of SNPs [start, start+count) for n individuals.

    Returns a uint8 array of shape (count, ld) whose row s is SNP start+s over
    the n individuals (SNP-major: one SNP column is contiguous), entries beyond
    n in a row are zero.  ``ld`` defaults to n.
    """
    ld = n if ld is None else ld
    if ld < n:
        raise ValueError("ld < n")
    if out is None:
        out = np.zeros((count, ld), dtype=np.uint8)
    chunk = max(1, (1 << 22) // max(n, 1))
    spans = [(s, min(count, s + chunk)) for s in range(0, count, chunk)]

    def work(span):
        s0, s1 = span
        out[s0:s1, :n] = _block(seed, n, start + s0, s1 - s0)

    nthr = threads or min(16, os.cpu_count() or 1)
    if len(spans) == 1 or nthr == 1:
        for sp in spans:
            work(sp)
    else:
        with ThreadPoolExecutor(nthr) as ex:
            list(ex.map(work, spans))
    return out
