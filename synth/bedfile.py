"""The synthetic genotypes as a SNP-major PLINK 1 binary genotype file (for
the out-of-core input path): the bytes 0x6c 0x1b 0x01, then one row of
(n + 3) // 4 bytes per SNP, four individuals per byte (individual i in bits
2 (i % 4), 2 (i % 4) + 1), codes 00 / 10 / 11 for 2 / 1 / 0 copies of the
first allele and 01 for a missing genotype (3 here).  File I/O only."""
from __future__ import annotations

import numpy as np

MAGIC = bytes([0x6C, 0x1B, 0x01])
_CODE = np.array([0b11, 0b10, 0b00, 0b01], dtype=np.uint8)  # genotype 0, 1, 2, missing -> code


def pack_rows(g: np.ndarray) -> np.ndarray:
    """(count, n) genotypes in {0, 1, 2, 3 = missing} -> (count, (n + 3) // 4) packed rows."""
    g = np.asarray(g, dtype=np.uint8)
    count, n = g.shape
    pad = (-n) % 4
    codes = _CODE[np.minimum(g, 3)]
    if pad:
        codes = np.concatenate([codes, np.zeros((count, pad), np.uint8)], axis=1)
    c = codes.reshape(count, -1, 4)
    return (c[:, :, 0] | (c[:, :, 1] << 2) | (c[:, :, 2] << 4) | (c[:, :, 3] << 6)).astype(np.uint8)


def write_bed(path, workload, m: int | None = None, chunk: int = 100_000) -> int:
    """Writes the first m SNPs of a workload; returns the file size in bytes."""
    m = workload.m if m is None else m
    with open(path, "wb") as f:
        f.write(MAGIC)
        for s0 in range(0, m, chunk):
            f.write(pack_rows(workload.genotypes(s0, min(chunk, m - s0))).tobytes())
    return 3 + m * ((workload.n + 3) // 4)
