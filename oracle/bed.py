"""CPU oracle of the 2-bit genotype decoding (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this module.  It reads the SNP-major PLINK 1 binary genotype format as
published with PLINK 1.07/1.9: three magic bytes 0x6c 0x1b 0x01; then, for
each SNP, ceil(n / 4) bytes; the genotype of individual i sits in byte i // 4
at bits 2 (i % 4) (low) and 2 (i % 4) + 1 (high); the code (high, low) = 00
is homozygous for the first allele, 10 heterozygous, 11 homozygous for the
second allele, 01 missing; the unused high bits of a SNP's last byte are
ignored.  A genotype is the count of the first allele (2, 1, 0), missing is 3.
Parity status: pinned by tests/test_oracle_bed.py against a hand-assembled
fixture (tests/golden/bed_tiny.txt) written from that definition."""
from __future__ import annotations

import numpy as np

MAGIC = (0x6C, 0x1B, 0x01)


def decode_rows(rows: np.ndarray, n: int) -> np.ndarray:
    """(count, >= ceil(n/4)) packed bytes -> (count, n) genotypes, one individual at a time."""
    rows = np.asarray(rows, dtype=np.uint8)
    out = np.empty((rows.shape[0], n), dtype=np.uint8)
    value = {0b00: 2, 0b10: 1, 0b11: 0, 0b01: 3}
    for j in range(rows.shape[0]):
        for i in range(n):
            byte = int(rows[j, i // 4])
            code = (byte >> (2 * (i % 4))) & 0b11
            out[j, i] = value[code]
    return out


def read_bed(path, n: int, m: int) -> np.ndarray:
    """(m, n) genotypes of a file; raises ValueError on a wrong magic or size."""
    data = np.fromfile(path, dtype=np.uint8)
    row = (n + 3) // 4
    if data.size < 3 or tuple(int(x) for x in data[:3]) != MAGIC:
        raise ValueError("not a SNP-major PLINK 1 binary genotype file")
    if data.size != 3 + m * row:
        raise ValueError(f"{data.size} bytes, {3 + m * row} expected")
    return decode_rows(data[3:].reshape(m, row), n)
