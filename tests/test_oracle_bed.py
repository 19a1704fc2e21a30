"""Pins of the 2-bit genotype decoder (oracle/bed.py) and host-side checks of
the out-of-core reader's file validation (no GPU needed)."""
import ctypes
import os

import numpy as np
import pytest

from oracle import bed
from synth import make_workload, pack_rows, write_bed

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    fields = {}
    rows = []
    for line in open(os.path.join(HERE, "golden", "bed_tiny.txt")):
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        if ":" in line:
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
        else:
            rows.append([int(x) for x in line.split()])
    data = bytes(int(x, 16) for x in fields["bytes"].split())
    return data, int(fields["n"]), int(fields["m"]), np.array(rows, dtype=np.uint8)


def test_hand_assembled_fixture(tmp_path):
    data, n, m, g = _golden()
    path = tmp_path / "tiny.bed"
    path.write_bytes(data)
    assert np.array_equal(bed.read_bed(path, n, m), g)
    assert np.array_equal(bed.decode_rows(np.frombuffer(data[3:], np.uint8).reshape(m, -1), n), g)


def test_bad_magic_and_size(tmp_path):
    data, n, m, _ = _golden()
    p1 = tmp_path / "magic.bed"
    p1.write_bytes(bytes([0x6C, 0x1B, 0x00]) + data[3:])  # individual-major mode is not read
    with pytest.raises(ValueError):
        bed.read_bed(p1, n, m)
    p2 = tmp_path / "size.bed"
    p2.write_bytes(data[:-1])
    with pytest.raises(ValueError):
        bed.read_bed(p2, n, m)


@pytest.mark.parametrize("n", [1, 4, 7, 301])
def test_synthetic_writer_agrees_with_the_decoder(tmp_path, n):
    """Two independent codes (the input writer, the oracle decoder) agree, missing genotypes included."""
    rng = np.random.default_rng(n)
    g = rng.integers(0, 4, size=(13, n)).astype(np.uint8)
    assert np.array_equal(bed.decode_rows(pack_rows(g), n), g)
    w = make_workload(0, m=37)
    path = tmp_path / "w.bed"
    size = write_bed(path, w)
    assert os.path.getsize(path) == size
    assert np.array_equal(bed.read_bed(path, w.n, w.m), w.genotypes(0, w.m))


def test_reader_rejects_bad_files_without_a_gpu(tmp_path):
    from paper_1207_2169_amd import clak
    lib = clak.lib()
    data, n, m, _ = _golden()
    h = ctypes.c_void_p()
    assert lib.clak_bed_open(ctypes.byref(h), str(tmp_path / "absent.bed").encode(), n, m, 2, 2) == clak.CLAK_E_ARG
    p1 = tmp_path / "magic.bed"
    p1.write_bytes(bytes([0x6C, 0x1B, 0x00]) + data[3:])
    assert lib.clak_bed_open(ctypes.byref(h), str(p1).encode(), n, m, 2, 2) == clak.CLAK_E_ARG
    assert b"PLINK" in lib.clak_last_error()
    p2 = tmp_path / "tiny.bed"
    p2.write_bytes(data)
    assert lib.clak_bed_open(ctypes.byref(h), str(p2).encode(), n, m + 1, 2, 2) == clak.CLAK_E_ARG
    assert lib.clak_bed_open(ctypes.byref(h), str(p2).encode(), n, m, 2, 1) == clak.CLAK_E_ARG
    assert lib.clak_bed_scan(None, None, None, None, 0, 1, None, None) == clak.CLAK_E_ARG
    assert lib.clak_bed_close(None) == clak.CLAK_E_ARG
