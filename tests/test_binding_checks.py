"""The Python binding's argument checks (no GPU needed): column-major views
of strided single columns, and refusal of tensors whose shapes or strides do
not match the plan, before any library call reads or writes them."""
import numpy as np
import pytest
import torch

from paper_1207_2169_amd import clak
from paper_1207_2169_amd.clak import Shape, _block_layout, _colmajor_view, _out_layout


def _read_colmajor(A, ld, rows, cols):
    """What the library reads: element (i, c) at offset i + c * ld of A's storage."""
    flat = torch.as_strided(A, (A.untyped_storage().nbytes() // A.element_size(),), (1,), 0)
    off = A.storage_offset()
    return np.array([[float(flat[off + i + c * ld]) for c in range(cols)] for i in range(rows)])


@pytest.mark.parametrize("j", [0, 2, 4])
def test_single_column_views_of_row_major_matrices(j):
    n, t = 7, 5
    Y = torch.arange(n * t, dtype=torch.float64).reshape(n, t)  # row-major: stride (t, 1)
    for view in (Y[:, j:j + 1], Y[:, j]):
        A, ld = _colmajor_view(view, "Y", (n, 1))
        assert A.stride(0) == 1 and ld >= n
        np.testing.assert_array_equal(_read_colmajor(A, ld, n, 1)[:, 0], Y[:, j].numpy())


def test_single_covariate_column_strided():
    n = 9
    XL = torch.randn(n, 3, dtype=torch.float64)  # row-major
    A, ld = _colmajor_view(XL[:, 1:2], "X_L", (n, 1))
    np.testing.assert_array_equal(_read_colmajor(A, ld, n, 1)[:, 0], XL[:, 1].numpy())


def test_column_major_views_are_passed_without_copy():
    n, t = 6, 4
    base = torch.randn(t, n + 3, dtype=torch.float64)  # columns of length n inside rows of n + 3
    view = base[:, :n].t()
    A, ld = _colmajor_view(view, "Y", (n, t))
    assert A.data_ptr() == view.data_ptr() and ld == n + 3
    np.testing.assert_array_equal(_read_colmajor(A, ld, n, t), view.numpy())
    # overlapping columns are copied
    ov = torch.as_strided(torch.randn(40, dtype=torch.float64), (n, t), (1, 2))
    A, ld = _colmajor_view(ov, "Y", (n, t))
    assert ld >= n
    np.testing.assert_array_equal(_read_colmajor(A, ld, n, t), ov.numpy())


def test_matrix_shapes_against_the_plan():
    with pytest.raises(ValueError, match="shape"):
        _colmajor_view(torch.zeros(5, 5, dtype=torch.float64), "Phi", (6, 6))
    with pytest.raises(ValueError, match="shape"):
        _colmajor_view(torch.zeros(6, 2, dtype=torch.float64), "X_L", (6, 3))
    with pytest.raises(ValueError, match="shape"):
        _colmajor_view(torch.zeros(6, 3, dtype=torch.float64), "Y", (6, 4))
    with pytest.raises(ValueError, match="2-D"):
        _colmajor_view(torch.zeros(2, 3, 4, dtype=torch.float64), "Y", None)


SH = Shape(n=20, p_L=3, t=4, max_block=16)


def _outs(t, m, dt=torch.float32, full=False, p=4):
    b = torch.empty((t, m, p) if full else (t, m), dtype=dt)
    return b, torch.empty((t, m), dtype=dt)


def test_block_layout_accepts_the_plan_shapes():
    G = torch.zeros(16, 20, dtype=torch.uint8)
    b, se = _outs(4, 16)
    assert _block_layout(SH, G, b, se) == (16, 20, clak.CLAK_G_U8, 16, clak.CLAK_OUT_F32)
    # views into wider outputs keep their leading dimension
    B, S = _outs(4, 100, torch.float64)
    fl = torch.zeros(4, 100, dtype=torch.uint8)
    pv = torch.empty(4, 100, dtype=torch.float64)
    r = _block_layout(SH, G[:10], B[:, 30:40], S[:, 30:40], fl[:, 30:40], pv[:, 30:40])
    assert r == (10, 20, clak.CLAK_G_U8, 100, clak.CLAK_OUT_F64)
    # full vector: (t, ldo, p) with a cell's entries contiguous
    full = Shape(20, 3, 4, 16, flags=clak.CLAK_OUT_FULL)
    b, se = _outs(4, 16, full=True)
    assert _block_layout(full, G, b, se)[3] == 16
    # 2-bit rows of (n + 3) / 4 bytes
    assert _block_layout(SH, torch.zeros(3, 5, dtype=torch.uint8), *_outs(4, 3), g_dtype=clak.CLAK_G_P2)[1] == 5


@pytest.mark.parametrize("case", ["too_many_snps", "short_rows", "se_rows", "se_cols", "b_cols", "b_stride",
                                  "b_dtype", "flags_rows", "flags_dtype", "pval_stride", "full_missing_p",
                                  "full_wrong_p", "full_stride", "genotype_dtype", "noncontig_rows",
                                  "overlapping_rows", "p2_short"])
def test_block_layout_refuses(case):
    G = torch.zeros(16, 20, dtype=torch.uint8)
    b, se = _outs(4, 16)
    fl = pv = None
    sh, gdt = SH, None
    if case == "too_many_snps":
        G = torch.zeros(17, 20, dtype=torch.uint8)
        b, se = _outs(4, 17)
    elif case == "short_rows":
        G = torch.zeros(16, 19, dtype=torch.uint8)
    elif case == "se_rows":
        b, se = _outs(3, 16)
    elif case == "se_cols":
        se = torch.empty(4, 15)
    elif case == "b_cols":
        b = torch.empty(4, 15)
    elif case == "b_stride":
        b = torch.empty(4, 32)[:, :16]
    elif case == "b_dtype":
        b = torch.empty(4, 16, dtype=torch.float64)
    elif case == "flags_rows":
        fl = torch.zeros(2, 16, dtype=torch.uint8)
    elif case == "flags_dtype":
        fl = torch.zeros(4, 16, dtype=torch.int32)
    elif case == "pval_stride":
        pv = torch.empty(4, 40)[:, :16]
    elif case == "full_missing_p":
        sh = Shape(20, 3, 4, 16, flags=clak.CLAK_OUT_FULL)
    elif case == "full_wrong_p":
        sh = Shape(20, 3, 4, 16, flags=clak.CLAK_OUT_FULL)
        b = torch.empty(4, 16, 3)
    elif case == "full_stride":
        sh = Shape(20, 3, 4, 16, flags=clak.CLAK_OUT_FULL)
        b = torch.empty(4, 16, 8)[:, :, :4]
    elif case == "genotype_dtype":
        G = torch.zeros(16, 20, dtype=torch.int32)
    elif case == "noncontig_rows":
        G = torch.zeros(20, 16, dtype=torch.uint8).t()
    elif case == "overlapping_rows":
        se = torch.as_strided(torch.empty(100), (4, 16), (8, 1))
    elif case == "p2_short":
        G = torch.zeros(16, 4, dtype=torch.uint8)
        gdt = clak.CLAK_G_P2
    with pytest.raises(ValueError):
        _block_layout(sh, G, b, se, fl, pv, gdt)


def test_single_trait_outputs_take_any_row_stride():
    sh = Shape(20, 3, 1, 16)
    b = torch.empty(3, 16)[1:2]
    se = torch.empty(1, 16)
    assert _out_layout(sh, b, se, None, None, 16) == (16, clak.CLAK_OUT_F32)
