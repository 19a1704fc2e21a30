"""CPU FP64 oracle for the GWAS grid of GLS problems (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It wraps ``liboracle.so`` (plain C, see ``oracle.h``), which
evaluates every (SNP, trait) cell directly from the problem statement of the
supplementary notes (section 1, equations GLS and probDef) through a Cholesky
factorisation of M_j, without the eigendecomposition used by the GPU path.
Parity status: pinned by ``tests/test_oracle_pins.py`` (closed forms, brute
force, exact rational arithmetic and invariants).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

OK, SNP_DEGENERATE, M_NOT_SPD, COV_SINGULAR = 0, 1, 2, 3


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from .build import build
            build()
        lib = ctypes.CDLL(path)
        P, I64 = ctypes.c_void_p, ctypes.c_int64
        lib.oracle_gls.argtypes = [I64, I64, P, I64, P, I64, P, I64, P, I64, P, P, I64, P, P,
                                   ctypes.c_int, P, P, P, ctypes.c_int]
        lib.oracle_gls.restype = ctypes.c_int
        lib.oracle_threads.argtypes = [ctypes.c_int]
        lib.oracle_threads.restype = ctypes.c_int
        _LIB = lib
    return _LIB


def threads(request: int = 0) -> int:
    return _lib().oracle_threads(int(request))


def _f64(a, ndim):
    a = np.asfortranarray(np.asarray(a, dtype=np.float64))
    if a.ndim == 1 and ndim == 2:
        a = a.reshape(-1, 1, order="F")
    return a


def gls_cells(Phi, XL, G, Y, h2, s2, snp_idx, trait_idx, var_paper: bool = False,
              threads: int = 0):
    """Oracle values for the cells (G[:, snp_idx[c]], Y[:, trait_idx[c]]).

    Phi (n, n); XL (n, pL); G (n, ng) SNP columns; Y (n, nt); h2, s2 (nt,).
    Returns b (ncells, p), var (ncells, p, p) and flag (ncells,) int32, with
    p = pL + 1 and the SNP effect last.
    """
    Phi = _f64(Phi, 2)
    n = Phi.shape[0]
    XL = _f64(XL, 2) if XL is not None and np.size(XL) else np.zeros((n, 0), order="F")
    G = _f64(G, 2)
    Y = _f64(Y, 2)
    h2 = np.ascontiguousarray(h2, dtype=np.float64).ravel()
    s2 = np.ascontiguousarray(s2, dtype=np.float64).ravel()
    snp = np.ascontiguousarray(snp_idx, dtype=np.int64).ravel()
    tr = np.ascontiguousarray(trait_idx, dtype=np.int64).ravel()
    pL = XL.shape[1]
    p = pL + 1
    if snp.size != tr.size:
        raise ValueError("snp_idx and trait_idx differ in length")
    if snp.size and (snp.max() >= G.shape[1] or tr.max() >= Y.shape[1] or tr.max() >= h2.size
                     or tr.max() >= s2.size):
        raise ValueError("cell index out of range")
    if Phi.shape != (n, n) or XL.shape[0] != n or G.shape[0] != n or Y.shape[0] != n:
        raise ValueError("shape mismatch")
    nc = snp.size
    b = np.empty((nc, p))
    var = np.empty((nc, p, p))
    flag = np.empty(nc, dtype=np.int32)
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    rc = _lib().oracle_gls(n, pL, ptr(Phi), n, ptr(XL) if pL else None, n, ptr(G), n, ptr(Y), n,
                           ptr(h2), ptr(s2), nc, ptr(snp), ptr(tr), 1 if var_paper else 0,
                           ptr(b), ptr(var), ptr(flag), int(threads))
    if rc != 0:
        raise ValueError("oracle_gls rejected its arguments")
    # var was written column-major per cell; transpose to [cell, row, col]
    var = np.ascontiguousarray(var.transpose(0, 2, 1))
    return b, var, flag


def gls_grid(Phi, XL, G, Y, h2, s2, var_paper: bool = False, threads: int = 0):
    """All cells of the m x t grid: b (m, t, p), var (m, t, p, p), flag (m, t)."""
    G = np.asarray(G)
    Y = np.asarray(Y)
    m = G.shape[1]
    t = 1 if Y.ndim == 1 else Y.shape[1]
    ii, jj = np.meshgrid(np.arange(m), np.arange(t), indexing="ij")
    b, var, flag = gls_cells(Phi, XL, G, Y, h2, s2, ii.ravel(), jj.ravel(), var_paper, threads)
    p = b.shape[1]
    return b.reshape(m, t, p), var.reshape(m, t, p, p), flag.reshape(m, t)


def snp_columns(geno_rows) -> np.ndarray:
    """uint8 SNP-major rows (count, >=n) -> float64 (n, count) columns."""
    g = np.asarray(geno_rows)
    return np.asfortranarray(g.T.astype(np.float64))
