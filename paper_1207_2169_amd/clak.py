"""ctypes binding of libclak (``include/clak.h``): argument marshalling only.

Every function carries the name of the C entry point it calls.  Matrices are
passed as torch tensors on the GPU; a tensor standing for an n x c
column-major matrix has logical shape (n, c) and unit stride along its first
dimension (the transpose of a contiguous (c, ld) tensor), and its leading
dimension is read from its strides.  Genotype blocks and outputs use the
SNP-major layout of the C ABI directly: G is (m_blk, ldg) with one SNP per row,
b and se are (t, ldo) with SNPs fastest.

There is no fallback: if the library is not built or cannot be loaded, every
call raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import NamedTuple, Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libclak.so")

CLAK_OK, CLAK_E_ARG, CLAK_E_STATE, CLAK_E_NOT_SPD, CLAK_E_COV_SINGULAR, CLAK_E_EIG, CLAK_E_WORKSPACE, \
    CLAK_E_DEVICE, CLAK_E_UNSUPPORTED = range(9)
STATUS_NAMES = {0: "CLAK_OK", 1: "CLAK_E_ARG", 2: "CLAK_E_STATE", 3: "CLAK_E_NOT_SPD",
                4: "CLAK_E_COV_SINGULAR", 5: "CLAK_E_EIG", 6: "CLAK_E_WORKSPACE", 7: "CLAK_E_DEVICE",
                8: "CLAK_E_UNSUPPORTED"}
CLAK_PREC_FP64, CLAK_PREC_MIXED = 0, 1
CLAK_VAR_MODEL, CLAK_VAR_PAPER = 0, 1
CLAK_OUT_SNP, CLAK_OUT_FULL, CLAK_STAGE_GENOTYPES, CLAK_CHOL = 0, 2, 4, 8
CLAK_G_U8, CLAK_G_F16, CLAK_G_P2 = 0, 1, 2
CLAK_OUT_F32, CLAK_OUT_F64 = 0, 1
CLAK_VC_ML, CLAK_VC_REML = 0, 1
CLAK_CELL_OK, CLAK_CELL_DEGENERATE, CLAK_CELL_BAD_GENOTYPE = 0, 1, 2
CLAK_STAGE_INGEST, CLAK_STAGE_ROTATE, CLAK_STAGE_ENCODE, CLAK_STAGE_GRID, CLAK_STAGE_COUNT = 0, 1, 2, 3, 4
STAGE_NAMES = ("ingest", "rotate", "encode", "grid")
CLAK_PROFILE_OFF, CLAK_PROFILE_SERIAL, CLAK_PROFILE_PIPELINED = 0, 1, 2

# exported symbol -> (restype, argtypes)
_P, _I64, _I, _U32, _SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_uint32, ctypes.c_size_t
SIGNATURES = {
    "clak_plan_create": (_I, [ctypes.POINTER(_P), _I64, _I64, _I64, _I64, _I, _U32]),
    "clak_plan_workspace_size": (_I, [_P, ctypes.POINTER(_SZ)]),
    "clak_plan_set_workspace": (_I, [_P, _P, _SZ]),
    "clak_plan_set_stream": (_I, [_P, _P]),
    "clak_set_kinship": (_I, [_P, _P, _I64]),
    "clak_set_eigen": (_I, [_P, _P, _I64, _P]),
    "clak_set_covariates": (_I, [_P, _P, _I64]),
    "clak_set_traits": (_I, [_P, _P, _I64, _P, _P]),
    "clak_estimate_vc": (_I, [_P, _P, _I64, _I, _P, _P, _P]),
    "clak_run_block": (_I, [_P, _I64, _P, _I, _I64, _P, _P, _I, _I64, _P, _P]),
    "clak_run_block_static": (_I, [_P, _I64, _P, _I, _I64, _P, _P, _I, _I64, _P, _P]),
    "clak_plan_block_scratch_size": (_I, [_P, ctypes.POINTER(_SZ)]),
    "clak_plan_destroy": (_I, [_P]),
    "clak_plan_set_profiling": (_I, [_P, _I]),
    "clak_plan_set_tuning": (_I, [_P, _I, _I, _I, _I]),
    "clak_plan_get_tuning": (_I, [_P, _P, _P, _P, _P]),
    "clak_plan_get_shape": (_I, [_P, _P, _P, _P, _P, _P, _P]),
    "clak_autotune": (_I, [_P, _I64, _P, _I, _I64, _P, _P, _I, _I64, _P, ctypes.c_char_p]),
    "clak_plan_get_profile": (_I, [_P, _P, _P]),
    "clak_plan_get_busy": (_I, [_P, _P]),
    "clak_bed_open": (_I, [ctypes.POINTER(_P), ctypes.c_char_p, _I64, _I64, _I64, _I]),
    "clak_bed_scan": (_I, [_P, _P, _P, _P, _I, _I64, _P, _P]),
    "clak_bed_close": (_I, [_P]),
    "clak_last_error": (ctypes.c_char_p, []),
    "clak_version": (ctypes.c_char_p, []),
}

class clak_block(ctypes.Structure):
    _fields_ = [("m_blk", ctypes.c_int64), ("G", ctypes.c_void_p), ("ldg", ctypes.c_int64),
                ("b", ctypes.c_void_p), ("se", ctypes.c_void_p), ("ldo", ctypes.c_int64),
                ("flags", ctypes.c_void_p), ("pval", ctypes.c_void_p)]


SIGNATURES.update({
    "clak_pipeline_create": (_I, [ctypes.POINTER(_P), _P, _I64, ctypes.POINTER(clak_block), _I, _I]),
    "clak_pipeline_launch": (_I, [_P]),
    "clak_pipeline_destroy": (_I, [_P]),
    "clak_batch_create": (_I, [ctypes.POINTER(_P), _I, ctypes.POINTER(_P), ctypes.POINTER(_I64),
                               ctypes.POINTER(clak_block), _I, _I]),
    "clak_batch_launch": (_I, [_P, _P]),
    "clak_batch_get_info": (_I, [_P, _P, _P, _P]),
    "clak_autotune_pipeline": (_I, [_P, _I64, ctypes.POINTER(clak_block), _I, _I, ctypes.c_char_p]),
    "clak_batch_destroy": (_I, [_P]),
})

_lib_handle = None
_BED_SNPS = {}  # SNPs of each open genotype file reader (outputs are checked against it)


class ClakError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def lib():
    """The loaded libclak (raises if it is missing)."""
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libclak.so is not built ({LIB_PATH}); run __graft_entry__.build()")
        h = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        _lib_handle = h
    return _lib_handle


def _check(status: int, where: str):
    if status != CLAK_OK:
        msg = lib().clak_last_error()
        raise ClakError(status, where, msg.decode() if msg else "")


def _dev(x: torch.Tensor, what: str, dtype=None):
    """A GPU tensor, or a pinned host tensor (the library reads it over PCIe; it
    refuses memory the device cannot address)."""
    if not isinstance(x, torch.Tensor) or not (x.is_cuda or x.is_pinned()):
        raise ValueError(f"{what} must be a torch tensor on the GPU or in pinned host memory")
    if dtype is not None and x.dtype != dtype:
        raise ValueError(f"{what} must be {dtype}, got {x.dtype}")
    return x


def _colmajor_view(A: torch.Tensor, what: str, shape=None):
    """(A', ld): A as an n x c column-major matrix the library can read with
    leading dimension ld (a copy when A's rows are not unit-strided, whatever
    its number of columns), after checking its shape against `shape`."""
    if A.dim() == 1:
        A = A.reshape(-1, 1)
    if A.dim() != 2:
        raise ValueError(f"{what} must be 2-D")
    if shape is not None and tuple(A.shape) != tuple(shape):
        raise ValueError(f"{what} must have shape {tuple(shape)}, got {tuple(A.shape)}")
    if (A.shape[0] > 1 and A.stride(0) != 1) or (A.shape[1] > 1 and A.stride(1) < A.shape[0]):
        A = A.t().contiguous().t()
    ld = A.stride(1) if A.shape[1] > 1 else A.shape[0]
    return A, max(ld, A.shape[0])


def _colmajor(A: torch.Tensor, what: str, shape=None):
    """(pointer, leading dimension, keep-alive tensor) of an n x c matrix."""
    _dev(A, what, torch.float64)
    A, ld = _colmajor_view(A, what, shape)
    return A.data_ptr(), ld, A


def _vector(x: torch.Tensor, what: str, count: int):
    """A contiguous float64 device vector of exactly `count` values."""
    x = _dev(x, what, torch.float64)
    if x.dim() != 1 or x.numel() != count:
        raise ValueError(f"{what} must be a 1-D tensor of {count} values, got shape {tuple(x.shape)}")
    return x.contiguous()


class Shape(NamedTuple):
    """The sizes and options of a plan (the arguments of clak_plan_create)."""
    n: int
    p_L: int
    t: int
    max_block: int
    precision: int = CLAK_PREC_FP64
    flags: int = 0


def clak_plan_get_shape(plan: int) -> Shape:
    """The sizes and options the plan was created with."""
    v = [ctypes.c_int64(0) for _ in range(4)] + [ctypes.c_int(0), ctypes.c_uint32(0)]
    _check(lib().clak_plan_get_shape(plan, *[ctypes.cast(ctypes.byref(x), _P) for x in v]), "clak_plan_get_shape")
    return Shape(*(x.value for x in v))


def clak_version() -> str:
    return lib().clak_version().decode()


def clak_plan_create(n: int, p_L: int, t: int, max_block: int, precision: int = CLAK_PREC_FP64,
                     flags: int = 0) -> int:
    h = _P()
    _check(lib().clak_plan_create(ctypes.byref(h), n, p_L, t, max_block, precision, flags), "clak_plan_create")
    return h.value


def clak_plan_workspace_size(plan: int) -> int:
    out = _SZ()
    _check(lib().clak_plan_workspace_size(plan, ctypes.byref(out)), "clak_plan_workspace_size")
    return out.value


def clak_plan_set_workspace(plan: int, ws: torch.Tensor):
    if not ws.is_cuda:
        raise ValueError("the workspace must be a GPU tensor")
    _dev(ws, "workspace", torch.uint8)
    _check(lib().clak_plan_set_workspace(plan, ws.data_ptr(), ws.numel()), "clak_plan_set_workspace")


def clak_plan_set_stream(plan: int, stream: Optional[torch.cuda.Stream] = None):
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(lib().clak_plan_set_stream(plan, s.cuda_stream), "clak_plan_set_stream")


def clak_set_kinship(plan: int, Phi: torch.Tensor):
    n = clak_plan_get_shape(plan).n
    ptr, ld, _keep = _colmajor(Phi, "Phi", (n, n))
    _check(lib().clak_set_kinship(plan, ptr, ld), "clak_set_kinship")


def clak_set_eigen(plan: int, Z: torch.Tensor, w: torch.Tensor):
    n = clak_plan_get_shape(plan).n
    ptr, ld, _keep = _colmajor(Z, "Z", (n, n))
    w = _vector(w, "w", n)
    _check(lib().clak_set_eigen(plan, ptr, ld, w.data_ptr()), "clak_set_eigen")


def clak_set_covariates(plan: int, XL: torch.Tensor):
    sh = clak_plan_get_shape(plan)
    ptr, ld, _keep = _colmajor(XL, "X_L", (sh.n, sh.p_L))
    _check(lib().clak_set_covariates(plan, ptr, ld), "clak_set_covariates")


def clak_set_traits(plan: int, Y: torch.Tensor, h2: torch.Tensor, s2: torch.Tensor):
    sh = clak_plan_get_shape(plan)
    ptr, ld, _keep = _colmajor(Y, "Y", (sh.n, sh.t))
    h2 = _vector(h2, "h2", sh.t)
    s2 = _vector(s2, "s2", sh.t)
    _check(lib().clak_set_traits(plan, ptr, ld, h2.data_ptr(), s2.data_ptr()), "clak_set_traits")


def clak_estimate_vc(plan: int, Y: torch.Tensor, method: int = CLAK_VC_REML, h2: Optional[torch.Tensor] = None,
                     s2: Optional[torch.Tensor] = None, loglik: Optional[torch.Tensor] = None):
    """Per-trait (h2, s2, loglik) of the reduced model; outputs are allocated when not given (float64, t values)."""
    sh = clak_plan_get_shape(plan)
    ptr, ld, _keep = _colmajor(Y, "Y", (sh.n, sh.t))
    t = sh.t
    outs = []
    for name, x in (("h2", h2), ("s2", s2), ("loglik", loglik)):
        if x is None:
            x = torch.empty(t, dtype=torch.float64, device=Y.device)
        x = _dev(x, name, torch.float64)
        if x.dim() != 1 or not x.is_contiguous() or x.numel() != t:
            raise ValueError(f"{name}: need a contiguous 1-D float64 tensor of t={t} values")
        outs.append(x)
    _check(lib().clak_estimate_vc(plan, ptr, ld, method, outs[0].data_ptr(), outs[1].data_ptr(), outs[2].data_ptr()),
           "clak_estimate_vc")
    return tuple(outs)


def clak_run_block(plan: int, G: torch.Tensor, b: torch.Tensor, se: torch.Tensor,
                   flags: Optional[torch.Tensor] = None, pval: Optional[torch.Tensor] = None,
                   g_dtype: Optional[int] = None):
    """G: (m_blk, ldg) uint8 or float16 SNP rows (uint8 rows of 2-bit codes with g_dtype=CLAK_G_P2);
    b, se, pval: (t, ldo[, p]) float32/64."""
    blk, gdt, odt = _block_args(clak_plan_get_shape(plan), G, b, se, flags, pval, g_dtype)
    _check(lib().clak_run_block(plan, blk.m_blk, blk.G, gdt, blk.ldg, blk.b, blk.se, odt, blk.ldo, blk.flags,
                                blk.pval), "clak_run_block")


def clak_run_block_static(plan: int, G: torch.Tensor, b: torch.Tensor, se: torch.Tensor,
                          flags: Optional[torch.Tensor] = None, pval: Optional[torch.Tensor] = None,
                          g_dtype: Optional[int] = None):
    """clak_run_block with the block's scratch in the library's device array (no allocation)."""
    blk, gdt, odt = _block_args(clak_plan_get_shape(plan), G, b, se, flags, pval, g_dtype)
    _check(lib().clak_run_block_static(plan, blk.m_blk, blk.G, gdt, blk.ldg, blk.b, blk.se, odt, blk.ldo,
                                       blk.flags, blk.pval), "clak_run_block_static")


def clak_plan_block_scratch_size(plan: int) -> int:
    out = _SZ()
    _check(lib().clak_plan_block_scratch_size(plan, ctypes.byref(out)), "clak_plan_block_scratch_size")
    return out.value


def clak_bed_open(path: str, n: int, m: int, block: int, depth: int = 4) -> int:
    """Reader of a SNP-major PLINK 1 binary genotype file (n individuals, m SNPs) in blocks of `block` SNPs."""
    h = _P()
    _check(lib().clak_bed_open(ctypes.byref(h), os.fsencode(path), n, m, block, depth), "clak_bed_open")
    _BED_SNPS[h.value] = int(m)
    return h.value


def clak_bed_scan(bed: int, plan: int, b: torch.Tensor, se: torch.Tensor, flags: Optional[torch.Tensor] = None,
                  pval: Optional[torch.Tensor] = None):
    """Every SNP of the file through the plan; b, se, flags, pval: (t, ldo[, p]) with ldo >= m (synchronous)."""
    for name, x in (("b", b), ("se", se), ("flags", flags), ("pval", pval)):
        if x is not None and not (isinstance(x, torch.Tensor) and x.is_cuda):
            raise ValueError(f"{name} must be a GPU tensor")
    ldo, odt = _out_layout(clak_plan_get_shape(plan), b, se, flags, pval, _BED_SNPS.get(bed, 1))
    fptr = flags.data_ptr() if flags is not None else None
    pptr = pval.data_ptr() if pval is not None else None
    _check(lib().clak_bed_scan(bed, plan, b.data_ptr(), se.data_ptr(), odt, ldo, fptr, pptr), "clak_bed_scan")


def clak_bed_close(bed: int):
    _check(lib().clak_bed_close(bed), "clak_bed_close")
    _BED_SNPS.pop(bed, None)


def clak_plan_set_tuning(plan: int, rot_cfg: int = 0, rot_rg: int = 0, grid_tt: int = 0, grid_xt: int = 0):
    _check(lib().clak_plan_set_tuning(plan, rot_cfg, rot_rg, grid_tt, grid_xt), "clak_plan_set_tuning")


def clak_plan_get_tuning(plan: int):
    """(rot_cfg, rot_rg, grid_tt, grid_xt) in effect; 0 means the built-in choice."""
    v = [ctypes.c_int(0) for _ in range(4)]
    _check(lib().clak_plan_get_tuning(plan, *[ctypes.cast(ctypes.byref(x), _P) for x in v]), "clak_plan_get_tuning")
    return tuple(x.value for x in v)


def clak_autotune(plan: int, G: torch.Tensor, b: torch.Tensor, se: torch.Tensor,
                  flags: Optional[torch.Tensor] = None, cache_path: Optional[str] = None):
    """clak_run_block that first picks (or reads from cache_path) the launch parameters."""
    blk, gdt, odt = _block_args(clak_plan_get_shape(plan), G, b, se, flags)
    cp = cache_path.encode() if cache_path is not None else None
    _check(lib().clak_autotune(plan, blk.m_blk, blk.G, gdt, blk.ldg, blk.b, blk.se, odt, blk.ldo, blk.flags, cp),
           "clak_autotune")


def clak_plan_set_profiling(plan: int, mode=CLAK_PROFILE_SERIAL):
    """mode: CLAK_PROFILE_SERIAL (True), CLAK_PROFILE_PIPELINED, or CLAK_PROFILE_OFF (False)."""
    mode = CLAK_PROFILE_SERIAL if mode is True else CLAK_PROFILE_OFF if mode is False else int(mode)
    _check(lib().clak_plan_set_profiling(plan, mode), "clak_plan_set_profiling")


def clak_plan_get_profile(plan: int):
    """{stage name: (total ms, launches)} since profiling was enabled."""
    ms = (ctypes.c_double * CLAK_STAGE_COUNT)()
    n = (ctypes.c_int64 * CLAK_STAGE_COUNT)()
    _check(lib().clak_plan_get_profile(plan, ctypes.cast(ms, _P), ctypes.cast(n, _P)), "clak_plan_get_profile")
    return {STAGE_NAMES[i]: (ms[i], n[i]) for i in range(CLAK_STAGE_COUNT)}


def clak_plan_get_busy(plan: int):
    """{stage name: ms during which at least one of its timed launches ran} since profiling was enabled."""
    busy = (ctypes.c_double * CLAK_STAGE_COUNT)()
    _check(lib().clak_plan_get_busy(plan, ctypes.cast(busy, _P)), "clak_plan_get_busy")
    return {STAGE_NAMES[i]: busy[i] for i in range(CLAK_STAGE_COUNT)}


def _out_layout(shape: Shape, b, se, flags, pval, m_blk: int):
    """(ldo, out_dtype) after checking the outputs of m_blk SNPs against the
    plan: se (t, >= m_blk) with unit-strided rows, b with se's layout (or
    (t, >= m_blk, p_L + 1), entries of a cell contiguous, under CLAK_OUT_FULL),
    flags (uint8) and pval (se's dtype) with se's layout."""
    t, p = shape.t, shape.p_L + 1
    if b.dtype != se.dtype or b.dtype not in (torch.float32, torch.float64):
        raise ValueError("b and se must share dtype float32 or float64")
    odt = CLAK_OUT_F32 if b.dtype == torch.float32 else CLAK_OUT_F64
    if se.dim() != 2 or se.stride(1) != 1:
        raise ValueError("se must be (t, ldo) with contiguous rows")
    if se.shape[0] < t or se.shape[1] < m_blk:
        raise ValueError(f"se has shape {tuple(se.shape)}; the plan writes (t={t}, m_blk={m_blk})")
    ldo = se.stride(0) if se.shape[0] > 1 else se.shape[1]
    if ldo < se.shape[1]:
        raise ValueError("se rows overlap (row stride below the row length)")

    def same_rows(x, name, row_stride, trailing=()):
        if x.dim() != 2 + len(trailing) or x.shape[0] < t or x.shape[1] < m_blk:
            raise ValueError(f"{name} has shape {tuple(x.shape)}; the plan writes (t={t}, m_blk={m_blk}"
                             + "".join(f", {d}" for d in trailing) + ")")
        want = (row_stride,) + tuple(int(np.prod(trailing[i:])) for i in range(len(trailing) + 1))
        got = tuple(x.stride())
        if got[1:] != want[1:] or (t > 1 and got[0] != want[0]):
            raise ValueError(f"{name} strides {got} do not match the output layout {want}")

    if shape.flags & CLAK_OUT_FULL:
        same_rows(b, "b", ldo * p, (p,))
    else:
        same_rows(b, "b", ldo)
    if flags is not None:
        if flags.dtype != torch.uint8:
            raise ValueError("flags must be uint8")
        same_rows(flags, "flags", ldo)
    if pval is not None:
        if pval.dtype != se.dtype:
            raise ValueError("pval must have the dtype of se")
        same_rows(pval, "pval", ldo)
    return ldo, odt


def _block_layout(shape: Shape, G, b, se, flags=None, pval=None, g_dtype=None):
    """(m_blk, ldg, g_dtype, ldo, out_dtype) of one block, every tensor checked
    against the plan's sizes (device-independent part of the checks)."""
    if g_dtype == CLAK_G_P2:
        if G.dtype != torch.uint8:
            raise ValueError("2-bit genotype rows must be a uint8 tensor")
        gdt, row = CLAK_G_P2, (shape.n + 3) // 4
    elif G.dtype == torch.uint8:
        gdt, row = CLAK_G_U8, shape.n
    elif G.dtype == torch.float16:
        gdt, row = CLAK_G_F16, shape.n
    else:
        raise ValueError("G must be uint8 or float16")
    if G.dim() != 2 or G.stride(1) != 1:
        raise ValueError("G must be 2-D with contiguous rows (one SNP per row)")
    m_blk = G.shape[0]
    if not 1 <= m_blk <= shape.max_block:
        raise ValueError(f"G holds {m_blk} SNPs; the plan takes 1 to max_block={shape.max_block}")
    if G.shape[1] < row:
        raise ValueError(f"G rows hold {G.shape[1]} entries; one SNP of n={shape.n} needs {row}")
    ldg = G.stride(0) if m_blk > 1 else G.shape[1]
    ldo, odt = _out_layout(shape, b, se, flags, pval, m_blk)
    return m_blk, ldg, gdt, ldo, odt


def _block_args(shape: Shape, G, b, se, flags=None, pval=None, g_dtype=None):
    """(clak_block, g_dtype, out_dtype) for one block, with the checks of clak_run_block."""
    _dev(G, "G")
    _dev(b, "b")
    _dev(se, "se")
    if flags is not None:
        _dev(flags, "flags")
    if pval is not None:
        _dev(pval, "pval")
    m_blk, ldg, gdt, ldo, odt = _block_layout(shape, G, b, se, flags, pval, g_dtype)
    blk = clak_block(m_blk, G.data_ptr(), ldg, b.data_ptr(), se.data_ptr(), ldo,
                     flags.data_ptr() if flags is not None else None, pval.data_ptr() if pval is not None else None)
    return blk, gdt, odt


def _block_array(shape: Shape, blocks):
    """blocks: sequence of (G, b, se[, flags[, pval]]) -> ctypes array, g_dtype, out_dtype."""
    items = [_block_args(shape, *blk) for blk in blocks]
    if not items:
        raise ValueError("no blocks")
    gdts = {it[1] for it in items}
    odts = {it[2] for it in items}
    if len(gdts) != 1 or len(odts) != 1:
        raise ValueError("all blocks must share the genotype and output dtypes")
    arr = (clak_block * len(items))(*[it[0] for it in items])
    return arr, items[0][1], items[0][2]


def clak_pipeline_create(plan: int, blocks) -> int:
    """Two-stream pipeline over blocks = [(G, b, se[, flags]), ...]: the ingest of a block
    overlaps the rotation and grid of the previous one."""
    arr, gdt, odt = _block_array(clak_plan_get_shape(plan), blocks)
    h = _P()
    _check(lib().clak_pipeline_create(ctypes.byref(h), plan, len(arr), arr, gdt, odt), "clak_pipeline_create")
    return h.value


def clak_autotune_pipeline(plan: int, blocks, cache_path: Optional[str] = None):
    """Picks the launch parameters by timing the pipeline over blocks = [(G, b, se[, flags]), ...]."""
    arr, gdt, odt = _block_array(clak_plan_get_shape(plan), blocks)
    cp = cache_path.encode() if cache_path is not None else None
    _check(lib().clak_autotune_pipeline(plan, len(arr), arr, gdt, odt, cp), "clak_autotune_pipeline")


def clak_pipeline_launch(pipe: int):
    _check(lib().clak_pipeline_launch(pipe), "clak_pipeline_launch")


def clak_pipeline_destroy(pipe: int):
    _check(lib().clak_pipeline_destroy(pipe), "clak_pipeline_destroy")


def clak_batch_create(plans, blocks_per_plan) -> int:
    """One submission over several plans (cohorts); blocks_per_plan[k] = [(G, b, se[, flags]), ...]."""
    if len(plans) != len(blocks_per_plan):
        raise ValueError("one block list per plan")
    parts = [_block_array(clak_plan_get_shape(p), bl) for p, bl in zip(plans, blocks_per_plan)]
    if len({x[1] for x in parts}) != 1 or len({x[2] for x in parts}) != 1:
        raise ValueError("all blocks must share the genotype and output dtypes")
    flat = [blk for x in parts for blk in x[0]]
    arr = (clak_block * len(flat))(*flat)
    gdt, odt = parts[0][1], parts[0][2]
    ph = (_P * len(plans))(*plans)
    nb = (_I64 * len(plans))(*[len(bl) for bl in blocks_per_plan])
    h = _P()
    _check(lib().clak_batch_create(ctypes.byref(h), len(plans), ph, nb, arr, gdt, odt), "clak_batch_create")
    return h.value


def clak_batch_launch(batch: int, stream: Optional[torch.cuda.Stream] = None):
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(lib().clak_batch_launch(batch, s.cuda_stream), "clak_batch_launch")


def clak_batch_get_info(batch: int):
    """(batched, rounds, streams) of a batch."""
    b, r, s = ctypes.c_int(0), ctypes.c_int64(0), ctypes.c_int(0)
    _check(lib().clak_batch_get_info(batch, ctypes.cast(ctypes.byref(b), _P), ctypes.cast(ctypes.byref(r), _P),
                                     ctypes.cast(ctypes.byref(s), _P)), "clak_batch_get_info")
    return bool(b.value), r.value, s.value


def clak_batch_destroy(batch: int):
    _check(lib().clak_batch_destroy(batch), "clak_batch_destroy")


def clak_plan_destroy(plan: int):
    _check(lib().clak_plan_destroy(plan), "clak_plan_destroy")


class Plan:
    """Owns one plan and its torch-allocated workspace (convenience wrapper)."""

    def __init__(self, n, p_L, t, max_block, precision=CLAK_PREC_FP64, flags=0, device=None,
                 stream: Optional[torch.cuda.Stream] = None):
        dev = torch.device("cuda" if device is None else device)
        with torch.cuda.device(dev):
            self.handle = clak_plan_create(n, p_L, t, max_block, precision, flags)
            try:
                nbytes = clak_plan_workspace_size(self.handle)
                self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
                clak_plan_set_workspace(self.handle, self.workspace)
                clak_plan_set_stream(self.handle, stream)
            except Exception:
                clak_plan_destroy(self.handle)
                raise
        self.n, self.p_L, self.t, self.max_block, self.precision, self.flags = n, p_L, t, max_block, precision, flags

    def close(self):
        if getattr(self, "handle", None):
            clak_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
