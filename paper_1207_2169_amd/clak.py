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
from typing import Optional

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
    "clak_plan_destroy": (_I, [_P]),
    "clak_plan_set_profiling": (_I, [_P, _I]),
    "clak_plan_set_tuning": (_I, [_P, _I, _I, _I, _I]),
    "clak_plan_get_tuning": (_I, [_P, _P, _P, _P, _P]),
    "clak_autotune": (_I, [_P, _I64, _P, _I, _I64, _P, _P, _I, _I64, _P, ctypes.c_char_p]),
    "clak_plan_get_profile": (_I, [_P, _P, _P]),
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
    "clak_batch_destroy": (_I, [_P]),
})

_lib_handle = None


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


def _colmajor(A: torch.Tensor, what: str):
    """(pointer, leading dimension, keep-alive tensor) of an n x c matrix."""
    _dev(A, what, torch.float64)
    if A.dim() == 1:
        A = A.reshape(-1, 1)
    if A.dim() != 2:
        raise ValueError(f"{what} must be 2-D")
    if A.stride(0) != 1 and A.shape[1] > 1:
        A = A.t().contiguous().t()
    ld = A.stride(1) if A.shape[1] > 1 else A.shape[0]
    return A.data_ptr(), max(ld, A.shape[0]), A


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
    ptr, ld, _keep = _colmajor(Phi, "Phi")
    _check(lib().clak_set_kinship(plan, ptr, ld), "clak_set_kinship")


def clak_set_eigen(plan: int, Z: torch.Tensor, w: torch.Tensor):
    ptr, ld, _keep = _colmajor(Z, "Z")
    w = _dev(w, "w", torch.float64).contiguous()
    _check(lib().clak_set_eigen(plan, ptr, ld, w.data_ptr()), "clak_set_eigen")


def clak_set_covariates(plan: int, XL: torch.Tensor):
    ptr, ld, _keep = _colmajor(XL, "X_L")
    _check(lib().clak_set_covariates(plan, ptr, ld), "clak_set_covariates")


def clak_set_traits(plan: int, Y: torch.Tensor, h2: torch.Tensor, s2: torch.Tensor):
    ptr, ld, _keep = _colmajor(Y, "Y")
    h2 = _dev(h2, "h2", torch.float64).contiguous()
    s2 = _dev(s2, "s2", torch.float64).contiguous()
    _check(lib().clak_set_traits(plan, ptr, ld, h2.data_ptr(), s2.data_ptr()), "clak_set_traits")


def clak_estimate_vc(plan: int, Y: torch.Tensor, method: int = CLAK_VC_REML, h2: Optional[torch.Tensor] = None,
                     s2: Optional[torch.Tensor] = None, loglik: Optional[torch.Tensor] = None):
    """Per-trait (h2, s2, loglik) of the reduced model; outputs are allocated when not given (float64, t values)."""
    ptr, ld, _keep = _colmajor(Y, "Y")
    t = _keep.shape[1]  # must be the plan's t
    outs = []
    for name, x in (("h2", h2), ("s2", s2), ("loglik", loglik)):
        if x is None:
            x = torch.empty(t, dtype=torch.float64, device=Y.device)
        x = _dev(x, name, torch.float64)
        if not x.is_contiguous() or x.numel() < t:
            raise ValueError(f"{name}: need a contiguous float64 tensor of at least t={t} values")
        outs.append(x)
    _check(lib().clak_estimate_vc(plan, ptr, ld, method, outs[0].data_ptr(), outs[1].data_ptr(), outs[2].data_ptr()),
           "clak_estimate_vc")
    return tuple(outs)


def clak_run_block(plan: int, G: torch.Tensor, b: torch.Tensor, se: torch.Tensor,
                   flags: Optional[torch.Tensor] = None, pval: Optional[torch.Tensor] = None,
                   g_dtype: Optional[int] = None):
    """G: (m_blk, ldg) uint8 or float16 SNP rows (uint8 rows of 2-bit codes with g_dtype=CLAK_G_P2);
    b, se, pval: (t, ldo[, p]) float32/64."""
    blk, gdt, odt = _block_args(G, b, se, flags, pval, g_dtype)
    _check(lib().clak_run_block(plan, blk.m_blk, blk.G, gdt, blk.ldg, blk.b, blk.se, odt, blk.ldo, blk.flags,
                                blk.pval), "clak_run_block")


def clak_bed_open(path: str, n: int, m: int, block: int, depth: int = 4) -> int:
    """Reader of a SNP-major PLINK 1 binary genotype file (n individuals, m SNPs) in blocks of `block` SNPs."""
    h = _P()
    _check(lib().clak_bed_open(ctypes.byref(h), os.fsencode(path), n, m, block, depth), "clak_bed_open")
    return h.value


def clak_bed_scan(bed: int, plan: int, b: torch.Tensor, se: torch.Tensor, flags: Optional[torch.Tensor] = None,
                  pval: Optional[torch.Tensor] = None):
    """Every SNP of the file through the plan; b, se, flags, pval: (t, ldo[, p]) with ldo >= m (synchronous)."""
    for name, x in (("b", b), ("se", se)):
        if not (isinstance(x, torch.Tensor) and x.is_cuda):
            raise ValueError(f"{name} must be a GPU tensor")
    if b.dtype != se.dtype or b.dtype not in (torch.float32, torch.float64):
        raise ValueError("b and se must share dtype float32 or float64")
    if se.dim() != 2 or se.stride(1) != 1:
        raise ValueError("se must be (t, ldo) with contiguous rows")
    ldo = se.stride(0) if se.shape[0] > 1 else se.shape[1]
    fptr = pptr = None
    if flags is not None:
        if flags.dtype != torch.uint8 or flags.shape != se.shape or flags.stride() != se.stride():
            raise ValueError("flags must be uint8 with the layout of se")
        fptr = flags.data_ptr()
    if pval is not None:
        if pval.dtype != se.dtype or pval.shape != se.shape or pval.stride() != se.stride():
            raise ValueError("pval must match se")
        pptr = pval.data_ptr()
    odt = CLAK_OUT_F32 if b.dtype == torch.float32 else CLAK_OUT_F64
    _check(lib().clak_bed_scan(bed, plan, b.data_ptr(), se.data_ptr(), odt, ldo, fptr, pptr), "clak_bed_scan")


def clak_bed_close(bed: int):
    _check(lib().clak_bed_close(bed), "clak_bed_close")


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
    blk, gdt, odt = _block_args(G, b, se, flags)
    cp = cache_path.encode() if cache_path is not None else None
    _check(lib().clak_autotune(plan, blk.m_blk, blk.G, gdt, blk.ldg, blk.b, blk.se, odt, blk.ldo, blk.flags, cp),
           "clak_autotune")


def clak_plan_set_profiling(plan: int, enable: bool = True):
    _check(lib().clak_plan_set_profiling(plan, 1 if enable else 0), "clak_plan_set_profiling")


def clak_plan_get_profile(plan: int):
    """{stage name: (total ms, launches)} since profiling was enabled."""
    ms = (ctypes.c_double * CLAK_STAGE_COUNT)()
    n = (ctypes.c_int64 * CLAK_STAGE_COUNT)()
    _check(lib().clak_plan_get_profile(plan, ctypes.cast(ms, _P), ctypes.cast(n, _P)), "clak_plan_get_profile")
    return {STAGE_NAMES[i]: (ms[i], n[i]) for i in range(CLAK_STAGE_COUNT)}


def _block_args(G, b, se, flags=None, pval=None, g_dtype=None):
    """(clak_block, g_dtype, out_dtype) for one block, with the checks of clak_run_block."""
    _dev(G, "G")
    if g_dtype == CLAK_G_P2:
        if G.dtype != torch.uint8:
            raise ValueError("2-bit genotype rows must be a uint8 tensor")
        gdt = CLAK_G_P2
    elif G.dtype == torch.uint8:
        gdt = CLAK_G_U8
    elif G.dtype == torch.float16:
        gdt = CLAK_G_F16
    else:
        raise ValueError("G must be uint8 or float16")
    if G.dim() != 2 or G.stride(1) != 1:
        raise ValueError("G must be 2-D with contiguous rows (one SNP per row)")
    _dev(b, "b")
    _dev(se, "se")
    if b.dtype != se.dtype or b.dtype not in (torch.float32, torch.float64):
        raise ValueError("b and se must share dtype float32 or float64")
    odt = CLAK_OUT_F32 if b.dtype == torch.float32 else CLAK_OUT_F64
    if se.dim() != 2 or se.stride(1) != 1:
        raise ValueError("se must be (t, ldo) with contiguous rows")
    ldo = se.stride(0) if se.shape[0] > 1 else se.shape[1]
    fptr = None
    if flags is not None:
        _dev(flags, "flags", torch.uint8)
        if flags.shape != se.shape or flags.stride() != se.stride():
            raise ValueError("flags must match the layout of se")
        fptr = flags.data_ptr()
    pptr = None
    if pval is not None:
        _dev(pval, "pval", se.dtype)
        if pval.shape != se.shape or pval.stride() != se.stride():
            raise ValueError("pval must match the layout of se")
        pptr = pval.data_ptr()
    blk = clak_block(G.shape[0], G.data_ptr(), G.stride(0), b.data_ptr(), se.data_ptr(), ldo, fptr, pptr)
    return blk, gdt, odt


def _block_array(blocks):
    """blocks: sequence of (G, b, se[, flags[, pval]]) -> ctypes array, g_dtype, out_dtype."""
    items = [_block_args(*blk) for blk in blocks]
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
    arr, gdt, odt = _block_array(blocks)
    h = _P()
    _check(lib().clak_pipeline_create(ctypes.byref(h), plan, len(arr), arr, gdt, odt), "clak_pipeline_create")
    return h.value


def clak_pipeline_launch(pipe: int):
    _check(lib().clak_pipeline_launch(pipe), "clak_pipeline_launch")


def clak_pipeline_destroy(pipe: int):
    _check(lib().clak_pipeline_destroy(pipe), "clak_pipeline_destroy")


def clak_batch_create(plans, blocks_per_plan) -> int:
    """One submission over several plans (cohorts); blocks_per_plan[k] = [(G, b, se[, flags]), ...]."""
    flat = [blk for bl in blocks_per_plan for blk in bl]
    arr, gdt, odt = _block_array(flat)
    ph = (_P * len(plans))(*plans)
    nb = (_I64 * len(plans))(*[len(bl) for bl in blocks_per_plan])
    h = _P()
    _check(lib().clak_batch_create(ctypes.byref(h), len(plans), ph, nb, arr, gdt, odt), "clak_batch_create")
    return h.value


def clak_batch_launch(batch: int, stream: Optional[torch.cuda.Stream] = None):
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(lib().clak_batch_launch(batch, s.cuda_stream), "clak_batch_launch")


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
