// C ABI of libclak: argument validation, call-order state machine, workspace
// carve-up, the FP64 eigensolver call and the per-block launch sequence.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "clak_internal.hpp"

using namespace clak;

namespace clak {

thread_local std::string g_err;

clak_status fail(clak_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

clak_status ok() {
  g_err.clear();
  return CLAK_OK;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return fail(CLAK_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

Plan* as_plan(clak_plan_t h) { return reinterpret_cast<Plan*>(h); }
Plan* as_plan_public(clak_plan_t h) { return as_plan(h); }

clak_status need_state(const Plan* p, int min_state, const char* what) {
  if (!p) return fail(CLAK_E_ARG, "%s: null plan", what);
  if (p->state < min_state) {
    static const char* names[] = {"workspace", "workspace", "kinship/eigen", "covariates", "traits"};
    return fail(CLAK_E_STATE, "%s: call order: %s must be set first", what, names[min_state]);
  }
  return CLAK_OK;
}

bool aligned(const void* ptr, size_t a) { return (reinterpret_cast<uintptr_t>(ptr) % a) == 0; }

CellOut cell_out(void* b, void* se, void* pval, uint8_t* flags, int64_t ldo, int out_dtype) {
  CellOut o;
  o.b = b;
  o.se = se;
  o.pval = pval;
  o.flags = flags;
  o.ldo = ldo;
  o.f64 = out_dtype == CLAK_OUT_F64;
  return o;
}

// True when the kernels of this device may dereference ptr: device memory of
// the plan's device, managed memory, or pinned host memory mapped at the same
// address.  Pageable host memory (which a kernel access would fault on) and
// unknown pointers are refused before anything is launched.
bool device_accessible(const Plan* p, const void* ptr) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, ptr) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  if (a.isManaged) return true;
  if (a.type == hipMemoryTypeDevice) return a.device == p->device;
  if (a.type == hipMemoryTypeHost) {  // the device address of ptr must be ptr itself
    if (!a.devicePointer || !a.hostPointer) return false;
    const char* dp = (const char*)a.devicePointer + ((const char*)ptr - (const char*)a.hostPointer);
    return dp == (const char*)ptr;
  }
  return a.type == hipMemoryTypeUnified || a.type == hipMemoryTypeManaged;
}

hipEvent_t take_event(Plan* p) {
  if (!p->event_pool.empty()) {
    hipEvent_t e = p->event_pool.back();
    p->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Waits for every timed stage, adds its duration, keeps its interval
// relative to the reference event, recycles the events.
clak_status drain_profile(Plan* p) {
  if (p->pending.empty()) return CLAK_OK;
  HIP_TRY(hipDeviceSynchronize());  // the bracketing events may sit on any stream of a pipeline
  for (auto& t : p->pending) {
    float ms = 0.0f, a = 0.0f, b = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, t.a, t.b));
    HIP_TRY(hipEventElapsedTime(&a, p->prof_ref, t.a));
    HIP_TRY(hipEventElapsedTime(&b, p->prof_ref, t.b));
    p->stage_ms[t.stage] += ms;
    p->stage_n[t.stage] += 1;
    p->stage_iv[t.stage].push_back({(double)a, (double)b});
    p->event_pool.push_back(t.a);
    p->event_pool.push_back(t.b);
  }
  p->pending.clear();
  return CLAK_OK;
}

// Length of the union of a stage's launch intervals (the time during which at
// least one of its kernels ran).
static double busy_ms(std::vector<std::pair<double, double>> iv) {
  std::sort(iv.begin(), iv.end());
  double total = 0.0, s = 0.0, e = -1e300;
  for (auto& x : iv) {
    if (x.first > e) {
      if (e > s) total += e - s;
      s = x.first;
      e = x.second;
    } else if (x.second > e) {
      e = x.second;
    }
  }
  if (!iv.empty() && e > s) total += e - s;
  return total;
}

clak_status sync_and_read_status(Plan* p) {
  HIP_TRY(hipMemcpyAsync(p->hstat, p->ws.dstat, sizeof(int) * DS_COUNT, hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  return CLAK_OK;
}

// Carves the buffers of one block slot from base (256-byte aligned pieces);
// returns their size.  With base == nullptr only the size is computed.
size_t slot_bytes(const Plan& p, Slot* S, char* base) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* ptr = base ? base + off : nullptr;
    off += (bytes + 255) / 256 * 256;
    return ptr;
  };
  const size_t np = p.n_pad, pl = p.pL, mb = p.mb_pad;
  Slot tmp;
  Slot& T = S ? *S : tmp;
  T = Slot();
  T.Gp = (int8_t*)take(mb * np);
  T.sstat = (double*)take(8 * mb * snp_stride(p.pL));
  T.ipart = (double*)take(8 * ING_MAX_SPLITS * (pl + 2) * mb);
  if (p.fused_t1) T.part = (double*)take(8 * (np / 64) * mb * (pl + 2));
  if (!p.fused_t1) T.X64 = (double*)take(8 * mb * np);
  if (p.prec == CLAK_PREC_MIXED && !p.fused_t1) T.Xd = (int8_t*)take(8 * mb * np);
  if (p.flags & CLAK_STAGE_GENOTYPES) T.Gh = (uint8_t*)take(p.max_block * host_pitch(p.n));
  return off;
}

// Carves the workspace.  With base == nullptr only the size is computed.
size_t workspace_bytes(const Plan& p, Workspace* w, char* base) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* ptr = base ? base + off : nullptr;
    off += (bytes + 255) / 256 * 256;
    return ptr;
  };
  const size_t np = p.n_pad, pl = p.pL, tp = p.t_pad;
  Workspace tmp;
  Workspace& W = w ? *w : tmp;
  W.Zt = (double*)take(8 * p.zrows * np);
  W.w = (double*)take(8 * np);
  W.evE = (double*)take(8 * np);
  W.dstat = (int*)take(sizeof(int) * DS_COUNT);
  W.QL = (double*)take(8 * np * pl);
  W.Rm = (double*)take(8 * pl * pl);
  W.Rinv = (double*)take(8 * pl * pl);
  W.XLt = (double*)take(8 * np * pl);
  W.Qt = (double*)take(8 * np * pl);
  W.Yt = (double*)take(8 * np * p.t);
  W.tpar = (double*)take(8 * tp * trait_stride(p.pL));
  if (p.flags & CLAK_CHOL) {
    W.Phi = (double*)take(8 * np * np);
    W.XL = (double*)take(8 * np * pl);
  }
  if (p.prec == CLAK_PREC_FP64 || p.fused_t1) {
    W.V64 = (double*)take(8 * tp * (pl + 1) * np);
    W.D64 = (double*)take(8 * tp * np);
  }
  if (p.prec == CLAK_PREC_MIXED) {
    W.Zd = (int8_t*)take(4 * p.zrows * np);
    W.zs = (double*)take(8 * p.zrows);
  }
  if (lin_rows(p)) W.Cq = (double*)take(8 * pl * (pl + 1));
  if (p.prec == CLAK_PREC_MIXED && !p.fused_t1) {
    W.Vd = (int8_t*)take(4 * tp * (pl + 1) * np);
    W.Dd = (int8_t*)take(4 * tp * np);
    W.vs = (double*)take(8 * tp * (pl + 1));
    W.ds = (double*)take(8 * tp);
  }
  for (int k = 0; k < NSLOTS; ++k) {
    const size_t sb = slot_bytes(p, &W.slot[k], base ? base + off : nullptr);
    off += sb;
  }
  if (w) {
    const Slot& S = W.slot[0];
    W.Gp = S.Gp;
    W.sstat = S.sstat;
    W.ipart = S.ipart;
    W.part = S.part;
    W.X64 = S.X64;
    W.Xd = S.Xd;
  }
  return off;
}

// The plan's sizes and derived paddings (no device call).
void init_shape(Plan& p, int64_t n, int64_t p_L, int64_t t, int64_t max_block, int precision, uint32_t flags) {
  p.n = n;
  p.pL = p_L;
  p.t = t;
  p.max_block = max_block;
  p.prec = precision;
  p.flags = flags;
  p.n_pad = roundup(n, KPAD);
  p.mb_pad = roundup(max_block, SNP_PAD);
  p.t_pad = roundup(t, TRAIT_PAD);
  p.fused_t1 = (t == 1);
  p.zlin = (lin_rows(p) && n + p_L + 1 <= p.n_pad) ? n : p.n_pad;
  p.zrows = p.n_pad + ((lin_rows(p) && p.zlin == p.n_pad) ? ZEXT : 0);
}

}  // namespace clak

extern "C" {

const char* clak_last_error(void) { return g_err.c_str(); }

const char* clak_version(void) { return "clak-mi355x 0.1 (gfx950)"; }

clak_status clak_plan_create(clak_plan_t* out, int64_t n, int64_t p_L, int64_t t, int64_t max_block,
                             int precision, uint32_t flags) {
  if (!out) return fail(CLAK_E_ARG, "plan_create: null output pointer");
  *out = nullptr;
  if (p_L < 1 || p_L > MAX_PL) return fail(CLAK_E_ARG, "plan_create: p_L=%lld outside [1,%d]", (long long)p_L, MAX_PL);
  if (n <= p_L) return fail(CLAK_E_ARG, "plan_create: need n > p_L (n=%lld)", (long long)n);
  if (t < 1) return fail(CLAK_E_ARG, "plan_create: t must be >= 1");
  if (max_block < 1) return fail(CLAK_E_ARG, "plan_create: max_block must be >= 1");
  if (precision != CLAK_PREC_FP64 && precision != CLAK_PREC_MIXED)
    return fail(CLAK_E_ARG, "plan_create: unknown precision %d", precision);
  if (flags & ~(CLAK_VAR_PAPER | CLAK_OUT_FULL | CLAK_STAGE_GENOTYPES | CLAK_CHOL))
    return fail(CLAK_E_ARG, "plan_create: unknown flags 0x%x", flags);
  if ((flags & CLAK_CHOL) && t != 1) return fail(CLAK_E_ARG, "plan_create: CLAK_CHOL needs t = 1");
  if (precision == CLAK_PREC_MIXED && p_L > 8)
    return fail(CLAK_E_UNSUPPORTED, "plan_create: mixed precision supports p_L <= 8");
  if (precision == CLAK_PREC_MIXED && n > MIXED_MAX_N)
    return fail(CLAK_E_UNSUPPORTED, "plan_create: mixed precision supports n <= %lld", (long long)MIXED_MAX_N);
  if (n > (int64_t)1 << 20 || t > (int64_t)1 << 24 || max_block > (int64_t)1 << 26)
    return fail(CLAK_E_UNSUPPORTED, "plan_create: size too large");
  Plan* p = new (std::nothrow) Plan();
  if (!p) return fail(CLAK_E_DEVICE, "plan_create: out of host memory");
  init_shape(*p, n, p_L, t, max_block, precision, flags);
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return fail(CLAK_E_DEVICE, "plan_create: no HIP device");
  }
  rocblas_handle h = nullptr;
  if (rocblas_create_handle(&h) != rocblas_status_success) {
    delete p;
    return fail(CLAK_E_DEVICE, "plan_create: rocblas_create_handle failed");
  }
  p->rocblas = h;
  if (hipHostMalloc((void**)&p->hstat, sizeof(int) * DS_COUNT, hipHostMallocDefault) != hipSuccess) {
    rocblas_destroy_handle(h);
    delete p;
    return fail(CLAK_E_DEVICE, "plan_create: pinned status buffer");
  }
  *out = reinterpret_cast<clak_plan_t>(p);
  return ok();
}

clak_status clak_plan_workspace_size(clak_plan_t h, size_t* bytes) {
  Plan* p = as_plan(h);
  if (!p || !bytes) return fail(CLAK_E_ARG, "plan_workspace_size: null argument");
  *bytes = workspace_bytes(*p, nullptr, nullptr);
  return ok();
}

clak_status clak_plan_set_workspace(clak_plan_t h, void* d_ws, size_t bytes) {
  Plan* p = as_plan(h);
  if (!p) return fail(CLAK_E_ARG, "plan_set_workspace: null plan");
  if (!d_ws) return fail(CLAK_E_WORKSPACE, "plan_set_workspace: null workspace");
  if (!aligned(d_ws, 256)) return fail(CLAK_E_WORKSPACE, "plan_set_workspace: workspace not 256-byte aligned");
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, d_ws) != hipSuccess || a.type != hipMemoryTypeDevice || a.device != p->device) {
    (void)hipGetLastError();
    return fail(CLAK_E_WORKSPACE, "plan_set_workspace: the workspace must be device memory of the plan's device");
  }
  size_t need = workspace_bytes(*p, nullptr, nullptr);
  if (bytes < need)
    return fail(CLAK_E_WORKSPACE, "plan_set_workspace: %zu bytes given, %zu needed", bytes, need);
  p->ws_base = d_ws;
  p->ws_bytes = bytes;
  workspace_bytes(*p, &p->ws, (char*)d_ws);
  p->state = ST_WS;
  return ok();
}

clak_status clak_plan_set_stream(clak_plan_t h, void* stream) {
  Plan* p = as_plan(h);
  if (!p) return fail(CLAK_E_ARG, "plan_set_stream: null plan");
  p->stream = (hipStream_t)stream;
  return ok();
}

// CLAK-Chol set-up of one trait: H = h2 Phi + (1 - h2) I = U^T U, U^-1 in
// place, rotation rows U^-T with unit weights, then the rotations of X_L and
// Q_L by it (what set_kinship and set_covariates do for CLAK-Eig).
static clak_status chol_factor(Plan* p, const double* d_h2) {
  Workspace& W = p->ws;
  const int64_t n = p->n, np = p->n_pad;
  HIP_TRY(hipMemsetAsync(W.dstat, 0, sizeof(int) * DS_COUNT, p->stream));
  HIP_TRY(launch_chol_build(*p, d_h2));
  clak_status s = sync_and_read_status(p);
  if (s) return s;
  if (p->hstat[DS_TRAIT_ARG]) return fail(CLAK_E_ARG, "set_traits: h2 outside [0,1]");
  rocblas_handle rb = (rocblas_handle)p->rocblas;
  if (rocblas_set_stream(rb, p->stream) != rocblas_status_success)
    return fail(CLAK_E_DEVICE, "set_traits: rocblas_set_stream failed");
  rocblas_status rs = rocsolver_dpotrf(rb, rocblas_fill_upper, (rocblas_int)n, W.Zt, (rocblas_int)np,
                                       W.dstat + DS_EIG_INFO);
  if (rs != rocblas_status_success) return fail(CLAK_E_DEVICE, "set_traits: rocsolver_dpotrf status %d", (int)rs);
  s = sync_and_read_status(p);
  if (s) return s;
  if (p->hstat[DS_EIG_INFO] != 0)
    return fail(CLAK_E_NOT_SPD, "set_traits: h2 Phi + (1 - h2) I is not positive definite (pivot %d)",
                p->hstat[DS_EIG_INFO]);
  rs = rocsolver_dtrtri(rb, rocblas_fill_upper, rocblas_diagonal_non_unit, (rocblas_int)n, W.Zt, (rocblas_int)np,
                        W.dstat + DS_EIG_INFO);
  if (rs != rocblas_status_success) return fail(CLAK_E_DEVICE, "set_traits: rocsolver_dtrtri status %d", (int)rs);
  HIP_TRY(launch_chol_fix(*p));
  HIP_TRY(launch_check_eigen(*p));
  if (p->prec == CLAK_PREC_MIXED) HIP_TRY(launch_split_digits(*p, 0, p->n_pad));
  HIP_TRY(launch_rotate_real(*p, W.XL, np, p->pL, W.XLt, np));
  if (p->prec == CLAK_PREC_MIXED)
    HIP_TRY(launch_qt_digits(*p));  // the centring rotation by the digit-encoded operand
  else
    HIP_TRY(launch_rotate_real(*p, W.QL, np, p->pL, W.Qt, np));
  s = sync_and_read_status(p);
  if (s) return s;
  if (p->hstat[DS_EIG_INFO] != 0) return fail(CLAK_E_NOT_SPD, "set_traits: singular Cholesky factor");
  if (p->hstat[DS_EIGVAL]) return fail(CLAK_E_ARG, "set_traits: non-finite inverse Cholesky factor");
  return CLAK_OK;
}

static clak_status finish_eigen(Plan* p) {
  // zero the status words, validate the eigenpairs, split Z^T into digits
  HIP_TRY(launch_check_eigen(*p));
  if (p->prec == CLAK_PREC_MIXED) HIP_TRY(launch_split_digits(*p, 0, p->n_pad));
  clak_status s = sync_and_read_status(p);
  if (s != CLAK_OK) return s;
  if (p->hstat[DS_EIGVAL]) return fail(CLAK_E_ARG, "non-finite eigenvalues or eigenvectors");
  p->state = ST_EIG;
  return ok();
}

clak_status clak_set_kinship(clak_plan_t h, const double* d_Phi, int64_t ld) {
  Plan* p = as_plan(h);
  clak_status s = need_state(p, ST_WS, "set_kinship");
  if (s) return s;
  if (!d_Phi) return fail(CLAK_E_ARG, "set_kinship: null Phi");
  if (!device_accessible(p, d_Phi)) return fail(CLAK_E_ARG, "set_kinship: Phi is not device-accessible memory");
  if (ld < p->n) return fail(CLAK_E_ARG, "set_kinship: ld=%lld < n", (long long)ld);
  p->state = ST_WS;
  const int64_t n = p->n, np = p->n_pad;
  Workspace& W = p->ws;
  if (p->flags & CLAK_CHOL) {
    // CLAK-Chol: keep Phi; the factorisation needs h2 and happens in set_traits
    HIP_TRY(hipMemsetAsync(W.dstat, 0, sizeof(int) * DS_COUNT, p->stream));
    HIP_TRY(hipMemcpy2DAsync(W.Phi, sizeof(double) * np, d_Phi, sizeof(double) * ld, sizeof(double) * n, n,
                             hipMemcpyDeviceToDevice, p->stream));
    HIP_TRY(launch_chol_check(*p));
    s = sync_and_read_status(p);
    if (s) return s;
    if (p->hstat[DS_EIGVAL]) return fail(CLAK_E_ARG, "set_kinship: non-finite Phi");
    p->state = ST_EIG;
    return ok();
  }
  HIP_TRY(hipMemsetAsync(W.Zt, 0, sizeof(double) * np * np, p->stream));
  HIP_TRY(hipMemsetAsync(W.w, 0, sizeof(double) * np, p->stream));
  HIP_TRY(hipMemsetAsync(W.dstat, 0, sizeof(int) * DS_COUNT, p->stream));
  HIP_TRY(hipMemcpy2DAsync(W.Zt, sizeof(double) * np, d_Phi, sizeof(double) * ld, sizeof(double) * n, n,
                           hipMemcpyDeviceToDevice, p->stream));
  rocblas_handle rb = (rocblas_handle)p->rocblas;
  if (rocblas_set_stream(rb, p->stream) != rocblas_status_success)
    return fail(CLAK_E_DEVICE, "set_kinship: rocblas_set_stream failed");
  rocblas_status rs = rocsolver_dsyevd(rb, rocblas_evect_original, rocblas_fill_lower, (rocblas_int)n, W.Zt,
                                       (rocblas_int)np, W.w, W.evE, W.dstat + DS_EIG_INFO);
  if (rs != rocblas_status_success) return fail(CLAK_E_DEVICE, "set_kinship: rocsolver_dsyevd status %d", (int)rs);
  s = sync_and_read_status(p);
  if (s) return s;
  if (p->hstat[DS_EIG_INFO] != 0)
    return fail(CLAK_E_EIG, "set_kinship: eigensolver did not converge (info=%d)", p->hstat[DS_EIG_INFO]);
  return finish_eigen(p);
}

clak_status clak_set_eigen(clak_plan_t h, const double* d_Z, int64_t ldz, const double* d_w) {
  Plan* p = as_plan(h);
  clak_status s = need_state(p, ST_WS, "set_eigen");
  if (s) return s;
  if (p->flags & CLAK_CHOL) return fail(CLAK_E_UNSUPPORTED, "set_eigen: a CLAK_CHOL plan takes Phi (set_kinship)");
  if (!d_Z || !d_w) return fail(CLAK_E_ARG, "set_eigen: null Z or w");
  if (!device_accessible(p, d_Z) || !device_accessible(p, d_w))
    return fail(CLAK_E_ARG, "set_eigen: Z or w is not device-accessible memory");
  if (ldz < p->n) return fail(CLAK_E_ARG, "set_eigen: ldz=%lld < n", (long long)ldz);
  p->state = ST_WS;
  const int64_t n = p->n, np = p->n_pad;
  Workspace& W = p->ws;
  HIP_TRY(hipMemsetAsync(W.Zt, 0, sizeof(double) * np * np, p->stream));
  HIP_TRY(hipMemsetAsync(W.w, 0, sizeof(double) * np, p->stream));
  HIP_TRY(hipMemsetAsync(W.dstat, 0, sizeof(int) * DS_COUNT, p->stream));
  HIP_TRY(hipMemcpy2DAsync(W.Zt, sizeof(double) * np, d_Z, sizeof(double) * ldz, sizeof(double) * n, n,
                           hipMemcpyDeviceToDevice, p->stream));
  HIP_TRY(hipMemcpyAsync(W.w, d_w, sizeof(double) * n, hipMemcpyDeviceToDevice, p->stream));
  return finish_eigen(p);
}

clak_status clak_set_covariates(clak_plan_t h, const double* d_XL, int64_t ld) {
  Plan* p = as_plan(h);
  clak_status s = need_state(p, ST_EIG, "set_covariates");
  if (s) return s;
  if (!d_XL) return fail(CLAK_E_ARG, "set_covariates: null X_L");
  if (!device_accessible(p, d_XL)) return fail(CLAK_E_ARG, "set_covariates: X_L is not device-accessible memory");
  if (ld < p->n) return fail(CLAK_E_ARG, "set_covariates: ld=%lld < n", (long long)ld);
  p->state = ST_EIG;
  Workspace& W = p->ws;
  HIP_TRY(hipMemsetAsync(W.dstat, 0, sizeof(int) * DS_COUNT, p->stream));
  HIP_TRY(launch_covariates(*p, d_XL, ld));
  if (p->flags & CLAK_CHOL) {
    // the rotation depends on h2: X_L is kept and rotated in set_traits
    HIP_TRY(hipMemsetAsync(W.XL, 0, sizeof(double) * p->n_pad * p->pL, p->stream));
    HIP_TRY(hipMemcpy2DAsync(W.XL, sizeof(double) * p->n_pad, d_XL, sizeof(double) * ld, sizeof(double) * p->n,
                             p->pL, hipMemcpyDeviceToDevice, p->stream));
  } else {
    HIP_TRY(launch_rotate_real(*p, d_XL, ld, p->pL, W.XLt, p->n_pad));
    if (p->prec == CLAK_PREC_MIXED)
      HIP_TRY(launch_qt_digits(*p));  // the centring rotation by the digit-encoded Z^T
    else
      HIP_TRY(launch_rotate_real(*p, W.QL, p->n_pad, p->pL, W.Qt, p->n_pad));
  }
  s = sync_and_read_status(p);
  if (s) return s;
  if (p->hstat[DS_COV] == 1) return fail(CLAK_E_ARG, "set_covariates: non-finite X_L");
  if (p->hstat[DS_COV] == 2) return fail(CLAK_E_COV_SINGULAR, "set_covariates: X_L is rank deficient");
  p->state = ST_COV;
  return ok();
}

clak_status clak_set_traits(clak_plan_t h, const double* d_Y, int64_t ldy, const double* d_h2,
                            const double* d_s2) {
  Plan* p = as_plan(h);
  clak_status s = need_state(p, ST_COV, "set_traits");
  if (s) return s;
  if (!d_Y || !d_h2 || !d_s2) return fail(CLAK_E_ARG, "set_traits: null Y, h2 or s2");
  if (!device_accessible(p, d_Y) || !device_accessible(p, d_h2) || !device_accessible(p, d_s2))
    return fail(CLAK_E_ARG, "set_traits: Y, h2 or s2 is not device-accessible memory");
  if (ldy < p->n) return fail(CLAK_E_ARG, "set_traits: ldy=%lld < n", (long long)ldy);
  p->state = ST_COV;
  Workspace& W = p->ws;
  if (p->flags & CLAK_CHOL) {
    s = chol_factor(p, d_h2);
    if (s) return s;
  }
  HIP_TRY(hipMemsetAsync(W.dstat, 0, sizeof(int) * DS_COUNT, p->stream));
  HIP_TRY(launch_rotate_real(*p, d_Y, ldy, p->t, W.Yt, p->n_pad));
  // per-trait h2 and s2 travel through the parameter block (slot pL*pL+pL: s2, +1: h2)
  const int64_t ts = trait_stride(p->pL);
  HIP_TRY(hipMemcpy2DAsync(W.tpar + p->pL * p->pL + p->pL, sizeof(double) * ts, d_s2, sizeof(double),
                           sizeof(double), p->t, hipMemcpyDeviceToDevice, p->stream));
  HIP_TRY(hipMemcpy2DAsync(W.tpar + p->pL * p->pL + p->pL + 1, sizeof(double) * ts, d_h2, sizeof(double),
                           sizeof(double), p->t, hipMemcpyDeviceToDevice, p->stream));
  HIP_TRY(launch_traits(*p));
  if (lin_rows(*p)) HIP_TRY(launch_uproj(*p));  // the extra rotation rows U^T = (Z W)^T and their digits
  s = sync_and_read_status(p);
  if (s) return s;
  if (p->hstat[DS_TRAIT_ARG])
    return fail(CLAK_E_ARG, "set_traits: %d trait(s) with h2 outside [0,1], s2 <= 0 or non-finite values",
                p->hstat[DS_TRAIT_ARG]);
  if (p->hstat[DS_TRAIT_SPD])
    return fail(CLAK_E_NOT_SPD, "set_traits: M_j not positive definite for %d trait(s)", p->hstat[DS_TRAIT_SPD]);
  if (p->hstat[DS_TRAIT_COV])
    return fail(CLAK_E_COV_SINGULAR, "set_traits: X_L^T M_j^-1 X_L singular for %d trait(s)",
                p->hstat[DS_TRAIT_COV]);
  p->state = ST_READY;
  return ok();
}

clak_status clak_estimate_vc(clak_plan_t h, const double* d_Y, int64_t ldy, int method, double* d_h2,
                             double* d_s2, double* d_loglik) {
  Plan* p = as_plan(h);
  clak_status s = need_state(p, ST_COV, "estimate_vc");
  if (s) return s;
  if (p->flags & CLAK_CHOL)
    return fail(CLAK_E_UNSUPPORTED, "estimate_vc: needs the eigenvalues of Phi (not a CLAK_CHOL plan)");
  if (method != CLAK_VC_ML && method != CLAK_VC_REML) return fail(CLAK_E_ARG, "estimate_vc: unknown method %d", method);
  if (!d_Y || !d_h2 || !d_s2) return fail(CLAK_E_ARG, "estimate_vc: null Y, h2 or s2");
  if (!device_accessible(p, d_Y) || !device_accessible(p, d_h2) || !device_accessible(p, d_s2) ||
      (d_loglik && !device_accessible(p, d_loglik)))
    return fail(CLAK_E_ARG, "estimate_vc: an argument is not device-accessible memory");
  if (!aligned(d_h2, 8) || !aligned(d_s2, 8) || (d_loglik && !aligned(d_loglik, 8)))
    return fail(CLAK_E_ARG, "estimate_vc: misaligned output");
  if (ldy < p->n) return fail(CLAK_E_ARG, "estimate_vc: ldy=%lld < n", (long long)ldy);
  Workspace& W = p->ws;
  HIP_TRY(hipMemsetAsync(W.dstat, 0, sizeof(int) * DS_COUNT, p->stream));
  HIP_TRY(launch_rotate_real(*p, d_Y, ldy, p->t, W.Yt, p->n_pad));
  HIP_TRY(launch_vc(*p, method, d_h2, d_s2, d_loglik));
  s = sync_and_read_status(p);
  if (s) return s;
  if (p->hstat[DS_TRAIT_ARG])
    return fail(CLAK_E_ARG, "estimate_vc: %d trait(s) with non-finite values", p->hstat[DS_TRAIT_ARG]);
  if (p->hstat[DS_TRAIT_COV])
    return fail(CLAK_E_COV_SINGULAR, "estimate_vc: X_L^T H^-1 X_L not positive definite for %d trait(s)",
                p->hstat[DS_TRAIT_COV]);
  return ok();
}

}  // extern "C"

namespace clak {

clak_status validate_block(const Plan* p, int64_t m_blk, const void* d_G, int g_dtype, int64_t ldg, const void* d_b,
                           const void* d_se, int out_dtype, int64_t ldo, const void* d_flags, const void* d_pval) {
  if (m_blk < 1 || m_blk > p->max_block)
    return fail(CLAK_E_ARG, "run_block: m_blk=%lld outside [1, max_block=%lld]", (long long)m_blk,
                (long long)p->max_block);
  if (!d_G || !d_b || !d_se) return fail(CLAK_E_ARG, "run_block: null G, b or se");
  if (g_dtype != CLAK_G_U8 && g_dtype != CLAK_G_F16 && g_dtype != CLAK_G_P2)
    return fail(CLAK_E_ARG, "run_block: unknown g_dtype %d", g_dtype);
  if (out_dtype != CLAK_OUT_F32 && out_dtype != CLAK_OUT_F64)
    return fail(CLAK_E_ARG, "run_block: unknown out_dtype %d", out_dtype);
  if (ldg < genotype_row_units(g_dtype, p->n))
    return fail(CLAK_E_ARG, "run_block: ldg=%lld < %lld (one genotype row)", (long long)ldg,
                (long long)genotype_row_units(g_dtype, p->n));
  if (ldo < m_blk) return fail(CLAK_E_ARG, "run_block: ldo=%lld < m_blk", (long long)ldo);
  const size_t esz = out_dtype == CLAK_OUT_F32 ? 4 : 8;
  if (!aligned(d_b, esz) || !aligned(d_se, esz) || !aligned(d_pval, esz))
    return fail(CLAK_E_ARG, "run_block: misaligned output");
  if (g_dtype == CLAK_G_F16 && !aligned(d_G, 2)) return fail(CLAK_E_ARG, "run_block: misaligned F16 genotypes");
  if (!device_accessible(p, d_G)) return fail(CLAK_E_ARG, "run_block: G is not device-accessible memory");
  if (!device_accessible(p, d_b) || !device_accessible(p, d_se) || (d_flags && !device_accessible(p, d_flags)) ||
      (d_pval && !device_accessible(p, d_pval)))
    return fail(CLAK_E_ARG, "run_block: an output is not device-accessible memory");
  return CLAK_OK;
}

// Enqueues the per-block stages on the given streams (ingest on s_in, the
// rest on s_main; the caller orders the two) using workspace slot `slot`.
clak_status enqueue_block(Plan* p, int slot, hipStream_t s_in, hipStream_t s_main, hipEvent_t ingested,
                          int64_t m_blk, const void* d_G, int g_dtype, int64_t ldg, const CellOut& out) {
  select_slot(*p, slot);
  const hipStream_t saved = p->stream;
  auto staged = [&](int stage, auto&& launch) -> hipError_t {
    if (!p->profiling) return launch();
    hipEvent_t a = take_event(p), b = take_event(p);
    if (!a || !b) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(a, p->stream);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess) e = hipEventRecord(b, p->stream);
    p->pending.push_back({stage, a, b});
    return e;
  };
  hipError_t e;
  p->stream = s_in;
  // CLAK_STAGE_GENOTYPES: the copy engine moves the block into the slot's staging buffer, the ingest reads it there
  const void* G = d_G;
  int64_t ld = ldg;
  const int64_t esz = g_dtype == CLAK_G_F16 ? 2 : 1;  // bytes per unit of ldg
  const bool stage_copy = p->ws.slot[slot].Gh != nullptr;
  const int64_t row_bytes = genotype_row_units(g_dtype, p->n) * esz;
  // rows that fit the staging pitch keep the caller's pitch and move as one
  // contiguous copy of the block's exact extent; wider rows are re-pitched
  const bool stage_flat = stage_copy && ldg * esz <= host_pitch(p->n);
  if (stage_copy) {
    G = p->ws.slot[slot].Gh;
    ld = stage_flat ? ldg : host_pitch(p->n) / esz;
  }
  e = staged(CLAK_STAGE_INGEST, [&] {
    if (stage_flat) {
      hipError_t c = hipMemcpyAsync(p->ws.slot[slot].Gh, d_G, (size_t)((m_blk - 1) * ldg * esz + row_bytes),
                                    hipMemcpyDefault, p->stream);
      if (c != hipSuccess) return c;
    } else if (stage_copy) {
      hipError_t c = hipMemcpy2DAsync(p->ws.slot[slot].Gh, host_pitch(p->n), d_G, ldg * esz, row_bytes, m_blk,
                                      hipMemcpyDefault, p->stream);
      if (c != hipSuccess) return c;
    }
    return launch_ingest(*p, m_blk, G, g_dtype, ld);
  });
  if (e == hipSuccess && ingested) e = hipEventRecord(ingested, s_in);
  if (e == hipSuccess && ingested && s_main != s_in) e = hipStreamWaitEvent(s_main, ingested, 0);
  p->stream = s_main;
  if (e == hipSuccess) e = staged(CLAK_STAGE_ROTATE, [&] { return launch_rotate_snps(*p, m_blk); });
  if (e == hipSuccess && p->prec == CLAK_PREC_MIXED && !p->fused_t1)
    e = staged(CLAK_STAGE_ENCODE, [&] { return launch_encode(*p, m_blk); });
  if (e == hipSuccess)
    e = staged(CLAK_STAGE_GRID, [&] { return launch_grid(*p, m_blk, out); });
  p->stream = saved;
  select_slot(*p, 0);
  if (e != hipSuccess) return fail(CLAK_E_DEVICE, "run_block: launch failed: %s", hipGetErrorString(e));
  return CLAK_OK;
}

}  // namespace clak

extern "C" {

clak_status clak_run_block(clak_plan_t h, int64_t m_blk, const void* d_G, int g_dtype, int64_t ldg, void* d_b,
                           void* d_se, int out_dtype, int64_t ldo, uint8_t* d_flags, void* d_pval) {
  Plan* p = as_plan(h);
  clak_status s = need_state(p, ST_READY, "run_block");
  if (s) return s;
  s = validate_block(p, m_blk, d_G, g_dtype, ldg, d_b, d_se, out_dtype, ldo, d_flags, d_pval);
  if (s) return s;
  s = enqueue_block(p, 0, p->stream, p->stream, nullptr, m_blk, d_G, g_dtype, ldg,
                    cell_out(d_b, d_se, d_pval, d_flags, ldo, out_dtype));
  if (s) return s;
  return ok();
}

clak_status clak_plan_set_tuning(clak_plan_t h, int rot_cfg, int rot_rg, int grid_tt, int grid_xt) {
  Plan* p = as_plan(h);
  if (!p) return fail(CLAK_E_ARG, "plan_set_tuning: null plan");
  auto pow2_le8 = [](int v) { return v == 0 || v == 1 || v == 2 || v == 4 || v == 8; };
  if (rot_cfg < 0 || rot_cfg >= ROT_CONFIGS || !pow2_le8(rot_rg) || !pow2_le8(grid_xt) ||
      !(grid_tt == 0 || grid_tt == 32 || grid_tt == 64))
    return fail(CLAK_E_ARG, "plan_set_tuning: rot_cfg=%d rot_rg=%d grid_tt=%d grid_xt=%d outside the tunable set",
                rot_cfg, rot_rg, grid_tt, grid_xt);
  p->rot_cfg = rot_cfg;
  p->rot_rg = rot_rg;
  p->grid_tt = grid_tt;
  p->grid_xt = grid_xt;
  return ok();
}

clak_status clak_plan_get_shape(clak_plan_t h, int64_t* n, int64_t* p_L, int64_t* t, int64_t* max_block,
                                int* precision, uint32_t* flags) {
  Plan* p = as_plan(h);
  if (!p) return fail(CLAK_E_ARG, "plan_get_shape: null plan");
  if (n) *n = p->n;
  if (p_L) *p_L = p->pL;
  if (t) *t = p->t;
  if (max_block) *max_block = p->max_block;
  if (precision) *precision = p->prec;
  if (flags) *flags = p->flags;
  return ok();
}

clak_status clak_plan_get_tuning(clak_plan_t h, int* rot_cfg, int* rot_rg, int* grid_tt, int* grid_xt) {
  Plan* p = as_plan(h);
  if (!p) return fail(CLAK_E_ARG, "plan_get_tuning: null plan");
  if (rot_cfg) *rot_cfg = p->rot_cfg;
  if (rot_rg) *rot_rg = p->rot_rg;
  if (grid_tt) *grid_tt = p->grid_tt;
  if (grid_xt) *grid_xt = p->grid_xt;
  return ok();
}

clak_status clak_autotune(clak_plan_t h, int64_t m_blk, const void* d_G, int g_dtype, int64_t ldg, void* d_b,
                          void* d_se, int out_dtype, int64_t ldo, uint8_t* d_flags, const char* cache_path) {
  Plan* p = as_plan(h);
  clak_status s = need_state(p, ST_READY, "autotune");
  if (s) return s;
  clak_block B{m_blk, d_G, ldg, d_b, d_se, ldo, d_flags, nullptr};
  s = autotune_blocks(p, 1, &B, g_dtype, out_dtype, cache_path, "autotune");
  return s ? s : ok();
}

clak_status clak_plan_set_profiling(clak_plan_t h, int mode) {
  Plan* p = as_plan(h);
  if (!p) return fail(CLAK_E_ARG, "plan_set_profiling: null plan");
  if (mode != CLAK_PROFILE_OFF && mode != CLAK_PROFILE_SERIAL && mode != CLAK_PROFILE_PIPELINED)
    return fail(CLAK_E_ARG, "plan_set_profiling: unknown mode %d", mode);
  clak_status s = drain_profile(p);
  if (s) return s;
  for (int i = 0; i < CLAK_STAGE_COUNT; ++i) {
    p->stage_ms[i] = 0.0;
    p->stage_n[i] = 0;
    p->stage_iv[i].clear();
  }
  if (mode != CLAK_PROFILE_OFF) {
    if (!p->prof_ref && hipEventCreate(&p->prof_ref) != hipSuccess)
      return fail(CLAK_E_DEVICE, "plan_set_profiling: event creation failed");
    HIP_TRY(hipEventRecord(p->prof_ref, p->stream));
  }
  p->profiling = mode;
  return ok();
}

clak_status clak_plan_get_profile(clak_plan_t h, double* ms, int64_t* launches) {
  Plan* p = as_plan(h);
  if (!p) return fail(CLAK_E_ARG, "plan_get_profile: null plan");
  clak_status s = drain_profile(p);
  if (s) return s;
  for (int i = 0; i < CLAK_STAGE_COUNT; ++i) {
    if (ms) ms[i] = p->stage_ms[i];
    if (launches) launches[i] = p->stage_n[i];
  }
  return ok();
}

clak_status clak_plan_get_busy(clak_plan_t h, double* busy) {
  Plan* p = as_plan(h);
  if (!p || !busy) return fail(CLAK_E_ARG, "plan_get_busy: null argument");
  clak_status s = drain_profile(p);
  if (s) return s;
  for (int i = 0; i < CLAK_STAGE_COUNT; ++i) busy[i] = busy_ms(p->stage_iv[i]);
  return ok();
}

clak_status clak_plan_destroy(clak_plan_t h) {
  Plan* p = as_plan(h);
  if (!p) return fail(CLAK_E_ARG, "plan_destroy: null plan");
  if (!p->pending.empty()) (void)hipStreamSynchronize(p->stream);
  for (auto& t : p->pending) {
    p->event_pool.push_back(t.a);
    p->event_pool.push_back(t.b);
  }
  for (hipEvent_t e : p->event_pool) (void)hipEventDestroy(e);
  if (p->prof_ref) (void)hipEventDestroy(p->prof_ref);
  if (p->rocblas) rocblas_destroy_handle((rocblas_handle)p->rocblas);
  if (p->hstat) (void)hipHostFree(p->hstat);
  delete p;
  return ok();
}

}  // extern "C"
