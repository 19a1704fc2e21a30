// Internal declarations of libclak: plan state, workspace carve-up and the
// kernel launchers shared by the ABI layer and the HIP translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <functional>
#include <utility>
#include <vector>

#include "../../include/clak.h"

namespace clak {

// Padding of the individual / eigen-index axis (the contraction axis K of
// every GEMM on the path) and of the SNP axis of a block.
constexpr int64_t KPAD = 128;
constexpr int64_t SNP_PAD = 256;  // multiple of every SNP tile width
constexpr int64_t TRAIT_PAD = 128;
constexpr int ROT_CONFIGS = 11;  // tile configurations of the mixed rotation (tunable)
constexpr int MAX_PL = 16;
constexpr int ING_MAX_SPLITS = 8;  // individual windows of the ingest are split over at most this many work-groups
constexpr int ING_WINDOWS_PER_WG = 4;  // and each work-group takes about this many windows
// int8 digit encoding: a value v with |v| <= s is stored as
// q = rint(v / s * QMAX), |q| <= QMAX < 2^31, split into four base-256 digits.
constexpr double QMAX = 2130706432.0;  // 127 * 2^24
constexpr int64_t MIXED_MAX_N = 32000; // int32 accumulators of the grid sums stay exact below this

__host__ __device__ inline int64_t roundup(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Per-SNP statistics written by the ingest kernel (doubles, stride snp_stride):
//   [0, pL)      v = Q_L^T g            (centring coefficients in the Q_L basis)
//   [pL, 2pL)    gamma = R^{-1} v       (centring coefficients in the X_L basis)
//   2pL          ||g - Q_L v||          (digit scale of the rotated SNP)
//   2pL + 1      cell flag of the SNP (0 ok, 1 degenerate, 2 bad genotype)
//   2pL + 2      max_k |x~_k| of the rotated, centred SNP (mixed path; written
//                by an atomic max on its bit pattern, so it is order-independent)
//   [2pL+3, 3pL+4)  single-trait mixed path: the linear cell sums c' and r'
//                (written by the rotation's U^T rows, see zlin)
__host__ __device__ inline int64_t snp_stride(int64_t pL) { return 3 * pL + 4; }
// Per-trait parameters written by the trait kernel (doubles, stride trait_stride):
//   [0, pL*pL)   L^{-1} (row-major, lower), L L^T = S_TL
//   [pL*pL, pL*pL+pL)  u = S_TL^{-1} b_T
//   pL*pL+pL     s2
__host__ __device__ inline int64_t trait_stride(int64_t pL) { return pL * pL + pL + 2; }

enum DevStatus : int {
  DS_EIG_INFO = 0,     // rocSOLVER info
  DS_COV = 1,          // 0 ok, 1 non-finite X_L, 2 rank deficient
  DS_TRAIT_ARG = 2,    // count of traits with bad h2 / s2 / non-finite y
  DS_TRAIT_SPD = 3,    // count of traits with h2 w_k + 1 - h2 <= 0
  DS_TRAIT_COV = 4,    // count of traits whose S_TL is not positive definite
  DS_EIGVAL = 5,       // non-finite eigenvalue / eigenvector input
  DS_COUNT = 64
};

// Where the per-cell results of one block go: cell (i, j) at element
// i + j * ldo (b holds p values per cell under CLAK_OUT_FULL).
struct CellOut {
  void* b = nullptr;
  void* se = nullptr;
  void* pval = nullptr;      // two-sided p-value of the Wald statistic (nullable)
  uint8_t* flags = nullptr;  // nullable
  int64_t ldo = 0;
  int f64 = 0;  // element type of b, se and pval: double if set, else float
};

// Buffers of one SNP block in flight.  The workspace holds NSLOTS such slots
// so that a pipeline can ingest blocks b+1 and b+2 while block b is rotated.
struct Slot {
  int8_t* Gp = nullptr;
  double* sstat = nullptr;
  double* ipart = nullptr;
  double* part = nullptr;
  double* X64 = nullptr;
  int8_t* Xd = nullptr;
  uint8_t* Gh = nullptr;  // CLAK_STAGE_GENOTYPES: copy of the caller's genotype block, rows of host_pitch bytes
};
// Workspace slots of the block pipeline: the ingest of block b reuses slot
// b % NSLOTS once block b - NSLOTS has finished.
constexpr int NSLOTS = 3;

// Row pitch (bytes) of the host-block staging buffer: n elements of up to 2 bytes, 16-byte aligned rows.
inline int64_t host_pitch(int64_t n) { return (2 * n + 15) / 16 * 16; }
// Units of ldg one genotype row of n individuals takes: n elements (u8, f16)
// or (n + 3) / 4 bytes (2-bit codes).
inline int64_t genotype_row_units(int g_dtype, int64_t n) { return g_dtype == CLAK_G_P2 ? (n + 3) / 4 : n; }

struct Workspace {
  Slot slot[NSLOTS];
  // common
  double* Zt = nullptr;     // zrows x n_pad: row k (stride n_pad) = eigenvector k, zero padded; rows zlin +
                            // q <= pL of a single-trait mixed plan hold column q of U = Z W
  double* w = nullptr;      // n_pad eigenvalues (zero beyond n)
  double* evE = nullptr;    // n_pad, eigensolver scratch
  int* dstat = nullptr;     // DS_COUNT device status words
  double* QL = nullptr;     // n_pad x pL, column-major: orthonormal basis of X_L, zero padded
  double* Rm = nullptr;     // pL x pL row-major upper triangle R, X_L = Q_L R
  double* Rinv = nullptr;   // pL x pL row-major R^{-1}
  double* XLt = nullptr;    // n_pad x pL column-major: Z^T X_L
  double* Qt = nullptr;     // n_pad x pL column-major: Z^T Q_L
  double* Yt = nullptr;     // n_pad x t  column-major: Z^T Y
  double* Phi = nullptr;    // CLAK_CHOL: n_pad x n_pad copy of Phi (lower triangle used)
  double* XL = nullptr;     // CLAK_CHOL: n_pad x pL copy of X_L (rotated at set_traits)
  double* tpar = nullptr;   // t_pad x trait_stride
  double* Cq = nullptr;     // single-trait mixed: pL x (pL+1) row-major, C = Q_L^T U (centring of the extra rows)
  // per block (the slot selected for the block being launched)
  int8_t* Gp = nullptr;     // mb_pad SNP rows x n_pad individuals, K-tiled (kt32), zero padded
  double* sstat = nullptr;  // mb_pad x snp_stride
  double* ipart = nullptr;  // ingest partials: [ING_MAX_SPLITS][pL+2][mb_pad]
  // rotated, centred SNPs in FP64 (both paths)
  double* X64 = nullptr;    // mb_pad x n_pad: row = SNP, eigen index contiguous
  // FP64 per-trait operand (FP64 path; mixed path when the fused t = 1 kernel runs)
  double* V64 = nullptr;    // t_pad*(pL+1) x n_pad: per-trait operand columns (row = column)
  double* D64 = nullptr;    // t_pad x n_pad: d_j
  double* part = nullptr;   // fused t = 1 kernel: [n_pad/64][pL+2][mb_pad] partial sums
  // mixed path
  int8_t* Zd = nullptr;     // 4 planes x zrows rows (Z^T) x n_pad, K-tiled (kt32)
  double* zs = nullptr;     // zrows: per-row digit scale (value = zs * sum digits 256^(3-p))
  int8_t* Xd = nullptr;     // 8 planes x mb_pad rows (SNPs) x n_pad, K-tiled (kt32): digits of x, then x^2
  int8_t* Vd = nullptr;     // 4 planes x t_pad*(pL+1) rows (vrow order) x n_pad, K-tiled (kt32)
  int8_t* Dd = nullptr;     // 4 planes x t_pad rows x n_pad, K-tiled (kt32)
  double* vs = nullptr;     // t_pad*(pL+1) digit scales of the operand columns
  double* ds = nullptr;     // t_pad digit scales of d_j
};

enum PlanState { ST_CREATED = 0, ST_WS = 1, ST_EIG = 2, ST_COV = 3, ST_READY = 4 };

struct Plan {
  int64_t n = 0, pL = 0, t = 0, max_block = 0;
  int prec = CLAK_PREC_FP64;
  uint32_t flags = 0;
  int64_t n_pad = 0, mb_pad = 0, t_pad = 0;
  // Rows of the rotation operand.  A single-trait mixed plan appends the pL + 1
  // rows of U^T = (Z W)^T (W: the trait operand columns) at row zlin, so that
  // the rotation also yields the linear cell sums c' = W_c^T x~ and
  // r' = W_r^T x~ of each SNP (U^T (g - Q_L v) = W^T x~): in the zero padding
  // rows n .. when n + pL + 1 <= n_pad (zrows = n_pad), else in one more tile
  // of ZEXT rows (zlin = n_pad, zrows = n_pad + ZEXT).  Other plans: zlin =
  // zrows = n_pad.
  int64_t zrows = 0, zlin = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  void* rocblas = nullptr;  // rocblas_handle
  void* ws_base = nullptr;
  size_t ws_bytes = 0;
  Workspace ws;
  int state = ST_CREATED;
  bool fused_t1 = false;    // single trait: rotate-and-reduce kernel, no stored X~
  // launch parameters chosen by clak_autotune or clak_plan_set_tuning (0: the
  // built-in choice): rotation tile configuration and XCD row groups, traits
  // per work-group and XCD trait groups of the grid contraction
  int rot_cfg = 0, rot_rg = 0, grid_tt = 0, grid_xt = 0;
  // stage profiler (CLAK_PROFILE_*): pending (stage, start, end) event
  // triples, per-stage totals, and every launch's interval relative to the
  // reference event recorded when profiling was enabled
  int profiling = CLAK_PROFILE_OFF;
  struct Timed {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<Timed> pending;
  std::vector<hipEvent_t> event_pool;
  hipEvent_t prof_ref = nullptr;
  double stage_ms[CLAK_STAGE_COUNT] = {0, 0, 0, 0};
  int64_t stage_n[CLAK_STAGE_COUNT] = {0, 0, 0, 0};
  std::vector<std::pair<double, double>> stage_iv[CLAK_STAGE_COUNT];
  int* hstat = nullptr;     // pinned host mirror of dstat
};

void init_shape(Plan& p, int64_t n, int64_t p_L, int64_t t, int64_t max_block, int precision, uint32_t flags);
size_t workspace_bytes(const Plan& p, Workspace* carve, char* base);
size_t slot_bytes(const Plan& p, Slot* carve, char* base);

// Number of work-groups the ingest splits the individuals of one SNP group
// over: one per ING_WINDOWS_PER_WG 128-individual windows, at most
// ING_MAX_SPLITS (fewer, longer work-groups hold fewer CUs that the rotation
// of the previous block could use).  It depends on n only, so every SNP's
// statistics are summed in the same order whatever the block split.
inline int ingest_splits(const Plan& p) {
  const int64_t windows = p.n_pad / 128, s = (windows + ING_WINDOWS_PER_WG - 1) / ING_WINDOWS_PER_WG;
  return (int)(s < ING_MAX_SPLITS ? s : ING_MAX_SPLITS);
}

constexpr int64_t ZEXT = 64;  // rows of the extra rotation tile (one 64-row tile)
// Single-trait mixed plans form the linear cell sums in the rotation's U^T
// rows; its other rows give only the quadratic sum a.
inline bool lin_rows(const Plan& p) { return p.fused_t1 && p.prec == CLAK_PREC_MIXED; }

// The built-in rotation tiles of the mixed path (rot_cfg 0): 64 x 256 SNPs
// (configuration 6) for single-trait plans over blocks of at least
// ROT_WIDE_MIN SNPs, else 64 x 128.  Measured at n = 1000 with blocks of
// 10^4 SNPs, a 64 x 256 launch alone is slower (55 against 50 us), but the
// block pipeline, where consecutive rotations overlap each other and the
// ingest, runs faster with it (CLAK-Eig 5.07 against 5.66 ms per 10^6 SNPs,
// CLAK-Chol 4.01 against 5.06 ms); at 2000 SNPs in one block the 64 x 128
// tiles are faster.
constexpr int64_t ROT_WIDE_MIN = 8192;
inline bool rot_wide_builtin(const Plan& p) { return lin_rows(p) && p.mb_pad >= ROT_WIDE_MIN; }
// Built-in XCD row groups of the rotation: 1 for CLAK-Chol's triangular
// operand with the wide tiles (4.01 against 4.26 ms per 10^6 SNPs), else 2.
inline int rot_rg_builtin(const Plan& p) { return (rot_wide_builtin(p) && (p.flags & CLAK_CHOL)) ? 1 : 2; }

// Rotation configuration 10, the Z-resident kernel (k_rotz.hip): mixed
// precision, n_pad <= 1024, plain operand, p_L <= 4.  Where it does not apply
// the configuration runs the built-in tiles.  Its single-trait partials are
// per 32-row slice, added in pairs by the finish.
bool rot_zs_applicable(const Plan& p);
inline bool rot_zs_active(const Plan& p) { return p.rot_cfg == 10 && rot_zs_applicable(p); }

// Points the per-block buffers of the workspace at slot k.
inline void select_slot(Plan& p, int k) {
  const Slot& s = p.ws.slot[k];
  p.ws.Gp = s.Gp;
  p.ws.sstat = s.sstat;
  p.ws.ipart = s.ipart;
  p.ws.part = s.part;
  p.ws.X64 = s.X64;
  p.ws.Xd = s.Xd;
}

// ---- ABI helpers (abi.cpp) ----
clak_status fail(clak_status s, const char* fmt, ...);
hipEvent_t take_event(Plan* p);
clak_status ok();
clak_status need_state(const Plan* p, int min_state, const char* what);
bool device_accessible(const Plan* p, const void* ptr);
CellOut cell_out(void* b, void* se, void* pval, uint8_t* flags, int64_t ldo, int out_dtype);
clak_status validate_block(const Plan* p, int64_t m_blk, const void* d_G, int g_dtype, int64_t ldg, const void* d_b,
                           const void* d_se, int out_dtype, int64_t ldo, const void* d_flags, const void* d_pval);
clak_status enqueue_block(Plan* p, int slot, hipStream_t s_in, hipStream_t s_main, hipEvent_t ingested,
                          int64_t m_blk, const void* d_G, int g_dtype, int64_t ldg, const CellOut& out);
clak_status autotune_blocks(Plan* p, int64_t n_blocks, const clak_block* blocks, int g_dtype, int out_dtype,
                            const char* cache_path, const char* what);
clak_status stream_blocks(Plan* p, int64_t n_blocks, int g_dtype, int out_dtype,
                          const std::function<clak_status(int64_t, clak_block*)>& get,
                          const std::function<clak_status(int64_t, hipStream_t)>& after, const char* what);

constexpr int MAX_BATCH = 16;  // plans in one batched launch

// One plan's block in a batched launch (several plans' blocks in one grid):
// the plan, the workspace slot the block uses, its size, input and outputs.
struct BatchItem {
  Plan* p = nullptr;
  int slot = 0;
  int64_t m_blk = 0;
  const void* G = nullptr;
  int64_t ldg = 0;
  CellOut out;
};

// ---- batched launchers: one grid over every item, on stream s (plans that
// batch_compatible accepts: mixed precision, several traits, the same p_L <= 3
// and output form, no copy-engine staging) ----
bool batch_compatible(const Plan& a, const Plan& b);
hipError_t launch_ingest_batch(const BatchItem* items, int count, int g_dtype, hipStream_t s);
hipError_t launch_rotate_batch(const BatchItem* items, int count, hipStream_t s);
hipError_t launch_encode_batch(const BatchItem* items, int count, hipStream_t s);
hipError_t launch_grid_batch(const BatchItem* items, int count, hipStream_t s);

// ---- launchers (implemented in the .hip files; all enqueue on p.stream) ----
// set-up
hipError_t launch_split_digits(const Plan& p, int64_t r0, int64_t r1);
hipError_t launch_dequant_rows(const Plan& p, int64_t r0, int64_t r1);
hipError_t launch_qt_digits(const Plan& p);
hipError_t launch_covariates(const Plan& p, const double* d_XL, int64_t ld);
hipError_t launch_rotate_real(const Plan& p, const double* B, int64_t ldb, int64_t ncols, double* out,
                              int64_t ldo);
hipError_t launch_traits(const Plan& p);
hipError_t launch_uproj(const Plan& p);
hipError_t launch_vc(const Plan& p, int method, double* h2, double* s2, double* ll);
hipError_t launch_check_eigen(const Plan& p);
hipError_t launch_chol_check(const Plan& p);
hipError_t launch_chol_build(const Plan& p, const double* d_h2);
hipError_t launch_chol_fix(const Plan& p);
// per block
hipError_t launch_ingest(const Plan& p, int64_t m_blk, const void* d_G, int g_dtype, int64_t ldg);
hipError_t launch_rotate_snps(const Plan& p, int64_t m_blk);
hipError_t launch_rotate_zs(const Plan& p, int64_t m_blk);
hipError_t launch_encode(const Plan& p, int64_t m_blk);
hipError_t launch_fin_t1(const Plan& p, int64_t m_blk, const CellOut& out);
hipError_t launch_grid(const Plan& p, int64_t m_blk, const CellOut& out);
hipError_t launch_grid_ring(const Plan& p, int64_t m_blk, const CellOut& out);

}  // namespace clak
