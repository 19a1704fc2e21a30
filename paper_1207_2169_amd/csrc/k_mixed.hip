// int8 digit-plane MFMA kernels of the mixed-precision path.
//
// Every real operand is carried as four int8 digit planes with one FP64 scale
// (per eigenvector row of Z^T, per SNP, per operand column): a value v with
// |v| <= s is q = rint(v / s * QMAX) = d0 256^3 + d1 256^2 + d2 256 + d3.
// Genotypes 0/1/2 are exact int8.  v_mfma_i32_16x16x64_i8 accumulates digit
// products exactly in int32, so the only rounding of the contractions is the
// encoding of their operands (and, in the grid, the digit products of weight
// 256^-4 and below, which are dropped).
#include "common.hpp"
#include "schur.hpp"

#include <type_traits>

namespace clak {

// v_mfma_i32_16x16x64_i8 lane layout (gfx950): lane l supplies 16 bytes of
// row l%16 of A and of column l%16 of B, both covering the same 16 values of
// the 64-deep contraction (chunk l/16); result register r holds C[4(l/16)+r][l%16].
__device__ __forceinline__ v4i mfma_i8(v4i a, v4i b, v4i c) {
  return __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, c, 0, 0, 0);
}

constexpr int LROW = 80;  // LDS row pitch in bytes for 64-byte K slices (bank-conflict-free 16-byte reads)

// ------------------------------------------------------------------ rotation
//
// The SNP rotation of multi-trait CLAK-Eig (section 3) on one SNP block, X~ = Z^T G.
// A work-group of WR x WC waves takes a BM = 32 WR (eigen rows) x BN = 32 CT
// WC (SNPs) tile; each wave owns 32 rows x CT 32-column MFMA tiles and all four
// digit planes of Z^T for them (v_mfma_i32_32x32x32_i8), so one genotype
// fragment feeds four MFMAs.  The K loop runs over 64-deep slices with LDS
// double buffering (one barrier per slice; the next slice's global loads are
// in flight during the current slice's MFMAs), or (DL) a ring of three or
// four slots filled by direct global-to-LDS loads (the next two or three
// slices in flight).  Work-groups are dispatched
// round-robin over the 8 XCDs; the tiles are laid out as an rg x (8 / rg)
// grid of (row group, SNP group) so that XCD x owns 1 / rg of the Z^T rows
// (which stay in its L2) for rg / 8 of the SNP tiles, walking each SNP tile
// over its row tiles before moving on (the genotype tile is then reused from
// L2).  With rg = 2, Z^T is read twice per block and the genotype panel four
// times, instead of eight times one or the other.
// Per element, the planes are recombined exactly, scaled, and the centring
// term (Z^T Q_L)[k] . v(i) is subtracted (FP64).  Then
//   EPI 0: the value is stored (SNP-major) and the SNP's max |x~_k| is raised
//          by an atomic max, for the digit encoding of the grid operand;
//   EPI 1: (single trait) the quadratic cell sum a = d^T (x~ o x~) of this
//          tile's rows is formed in FP64 and written as one partial per (row
//          tile, SNP); x~ never leaves the chip.  Rows zl .. zl + p_L of the
//          operand (zero padding rows, or one more tile) hold U^T = (Z W)^T,
//          centred by C = Q_L^T U: for them x~ is a linear cell sum (c', then
//          r') of the SNP, which goes to the SNP's statistics.
//
// Waves per SIMD the register budget is cut for: three for the one-column-tile
// configuration (64 accumulation registers), else one or two.
template <int PL, int EPI, int CT>
constexpr int rot_waves() {
  return CT == 1 ? (PL <= 4 ? 3 : 2) : ((CT > 2 || (EPI == 1 && PL > 3)) ? 1 : 2);
}

// Arguments of the rotation of one plan's block (see rot_tile).
struct RotArgs {
  int64_t np, nz, zl, mb, mbp, ntn;
  int rg, tri;
  const int8_t* Zd;
  const double* zs;
  const int8_t* Gp;
  const double* Qt;
  const double* Cq;
  double* sstat;
  double* X;
  const double* Dv;
  double* part;
};

// Work-group bid of the rotation grid of one plan's block.
template <int PL, int EPI, int CT, int WR, int WC, int DL>
__device__ __forceinline__ void rot_tile(int64_t np, int64_t nz, int64_t zl, int64_t mb, int64_t mbp, int64_t ntn,
                                         int rg, int tri, const int8_t* __restrict__ Zd,
                                         const double* __restrict__ zs, const int8_t* __restrict__ Gp,
                                         const double* __restrict__ Qt, const double* __restrict__ Cq,
                                         double* __restrict__ sstat, double* __restrict__ X,
                                         const double* __restrict__ Dv, double* __restrict__ part, int64_t bid) {
  constexpr int NT = 64 * WR * WC, BM = 32 * WR, BN = 32 * CT * WC, BK = 64;
  constexpr int A_STAGE = 4 * BM * LROW, B_STAGE = BN * LROW;
  constexpr int A_LD = 16 * BM / NT, B_LD = 4 * BN / NT;  // 16-byte loads per thread per slice
  static_assert(16 * BM % NT == 0 && 4 * BN % NT == 0, "tile / thread mismatch");
  // DL: stages of whole 1 KB MFMA fragments (32 rows x 32 bytes of K), FA of
  // Z^T (plane, row block, K half) then FB of the genotypes (column block, K
  // half), written by direct global-to-LDS loads into a ring of DL (3 or 4)
  // slots, each its own LDS array so that the compiler can tell them apart
  static_assert(DL == 0 || DL == 3 || DL == 4, "ring depth");
  constexpr int FA = 8 * WR, FB = 2 * CT * WC, FS = FA + FB;
  // slot 0 also holds the epilogue's per-wave-row partials of a (EPI 1); it is
  // sized for them should they ever exceed a slice
  constexpr int PS_BYTES = EPI == 1 ? WR * BN * 8 : 0;
  constexpr int SMEM = DL ? (FS * 1024 > PS_BYTES ? FS * 1024 : PS_BYTES) : 2 * (A_STAGE + B_STAGE);
  __shared__ __attribute__((aligned(1024))) int8_t smem[SMEM];
  __shared__ __attribute__((aligned(1024))) int8_t smem1[DL ? FS * 1024 : 16];
  __shared__ __attribute__((aligned(1024))) int8_t smem2[DL ? FS * 1024 : 16];
  __shared__ __attribute__((aligned(1024))) int8_t smem3[DL == 4 ? FS * 1024 : 16];
  // epilogue tables, fetched while the first slices load
  constexpr int NTAB = BM * PL + BM + BN * PL + (EPI == 1 ? BM : 0);
  __shared__ double tab[NTAB];
  double* Qs = tab;             // [BM][PL]   (Z^T Q_L) rows of the tile
  double* zS = Qs + BM * PL;    // [BM]       digit scales of Z^T rows
  double* vS = zS + BM;         // [BN][PL]   centring coefficients of the SNPs
  double* Vs = vS + BN * PL;    // [BM]       d of the tile's rows (EPI 1)
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wr = wid / WC, wc = wid % WC;
  const int64_t ntm = nz / BM;
  const int64_t sg = 8 / rg, gm = (ntm + rg - 1) / rg, gn = (ntn + sg - 1) / sg;
  const int64_t xcd = bid % 8, idx = bid / 8;
  // lower-triangular Z^T (CLAK-Chol): row tile tm needs the first tm + 1 K
  // tiles only; the row tiles of a row group are interleaved across the row
  // groups (equal work per XCD) and taken heaviest first
  const int64_t tm = tri ? ntm - 1 - ((idx % gm) * rg + xcd % rg) : (xcd % rg) * gm + idx % gm;
  const int64_t tn = (xcd / rg) * gn + idx / gm;
  if (tm < 0 || tm >= ntm || tn >= ntn || idx >= gm * gn) return;
  const int64_t m0 = tm * BM, n0 = tn * BN;
  const int64_t zplane = nz * np;
  const int KT = (int)((tri ? min(np, m0 + BM) : np) / BK);

  v16i acc[CT][4];
#pragma unroll
  for (int j = 0; j < CT; ++j)
#pragma unroll
    for (int p = 0; p < 4; ++p) acc[j][p] = (v16i){};

  // Staging: the 16-byte chunks of a stage go in groups of 64, one group per
  // (plane, 32-row block, half of the 64-byte slice); lane l of a group takes
  // row l % 32, chunk l / 32 of that half, the lane pattern of the fragment
  // reads, so the LDS stores are free of bank conflicts.
  // every table value of this thread is loaded first, then stored, so the
  // loads are in flight together
  auto load_tables = [&]() {
    const int64_t ss = snp_stride(PL);
    constexpr int JQ = (BM * PL + NT - 1) / NT, JZ = (BM + NT - 1) / NT, JV = (BN * PL + NT - 1) / NT;
    constexpr int JD = EPI == 1 ? (BM + NT - 1) / NT : 0;
    double tq[JQ], tz[JZ], tv[JV], td[JD > 0 ? JD : 1];
#pragma unroll
    for (int j = 0; j < JQ; ++j) {
      const int e = tid + j * NT;
      const int64_t row = m0 + e / PL;
      const int a = e % PL;
      tq[j] = 0.0;
      if (e < BM * PL)
        tq[j] = (row >= zl && row <= zl + PL) ? Cq[a * (PL + 1) + (row - zl)] : (row < np ? Qt[row + a * np] : 0.0);
    }
#pragma unroll
    for (int j = 0; j < JZ; ++j) {
      const int e = tid + j * NT;
      tz[j] = e < BM ? zs[m0 + e] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < JV; ++j) {
      const int e = tid + j * NT;
      tv[j] = e < BN * PL ? sstat[(n0 + e / PL) * ss + e % PL] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < JD; ++j) {
      const int e = tid + j * NT;
      td[j] = (e < BM && m0 + e < np) ? Dv[m0 + e] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < JQ; ++j)
      if (tid + j * NT < BM * PL) Qs[tid + j * NT] = tq[j];
#pragma unroll
    for (int j = 0; j < JZ; ++j)
      if (tid + j * NT < BM) zS[tid + j * NT] = tz[j];
#pragma unroll
    for (int j = 0; j < JV; ++j)
      if (tid + j * NT < BN * PL) vS[tid + j * NT] = tv[j];
#pragma unroll
    for (int j = 0; j < JD; ++j)
      if (tid + j * NT < BM) Vs[tid + j * NT] = td[j];
  };

  if constexpr (DL) {
    // Each wave moves FS / (WR WC) fragments per stage; lane l fetches bytes
    // [16 (l / 32), +16) of row l % 32 of its fragment, which the load writes
    // to byte 16 l of the fragment's LDS slot, the order of the MFMA operand
    // reads (conflict-free, contiguous).  The loads of the next DL - 1 K
    // slices are in flight while one is multiplied.
    constexpr int NW = WR * WC, LPW = FS / NW, LPA = FA / NW;
    static_assert(FA % NW == 0 && FB % NW == 0 && LPW < 32, "fragments per wave");
    const int w = __builtin_amdgcn_readfirstlane(wid);
    const int loff = 32 * (lane & 31) + 16 * (lane >> 5);
    // fragment q of this wave is fi = q NW + w: Z^T fragments for q < LPA
    const int8_t* za = Zd + m0 * 32 + loff;
    const int8_t* gb = Gp + n0 * 32 + loff;
    auto slot = [&](auto u) -> int8_t* {
      if constexpr (decltype(u)::value == 0) return smem;
      else if constexpr (decltype(u)::value == 1) return smem1;
      else if constexpr (decltype(u)::value == 2) return smem2;
      else return smem3;
    };
    auto issue = [&](auto u, int kt) {
      int8_t* st = slot(u);
      const int64_t s0 = 2 * (int64_t)kt;  // first 32-byte K slice of the stage
#pragma unroll
      for (int q = 0; q < LPW; ++q) {
        const int fi = q * NW + w;
        const int8_t* src;
        if (q < LPA) {
          const int h = fi & 1, r = (fi >> 1) % WR, pl = (fi >> 1) / WR;
          src = za + pl * zplane + ((s0 + h) * nz + 32 * r) * 32;
        } else {
          const int h = (fi - FA) & 1, c = (fi - FA) >> 1;
          src = gb + ((s0 + h) * mbp + 32 * c) * 32;
        }
        __builtin_amdgcn_global_load_lds(src, (lds_ptr_t)(st + fi * 1024), 16, 0, 0);
      }
    };
    // Slice kt sits in slot kt % DL.  Every step has the same shape, so the
    // outstanding loads are the same on every path into a step: wait until
    // this wave's loads of slice kt have landed (only those of the next DL - 2
    // slices remain), barrier (every wave's loads of kt are in; every wave is
    // done reading slice kt - 1), load slice kt + DL - 1 into the slot kt - 1
    // used, multiply slice kt.  Past the last slice the load repeats slice
    // KT - 1 into a slot that is not read again; it stays in bounds.
    // Within a step, the fragments of both 32-deep halves are read first (the
    // first MFMAs then wait for the LDS only once), and the next slice's
    // direct loads are spread over the MFMAs.
    auto step = [&](auto u, int kt) {
      wait_vm<(DL - 2) * LPW>();
      lds_barrier();
      const int8_t* st = slot(u) + 16 * lane;
      v4i b[2][CT], a[2][4];
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          a[ks][p] = *(const v4i*)(st + (2 * (p * WR + wr) + ks) * 1024);
          if (p < CT) b[ks][p] = *(const v4i*)(st + (FA + 2 * (CT * wc + p) + ks) * 1024);
        }
      }
      issue(std::integral_constant<int, (decltype(u)::value + DL - 1) % DL>{}, min(kt + DL - 1, KT - 1));
#pragma unroll
      for (int ks = 0; ks < 2; ++ks)
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) acc[ct][p] = mfma32_i8(a[ks][p], b[ks][ct], acc[ct][p]);
      // schedule: all LDS reads, then MFMAs with the direct loads between them
      __builtin_amdgcn_sched_group_barrier(0x100, 8 + 2 * CT, 0);
#pragma unroll
      for (int q = 0; q < LPW; ++q) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
      }
      __builtin_amdgcn_sched_group_barrier(0x008, 8 * CT - LPW, 0);
    };
    using U0 = std::integral_constant<int, 0>;
    using U1 = std::integral_constant<int, 1>;
    using U2 = std::integral_constant<int, 2>;
    using U3 = std::integral_constant<int, 3>;
    // the first slices' loads go out before the tables', whose LDS writes
    // wait for them
    issue(U0{}, 0);
    issue(U1{}, min(1, KT - 1));
    if constexpr (DL == 4) issue(U2{}, min(2, KT - 1));
    load_tables();
    int kt = 0;
    for (; kt + DL <= KT; kt += DL) {
      step(U0{}, kt);
      step(U1{}, kt + 1);
      step(U2{}, kt + 2);
      if constexpr (DL == 4) step(U3{}, kt + 3);
    }
    if (kt < KT) step(U0{}, kt);
    if (kt + 1 < KT) step(U1{}, kt + 1);
    if constexpr (DL == 4)
      if (kt + 2 < KT) step(U2{}, kt + 2);
    wait_vm<0>();  // no load is left in flight
    __syncthreads();  // the epilogue reuses the ring
  } else {
    v4i ra[A_LD], rb[B_LD];
    const int srow = lane & 31, sch = lane >> 5;
    auto gload = [&](int kt) {
      const int64_t k0 = (int64_t)kt * BK;
  #pragma unroll
      for (int q = 0; q < A_LD; ++q) {  // group (tid + NT q) / 64: half g % 2, row block (g / 2) % (BM / 32), plane
        const int g = (tid + NT * q) >> 6;
        const int kh = g & 1, rb32 = (g >> 1) % (BM / 32), pl = (g >> 1) / (BM / 32);
        ra[q] = *(const v4i*)(Zd + pl * zplane + kt32(m0 + 32 * rb32 + srow, k0 + 32 * kh, nz) + 16 * sch);
      }
  #pragma unroll
      for (int q = 0; q < B_LD; ++q) {
        const int g = (tid + NT * q) >> 6;
        const int kh = g & 1, rb32 = g >> 1;
        rb[q] = *(const v4i*)(Gp + kt32(n0 + 32 * rb32 + srow, k0 + 32 * kh, mbp) + 16 * sch);
      }
    };
    auto lstore = [&](int buf) {
      int8_t* As = smem + buf * A_STAGE;
      int8_t* Bs = smem + 2 * A_STAGE + buf * B_STAGE;
  #pragma unroll
      for (int q = 0; q < A_LD; ++q) {
        const int g = (tid + NT * q) >> 6;
        const int kh = g & 1, rb32 = (g >> 1) % (BM / 32), pl = (g >> 1) / (BM / 32);
        *(v4i*)(As + (pl * BM + 32 * rb32 + srow) * LROW + 16 * (2 * kh + sch)) = ra[q];
      }
  #pragma unroll
      for (int q = 0; q < B_LD; ++q) {
        const int g = (tid + NT * q) >> 6;
        const int kh = g & 1, rb32 = g >> 1;
        *(v4i*)(Bs + (32 * rb32 + srow) * LROW + 16 * (2 * kh + sch)) = rb[q];
      }
    };

    gload(0);
    load_tables();
    lstore(0);
    __syncthreads();
    if (KT > 1) gload(1);
    for (int kt = 0; kt < KT; ++kt) {
      const int buf = kt & 1;
      const int8_t* As = smem + buf * A_STAGE;
      const int8_t* Bs = smem + 2 * A_STAGE + buf * B_STAGE;
  #pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        v4i b[CT], a[4];
  #pragma unroll
        for (int ct = 0; ct < CT; ++ct)
          b[ct] = *(const v4i*)(Bs + (32 * (CT * wc + ct) + (lane & 31)) * LROW + 16 * (lane >> 5) + 32 * ks);
  #pragma unroll
        for (int p = 0; p < 4; ++p)
          a[p] = *(const v4i*)(As + (p * BM + 32 * wr + (lane & 31)) * LROW + 16 * (lane >> 5) + 32 * ks);
  #pragma unroll
        for (int p = 0; p < 4; ++p)
  #pragma unroll
          for (int ct = 0; ct < CT; ++ct) acc[ct][p] = mfma32_i8(a[p], b[ct], acc[ct][p]);
      }
      if (kt + 1 < KT) {
        lstore(buf ^ 1);
        if (kt + 2 < KT) gload(kt + 2);
      }
      __syncthreads();
    }

  }

  // pair the four digit-plane sums exactly in int32 (|sum| < 2^23 for
  // n_pad <= 32768), halving the live accumulator registers
  int hi[CT][16], lo[CT][16];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      hi[ct][e] = acc[ct][0][e] * 256 + acc[ct][1][e];
      lo[ct][e] = acc[ct][2][e] * 256 + acc[ct][3][e];
    }

  // per-wave-row partial sums (EPI 1) reuse the staging buffers, free after the last barrier
  double* Ps = (double*)smem;  // [WR][BN]
  const bool ext = m0 >= np;   // the extra row tile holding U^T (EPI 1): no partial
  static_assert(PS_BYTES <= SMEM, "LDS reuse");
  // With two column tiles, the second tile's plane sums wait in the free ring
  // slots 1 and 2 while the first tile is finished (direct-load rotation,
  // single trait): 32 registers fewer across the epilogue, which otherwise
  // spills.  Each thread reads back only its own values.
  constexpr bool STASH = DL && EPI == 1 && CT == 2;
  static_assert(!STASH || 16 * NT * 4 <= FS * 1024, "stash size");
  if constexpr (STASH) {
    int* sh = (int*)smem1;
    int* sl = (int*)smem2;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      sh[e * NT + tid] = hi[1][e];
      sl[e * NT + tid] = lo[1][e];
    }
  }
  const int64_t ss = snp_stride(PL);

  // one column tile at a time (the scheduler is kept from overlapping the
  // tiles' table reads, which would not fit the registers).  Only the row tile
  // holding the U^T rows (EPI 1) needs the per-row test between a stored row
  // and a summed one; every other tile takes the code without it (the same
  // arithmetic, no divergent branch per element)
  const bool urow_tile = EPI == 1 && zl <= m0 + BM - 1 && zl + PL >= m0;
  auto columns = [&](auto with_urows) {
  constexpr bool UR = decltype(with_urows)::value;
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    __builtin_amdgcn_sched_barrier(0);
    const int cl = 32 * (CT * wc + ct) + (lane & 31);
    const int64_t col = n0 + cl;
    int hc[16], lc[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      if (STASH && ct == 1) {
        hc[e] = ((const int*)smem1)[e * NT + tid];
        lc[e] = ((const int*)smem2)[e * NT + tid];
      } else {
        hc[e] = hi[ct][e];
        lc[e] = lo[ct][e];
      }
    }
    double v[PL];
#pragma unroll
    for (int a = 0; a < PL; ++a) v[a] = vS[cl * PL + a];
    double pa = 0.0;
    double mx = 0.0;
#pragma unroll
    for (int gq = 0; gq < 4; ++gq) {
      const int rb0 = 32 * wr + 8 * gq + 4 * (lane >> 5);  // row within the tile
      double xs[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = rb0 + r, e = 4 * gq + r;
        double x = fma((double)hc[e], 65536.0, (double)lc[e]) * zS[rr];
#pragma unroll
        for (int a = 0; a < PL; ++a) x -= Qs[rr * PL + a] * v[a];
        xs[r] = x;
        if (EPI == 0) {
          mx = fmax(mx, fabs(x));
        } else if (!UR) {
          pa += Vs[rr] * x * x;
        } else {
          const int64_t row = m0 + rr;
          if (row >= zl && row <= zl + PL)
            sstat[col * ss + 2 * PL + 3 + (row - zl)] = x;
          else
            pa += Vs[rr] * x * x;
        }
      }
      if (EPI == 0) *(v4d*)(X + col * np + m0 + rb0) = (v4d){xs[0], xs[1], xs[2], xs[3]};
      __builtin_amdgcn_sched_barrier(0);  // keep the row groups' table reads from being hoisted together
    }
    if (EPI == 0) {
      const double m = fmax(mx, __shfl_xor(mx, 32, 64));
      if ((lane >> 5) == 0 && col < mb)
        atomicMax((unsigned long long*)(sstat + col * ss + 2 * PL + 2), (unsigned long long)__double_as_longlong(m));
    } else {
      const double sq = pa + __shfl_xor(pa, 32, 64);
      if ((lane >> 5) == 0) Ps[wr * BN + cl] = sq;
    }
  }
  };
  if (urow_tile)
    columns(std::true_type{});
  else
    columns(std::false_type{});
  if (EPI == 1 && !ext) {
    __syncthreads();
    // the WR row slices of the tile combine (fixed order); one partial per
    // (row tile, SNP)
    for (int cl = tid; cl < BN; cl += NT) {
      double sum = 0.0;
#pragma unroll
      for (int w = 0; w < WR; ++w) sum += Ps[w * BN + cl];
      part[tm * mbp + n0 + cl] = sum;
    }
  }
}

template <int PL, int EPI, int CT, int WR, int WC, int DL>
__global__ void __launch_bounds__(64 * WR * WC, (rot_waves<PL, EPI, CT>())) k_rot_i8(RotArgs a) {
  rot_tile<PL, EPI, CT, WR, WC, DL>(a.np, a.nz, a.zl, a.mb, a.mbp, a.ntn, a.rg, a.tri, a.Zd, a.zs, a.Gp, a.Qt, a.Cq,
                                    a.sstat, a.X, a.Dv, a.part, blockIdx.x);
}

// The rotations of several plans' blocks in one launch.
template <int PL, int EPI, int CT, int WR, int WC, int DL>
__global__ void __launch_bounds__(64 * WR * WC, (rot_waves<PL, EPI, CT>())) k_rot_i8_batch(BatchArgs<RotArgs> B) {
  const int64_t b = blockIdx.x;
  const int k = batch_plan(B, b);
  const RotArgs& a = B.a[k];
  rot_tile<PL, EPI, CT, WR, WC, DL>(a.np, a.nz, a.zl, a.mb, a.mbp, a.ntn, a.rg, a.tri, a.Zd, a.zs, a.Gp, a.Qt, a.Cq,
                                    a.sstat, a.X, a.Dv, a.part, b - B.start[k]);
}

// Rotation tile configurations (CT 32-column MFMA tiles per wave, WR x WC
// waves; DL: staged by direct global-to-LDS loads into a ring of three (DL3)
// or four (DL4) K slices, two or three slices in flight and no staging
// registers or LDS stores issued by the waves, else through registers one
// slice ahead), all with 64-row
// tiles so that the single-trait partials (one per 64-row tile, combined over
// the WR = 2 wave rows in a fixed order) are bitwise the same whichever is
// chosen:
//   0: 2, 2, 2, DL3 64 x 128 tile, 4 waves (two work-groups per CU); built-in
//   1: 4, 2, 1      64 x 128 tile, 2 waves, four column tiles per wave
//   2: 2, 2, 4      64 x 256 tile, 8 waves
//   3: 4, 2, 2      64 x 256 tile, 4 waves, four column tiles per wave
//   4: 1, 2, 2      64 x 64 tile, 4 waves, one column tile per wave (three
//                   work-groups per CU: more loads in flight per CU)
//   5: 2, 2, 2      as 0, register-staged
//   6: 2, 2, 4, DL3 as 2, direct loads (one work-group per CU)
//   7: 1, 2, 2, DL3 as 4, direct loads
//   8: 2, 2, 4, DL4 as 6, three slices in flight
//   9: 2, 2, 2, DL4 as 0, three slices in flight (one work-group per CU)
//  10: the Z-resident kernel (k_rotz.hip), where it applies
constexpr int ROT_BM = 64;
static_assert(ROT_CONFIGS == 11, "rotation configurations");
static_assert(SNP_PAD % 256 == 0 && KPAD % ROT_BM == 0 && ZEXT == ROT_BM, "rotation tiles must divide the paddings");

// Single-trait finish: sums the per-row-tile partials of each SNP in a fixed
// order and solves the cell (Schur complement, FP64).  A work-group takes 64
// SNPs; its four waves sum interleaved row tiles, then wave 0 adds the four.
// With pair (the Z-resident rotation) the partials are per 32-row slice and a
// 64-row tile's partial is the sum of its two slices', first slice first, as
// the staged rotations form it.
// LIN 0 (FP64 path): each partial holds c', r' and a.  LIN 1 (mixed path):
// each partial holds a; c' and r' are in the SNP's statistics (written by the
// rotation's extra row tile).
template <int PL, int LIN>
__global__ void __launch_bounds__(256) k_fin_t1(int64_t nrt, int64_t m_blk, int64_t mbp, int pair,
                                                const double* __restrict__ part, const double* __restrict__ tpar,
                                                const double* __restrict__ sstat, uint32_t flags, CellOut out) {
  constexpr int NP = LIN ? 1 : PL + 2;  // partial values per row tile
  __shared__ double red[4][64][NP + 1];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  double s[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) s[q] = 0.0;
  if (i < m_blk) {
    if (LIN && pair)
      for (int64_t rt = wid; rt < nrt; rt += 4) s[0] += part[(2 * rt) * mbp + i] + part[(2 * rt + 1) * mbp + i];
    else
      for (int64_t rt = wid; rt < nrt; rt += 4) {
#pragma unroll
        for (int q = 0; q < NP; ++q) s[q] += part[(rt * NP + q) * mbp + i];
      }
  }
#pragma unroll
  for (int q = 0; q < NP; ++q) red[wid][lane][q] = s[q];
  __syncthreads();
  if (wid != 0 || i >= m_blk) return;
#pragma unroll
  for (int q = 0; q < NP; ++q) s[q] = ((red[0][lane][q] + red[1][lane][q]) + red[2][lane][q]) + red[3][lane][q];
  const double* st = sstat + i * snp_stride(PL);
  if constexpr (LIN) {
    double c[PL];
#pragma unroll
    for (int a = 0; a < PL; ++a) c[a] = st[2 * PL + 3 + a];
    schur_store<PL>(c, st[3 * PL + 3], s[0], tpar, st, flags, i, 0, out);
  } else {
    schur_store<PL>(s, s[PL], s[PL + 1], tpar, st, flags, i, 0, out);
  }
}

// Digit encoding of the rotated SNPs for the grid contraction: x with scale
// max_k |x_k|, x o x with scale (max_k |x_k|)^2, four planes each, written
// K-tiled.  A work-group takes one 32-deep slice of 32 SNPs; eight threads
// share a SNP (four eigen rows each), so every plane receives one contiguous
// kilobyte per work-group.
struct QuantArgs {
  int64_t np, mbp, nbx;  // nbx: 32-SNP groups of the block (the work-groups along the SNPs)
  int pL;
  const double* X;
  const double* sstat;
  int8_t* Xd;
};

// Work-group (bx, by): SNPs 32 bx .., eigen rows 32 by ..
__device__ __forceinline__ void quant_tile(const QuantArgs& a, int64_t bx, int64_t by) {
  const int64_t np = a.np, mbp = a.mbp;
  const int pL = a.pL;
  const double* __restrict__ X = a.X;
  const double* __restrict__ sstat = a.sstat;
  int8_t* __restrict__ Xd = a.Xd;
  const int64_t i = bx * 32 + (threadIdx.x >> 3);
  const int64_t k = by * 32 + 4 * (threadIdx.x & 7);
  const int64_t xplane = mbp * np;
  const double mx = sstat[i * snp_stride(pL) + 2 * pL + 2];
  const double inv = mx > 0.0 ? 1.0 / mx : 0.0, inv2 = inv * inv;
  const v4d x = *(const v4d*)(X + i * np + k);
  int32_t pk[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    int8_t d[4], e[4];
    digits4(quantize(x[r], inv), d);
    digits4(quantize(x[r] * x[r], inv2), e);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      pk[q] |= ((int32_t)(uint8_t)d[q]) << (8 * r);
      pk[4 + q] |= ((int32_t)(uint8_t)e[q]) << (8 * r);
    }
  }
  const int64_t off = kt32(i, k, mbp);
#pragma unroll
  for (int q = 0; q < 8; ++q) *(int32_t*)(Xd + q * xplane + off) = pk[q];
}

__global__ void __launch_bounds__(256) k_quant(QuantArgs a) { quant_tile(a, blockIdx.x, blockIdx.y); }

// The encodings of several plans' blocks in one launch (grid flattened per
// plan: nbx x n_pad / 32 work-groups).
__global__ void __launch_bounds__(256) k_quant_batch(BatchArgs<QuantArgs> B) {
  const int64_t b = blockIdx.x;
  const int k = batch_plan(B, b);
  const int64_t l = b - B.start[k];
  quant_tile(B.a[k], l % B.a[k].nbx, l / B.a[k].nbx);
}

// Ring depth actually used: a four-slot ring whose LDS (slots, the larger
// slot 0 for the single-trait partials, epilogue tables) would not fit a CU
// falls back to three slots.
template <int PL, int EPI, int CT, int WR, int WC, int DL>
constexpr int rot_ring() {
  constexpr int BM = 32 * WR, BN = 32 * CT * WC, FS = 8 * WR + 2 * CT * WC;
  constexpr int ps = EPI == 1 ? WR * BN * 8 : 0;
  constexpr int tab = (BM * PL + BM + BN * PL + (EPI == 1 ? BM : 0)) * 8;
  constexpr int lds = (FS * 1024 > ps ? FS * 1024 : ps) + (DL - 1) * FS * 1024 + tab;
  return (DL == 4 && lds > 159 * 1024) ? 3 : DL;
}

template <int CT, int WR, int WC, int DL>
static hipError_t rotate_cfg(const Plan& p, int64_t m_blk) {
  constexpr int BN = 32 * CT * WC;
  static_assert(32 * WR == ROT_BM && SNP_PAD % BN == 0, "rotation tile");
  const Workspace& W = p.ws;
  const int64_t ntn = roundup(m_blk, SNP_PAD) / BN, ntm = p.zrows / ROT_BM;
  const int rg = p.rot_rg ? p.rot_rg : rot_rg_builtin(p);  // XCD grid: rg row groups x 8 / rg SNP groups
  const int tri = (p.flags & CLAK_CHOL) ? 1 : 0;
  const int64_t gm = (ntm + rg - 1) / rg, gn = (ntn + 8 / rg - 1) / (8 / rg);
  dim3 grid((unsigned)(8 * gm * gn));
  dim3 block(64 * WR * WC);
#define CLAK_ROT(PLV, EPI, XP, DP, PP)                                                                         \
  case PLV:                                                                                                        \
    k_rot_i8<PLV, EPI, CT, WR, WC, rot_ring<PLV, EPI, CT, WR, WC, DL>()><<<grid, block, 0, p.stream>>>(RotArgs{    \
        p.n_pad, p.zrows, p.zlin, m_blk, p.mb_pad, ntn, rg, tri, W.Zd, W.zs, W.Gp, W.Qt, W.Cq, W.sstat, XP, DP, PP}); \
    break;
  if (p.fused_t1) {
    switch (p.pL) {
#define CLAK_R1(PLV) CLAK_ROT(PLV, 1, nullptr, W.D64, W.part)
      CLAK_R1(1) CLAK_R1(2) CLAK_R1(3) CLAK_R1(4) CLAK_R1(5) CLAK_R1(6) CLAK_R1(7) CLAK_R1(8)
#undef CLAK_R1
      default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  switch (p.pL) {
#define CLAK_R0(PLV) CLAK_ROT(PLV, 0, W.X64, nullptr, nullptr)
    CLAK_R0(1) CLAK_R0(2) CLAK_R0(3) CLAK_R0(4) CLAK_R0(5) CLAK_R0(6) CLAK_R0(7) CLAK_R0(8)
#undef CLAK_R0
    default:
      return hipErrorInvalidValue;
  }
#undef CLAK_ROT
  return hipGetLastError();
}

hipError_t launch_rotate_snps_mixed(const Plan& p, int64_t m_blk) {
  if (rot_zs_active(p)) return launch_rotate_zs(p, m_blk);
  switch (p.rot_cfg && p.rot_cfg != 10 ? p.rot_cfg : (rot_wide_builtin(p) ? 6 : 0)) {
    case 1:
      return rotate_cfg<4, 2, 1, 0>(p, m_blk);
    case 2:
      return rotate_cfg<2, 2, 4, 0>(p, m_blk);
    case 3:
      return rotate_cfg<4, 2, 2, 0>(p, m_blk);
    case 4:
      return rotate_cfg<1, 2, 2, 0>(p, m_blk);
    case 5:
      return rotate_cfg<2, 2, 2, 0>(p, m_blk);
    case 6:
      return rotate_cfg<2, 2, 4, 3>(p, m_blk);
    case 7:
      return rotate_cfg<1, 2, 2, 3>(p, m_blk);
    case 8:
      return rotate_cfg<2, 2, 4, 4>(p, m_blk);
    case 9:
      return rotate_cfg<2, 2, 2, 4>(p, m_blk);

    default:
      return rotate_cfg<2, 2, 2, 3>(p, m_blk);
  }
}

// Batched rotations of several multi-trait plans' blocks, with the built-in
// tiles of such plans (64 x 128, direct loads into a three-slot ring); each
// plan keeps its own XCD row grouping.
template <int PL>
static hipError_t rotate_batch_pl(const BatchItem* it, int count, hipStream_t st) {
  constexpr int CT = 2, WR = 2, WC = 2, DL = 3, BN = 32 * CT * WC;
  BatchArgs<RotArgs> B{};
  B.count = count;
  for (int k = 0; k < count; ++k) {
    const Plan& p = *it[k].p;
    const Slot& S = p.ws.slot[it[k].slot];
    const int64_t ntn = roundup(it[k].m_blk, SNP_PAD) / BN, ntm = p.zrows / ROT_BM;
    const int rg = p.rot_rg ? p.rot_rg : rot_rg_builtin(p);
    const int64_t gm = (ntm + rg - 1) / rg, gn = (ntn + 8 / rg - 1) / (8 / rg);
    B.a[k] = RotArgs{p.n_pad, p.zrows, p.zlin, it[k].m_blk, p.mb_pad, ntn, rg, 0, p.ws.Zd, p.ws.zs, S.Gp, p.ws.Qt,
                     p.ws.Cq, S.sstat, S.X64, nullptr, nullptr};
    B.start[k + 1] = B.start[k] + 8 * gm * gn;
  }
  k_rot_i8_batch<PL, 0, CT, WR, WC, rot_ring<PL, 0, CT, WR, WC, DL>()>
      <<<dim3((unsigned)B.start[count]), dim3(64 * WR * WC), 0, st>>>(B);
  return hipGetLastError();
}

hipError_t launch_rotate_batch(const BatchItem* it, int count, hipStream_t st) {
  if (count < 1 || count > MAX_BATCH) return hipErrorInvalidValue;
  switch (it[0].p->pL) {
    case 1:
      return rotate_batch_pl<1>(it, count, st);
    case 2:
      return rotate_batch_pl<2>(it, count, st);
    case 3:
      return rotate_batch_pl<3>(it, count, st);
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_encode_batch(const BatchItem* it, int count, hipStream_t st) {
  if (count < 1 || count > MAX_BATCH) return hipErrorInvalidValue;
  BatchArgs<QuantArgs> B{};
  B.count = count;
  for (int k = 0; k < count; ++k) {
    const Plan& p = *it[k].p;
    const Slot& S = p.ws.slot[it[k].slot];
    const int64_t nbx = (it[k].m_blk + 31) / 32;
    B.a[k] = QuantArgs{p.n_pad, p.mb_pad, nbx, (int)p.pL, S.X64, S.sstat, S.Xd};
    B.start[k + 1] = B.start[k] + nbx * (p.n_pad / 32);
  }
  k_quant_batch<<<dim3((unsigned)B.start[count]), 256, 0, st>>>(B);
  return hipGetLastError();
}

hipError_t launch_encode(const Plan& p, int64_t m_blk) {
  if (p.prec != CLAK_PREC_MIXED || p.fused_t1) return hipSuccess;
  dim3 qgrid((unsigned)((m_blk + 31) / 32), (unsigned)(p.n_pad / 32));
  k_quant<<<qgrid, 256, 0, p.stream>>>(
      QuantArgs{p.n_pad, p.mb_pad, (m_blk + 31) / 32, (int)p.pL, p.ws.X64, p.ws.sstat, p.ws.Xd});
  return hipGetLastError();
}
// ------------------------------------------------------------------ grid
//
// The inner loop of the multi-trait CLAK-Eig listing for a tile of 64 SNPs x
// 16 traits: W_R^T W_L, W_R^T Y_j and W_R^T W_R become, with the per-trait
// operand of the trait kernel, c' = V_c^T x, r' = (D e)^T x and a = d^T (x o x).
// x (4 planes) multiplies the 16 (PL+1) operand columns, x o x (4 planes) the
// 16 d columns.  Digit products are grouped by total weight g = a + b <= 3
// into four exact int32 accumulators.
template <int PL>
__global__ void __launch_bounds__(256) k_grid_i8(int64_t np, int64_t m_blk, int64_t mbp, int64_t t, int64_t tp,
                                                 const int8_t* __restrict__ Xd,
                                                 int64_t xplane, const int8_t* __restrict__ Vd,
                                                 int64_t vplane, const int8_t* __restrict__ Dd, int64_t dplane,
                                                 const double* __restrict__ vs, const double* __restrict__ ds,
                                                 const double* __restrict__ tpar, const double* __restrict__ sstat,
                                                 uint32_t flags, CellOut out) {
  constexpr int NCV = 16 * (PL + 1), NC = NCV + 16, NCT = NC / 16, BK = 64;
  constexpr int A_BYTES = 8 * 64 * LROW, B_BYTES = 4 * NC * LROW;
  constexpr int C_BYTES = 16 * (NC + 1) * 8;
  constexpr int SMEM = (A_BYTES + B_BYTES) > C_BYTES ? (A_BYTES + B_BYTES) : C_BYTES;
  __shared__ __attribute__((aligned(16))) int8_t smem[SMEM];
  int8_t(*As)[64][LROW] = (int8_t(*)[64][LROW])smem;             // [8][64][LROW]
  int8_t(*Bs)[NC][LROW] = (int8_t(*)[NC][LROW])(smem + A_BYTES);  // [4][NC][LROW]
  double(*Cs)[NC + 1] = (double(*)[NC + 1])smem;                  // [16][NC+1]
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int64_t i0 = (int64_t)blockIdx.x * 64, j0 = (int64_t)blockIdx.y * 16;

  v4i acc[NCT][4];
#pragma unroll
  for (int c = 0; c < NCT; ++c)
#pragma unroll
    for (int g = 0; g < 4; ++g) acc[c][g] = (v4i){0, 0, 0, 0};

  for (int64_t k0 = 0; k0 < np; k0 += BK) {
    // A: 8 planes x 64 SNPs x 64 bytes
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int c = tid + 256 * q;
      const int pl = c >> 8, s = (c >> 2) & 63, kq = c & 3;
      *(v4i*)(&As[pl][s][16 * kq]) = *(const v4i*)(Xd + pl * xplane + kt32(i0 + s, k0 + 16 * kq, mbp));
    }
    // B: 4 planes x NC columns x 64 bytes
    for (int c = tid; c < 4 * NC * 4; c += 256) {
      const int pl = c / (NC * 4), rem = c % (NC * 4), col = rem >> 2, kq = rem & 3;
      const int8_t* src =
          (col < NCV) ? Vd + pl * vplane + kt32(vrow(j0 + col / (PL + 1), col % (PL + 1), PL + 1), k0 + 16 * kq, tp * (PL + 1))
                      : Dd + pl * dplane + kt32(j0 + col - NCV, k0 + 16 * kq, tp);
      *(v4i*)(&Bs[pl][col][16 * kq]) = *(const v4i*)src;
    }
    __syncthreads();
    v4i xa[4], xq[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      xa[p] = *(const v4i*)(&As[p][16 * wid + (lane & 15)][16 * (lane >> 4)]);
      xq[p] = *(const v4i*)(&As[4 + p][16 * wid + (lane & 15)][16 * (lane >> 4)]);
    }
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) {
      v4i bv[4];
#pragma unroll
      for (int p = 0; p < 4; ++p) bv[p] = *(const v4i*)(&Bs[p][16 * ct + (lane & 15)][16 * (lane >> 4)]);
      const v4i* A = (ct < PL + 1) ? xa : xq;
      acc[ct][0] = mfma_i8(A[0], bv[0], acc[ct][0]);
      acc[ct][1] = mfma_i8(A[0], bv[1], acc[ct][1]);
      acc[ct][1] = mfma_i8(A[1], bv[0], acc[ct][1]);
      acc[ct][2] = mfma_i8(A[0], bv[2], acc[ct][2]);
      acc[ct][2] = mfma_i8(A[1], bv[1], acc[ct][2]);
      acc[ct][2] = mfma_i8(A[2], bv[0], acc[ct][2]);
      acc[ct][3] = mfma_i8(A[0], bv[3], acc[ct][3]);
      acc[ct][3] = mfma_i8(A[1], bv[2], acc[ct][3]);
      acc[ct][3] = mfma_i8(A[2], bv[1], acc[ct][3]);
      acc[ct][3] = mfma_i8(A[3], bv[0], acc[ct][3]);
    }
    __syncthreads();
  }

  // epilogue: values in FP64 through LDS, one wave's 16 SNPs at a time
  const int64_t ss = snp_stride(PL);
  for (int w = 0; w < 4; ++w) {
    if (wid == w) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + 16 * w + 4 * (lane >> 4) + r;
        const double gs = sstat[i * ss + 2 * PL + 2];  // max_k |x~_k| of SNP i
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
          const int c = 16 * ct + (lane & 15);
          const double S = (((double)acc[ct][0][r] * 256.0 + (double)acc[ct][1][r]) * 256.0 + (double)acc[ct][2][r]) *
                               256.0 + (double)acc[ct][3][r];
          const double scale = (c < NCV) ? gs * vs[j0 * (PL + 1) + c] : gs * gs * ds[j0 + c - NCV];
          Cs[4 * (lane >> 4) + r][c] = S * scale * (1.0 / 127.0);
        }
      }
    }
    __syncthreads();
    {
      const int s = tid & 15, jj = tid >> 4;
      const int64_t i = i0 + 16 * w + s, j = j0 + jj;
      if (i < m_blk && j < t) {
        double c[PL];
#pragma unroll
        for (int l = 0; l < PL; ++l) c[l] = Cs[s][jj * (PL + 1) + l];
        const double r = Cs[s][jj * (PL + 1) + PL];
        const double a = Cs[s][NCV + jj];
        schur_store<PL>(c, r, a, tpar + j * trait_stride(PL), sstat + i * ss, flags, i, j, out);
      }
    }
    __syncthreads();
  }
}

// Grid contraction on v_mfma_i32_32x32x32_i8 for p_L <= 3.  A work-group
// takes 128 SNPs (one 32-SNP row tile per wave) x TT traits and keeps at most
// four 32 x 32 output tiles per wave (four digit-weight accumulators each,
// 256 accumulation registers).  It runs 1 + TT / 32 passes over K:
//   pass 0     : a = d^T (x o x) for the TT traits (x o x digits against d),
//                parked in FP64 registers;
//   pass 1 + g : for trait group g (32 traits), the p_L + 1 operand entries
//                q (q < p_L whitened covariates, q = p_L weighted residual)
//                against x, one 32-column tile per entry; then each lane
//                holds complete cells (16 SNPs of one trait) and solves them.
// The operand planes keep each entry of a 32-trait group in 32 consecutive
// rows, so each MFMA tile is one entry of 32 traits.  All passes form one sequence
// of 32-deep stages, double-buffered in LDS with a 48-byte row pitch
// (conflict-free 16-byte fragment reads), so the loads of the next pass are
// in flight during a pass's epilogue.  With the K-tiled digit layout every
// stage of a row tile is one contiguous run in HBM.  Work-groups go
// round-robin over the 8 XCDs; XCD x owns trait group x % xt (of xt groups)
// and SNP group x / xt, so its share of the trait operand stays in its L2.
constexpr int G32_PITCH = 48, G32_BM = 128, G32_STAGE = (4 * G32_BM + 4 * 4 * 32) * G32_PITCH;

// One 32-deep stage: NT output tiles of 32 x 32, digit products grouped by
// weight a + b <= 3 into acc[t][a + b].
template <int NT>
__device__ __forceinline__ void g32_stage(v16i (&acc)[4][4], const int8_t* As, const int8_t* Bs, int afrag,
                                          int bfrag) {
  v4i a[4];
#pragma unroll
  for (int p = 0; p < 4; ++p) a[p] = *(const v4i*)(As + p * G32_BM * G32_PITCH + afrag);
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    v4i b[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) b[p] = *(const v4i*)(Bs + (p * 4 + t) * 32 * G32_PITCH + bfrag);
    acc[t][0] = mfma32_i8(a[0], b[0], acc[t][0]);
    acc[t][1] = mfma32_i8(a[0], b[1], acc[t][1]);
    acc[t][2] = mfma32_i8(a[0], b[2], acc[t][2]);
    acc[t][3] = mfma32_i8(a[0], b[3], acc[t][3]);
    acc[t][1] = mfma32_i8(a[1], b[0], acc[t][1]);
    acc[t][2] = mfma32_i8(a[1], b[1], acc[t][2]);
    acc[t][3] = mfma32_i8(a[1], b[2], acc[t][3]);
    acc[t][2] = mfma32_i8(a[2], b[0], acc[t][2]);
    acc[t][3] = mfma32_i8(a[2], b[1], acc[t][3]);
    acc[t][3] = mfma32_i8(a[3], b[0], acc[t][3]);
  }
}


// One pass over K into NT accumulator tiles.  Lane l of wave w stages row
// 32 w + l % 32, half l / 32, of each 32-row group: the same lane pattern as
// the fragment reads, which keeps the LDS stores free of bank conflicts.
// pa: this lane's chunk of digit plane 0 of the SNP row tile (planes xplane
// apart, stages astride apart); pb: its chunk of operand plane w, first
// 32-row group (further groups 1024 bytes apart, stages bstride apart).
template <int NT>
__device__ __forceinline__ void g32_pass(v16i (&acc)[4][4], int8_t* smem, const int8_t* pa, int64_t xplane,
                                         int64_t astride, const int8_t* pb, int64_t bstride, int KT, int afrag,
                                         int bfrag) {
  const int wid = threadIdx.x >> 6;
  v4i ra[4], rb[NT];
  auto gload = [&](int kt) {
#pragma unroll
    for (int p = 0; p < 4; ++p) ra[p] = *(const v4i*)(pa + p * xplane + kt * astride);
#pragma unroll
    for (int u = 0; u < NT; ++u) rb[u] = *(const v4i*)(pb + u * 1024 + kt * bstride);
  };
  auto lstore = [&](int buf) {
    int8_t* As = smem + buf * G32_STAGE;
    int8_t* Bs = As + 4 * G32_BM * G32_PITCH;
#pragma unroll
    for (int p = 0; p < 4; ++p) *(v4i*)(As + p * G32_BM * G32_PITCH + afrag) = ra[p];
#pragma unroll
    for (int u = 0; u < NT; ++u) *(v4i*)(Bs + (wid * 4 + u) * 32 * G32_PITCH + bfrag) = rb[u];
  };
  gload(0);
  lstore(0);
  __syncthreads();
  if (KT > 1) gload(1);
  for (int kt = 0; kt < KT; ++kt) {
    const int8_t* As = smem + (kt & 1) * G32_STAGE;
    g32_stage<NT>(acc, As, As + 4 * G32_BM * G32_PITCH, afrag, bfrag);
    if (kt + 1 < KT) {
      lstore((kt + 1) & 1);
      if (kt + 2 < KT) gload(kt + 2);
    }
    __syncthreads();
  }
}

template <int PL, int TT>
__global__ void __launch_bounds__(256, 1)
    k_grid32(int64_t np, int64_t m_blk, int64_t mbp, int64_t t, int64_t tp, int64_t ntn, int64_t ntt, int xt,
             const int8_t* __restrict__ Xd, const int8_t* __restrict__ Vd, const int8_t* __restrict__ Dd,
             const double* __restrict__ vs, const double* __restrict__ ds, const double* __restrict__ tpar,
             const double* __restrict__ sstat, uint32_t flags, CellOut out) {
  constexpr int NV = PL + 1, NG = TT / 32, NH = (NV + 3) / 4;  // NH chunks of at most four entries
  static_assert(NG <= 4 && NH <= 3, "at most four accumulator tiles per wave, p_L <= 11");
  __shared__ __attribute__((aligned(16))) int8_t smem[2 * G32_STAGE];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int64_t xcd = blockIdx.x % 8, idx = blockIdx.x / 8, xs = 8 / xt;
  const int64_t gt = (ntt + xt - 1) / xt, gs = (ntn + xs - 1) / xs;
  const int64_t tt = (xcd % xt) * gt + idx % gt, tn = (xcd / xt) * gs + idx / gt;
  if (idx >= gt * gs || tt >= ntt || tn >= ntn) return;
  const int64_t i0 = tn * G32_BM, j0 = tt * TT;
  const int64_t xplane = mbp * np, vrows = tp * NV, vplane = vrows * np, dplane = tp * np;
  const int KT = (int)(np / 32);
  const int afrag = (32 * wid + (lane & 31)) * G32_PITCH + 16 * (lane >> 5);
  const int bfrag = (lane & 31) * G32_PITCH + 16 * (lane >> 5);
  // this lane's staging chunk: row lane % 32 of a 32-row group, half lane / 32
  const int lchunk = (lane & 31) * 32 + 16 * (lane >> 5);
  const int8_t* pa = Xd + (i0 + 32 * wid) * 32 + lchunk;
  const int64_t ss = snp_stride(PL);

  v16i acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int g = 0; g < 4; ++g) acc[u][g] = (v16i){};
  // pass 0: a = d^T (x o x) of the TT traits, unscaled
  g32_pass<NG>(acc, smem, pa + 4 * xplane, xplane, mbp * 32, Dd + wid * dplane + j0 * 32 + lchunk, tp * 32, KT, afrag,
               bfrag);
  double araw[NG][16];
#pragma unroll
  for (int u = 0; u < NG; ++u)
#pragma unroll
    for (int r = 0; r < 16; ++r) araw[u][r] = g32_value(acc[u], r);

#pragma unroll
  for (int g = 0; g < NG; ++g) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[u][e] = (v16i){};
    // lane: trait j0 + 32 g + lane % 32, SNP rows 8 (r / 4) + 4 (lane / 32) + r % 4 of the wave's tile
    const int64_t j = j0 + 32 * g + (lane & 31);
    const int8_t* pv = Vd + wid * vplane + vrow(j0 + 32 * g, 0, NV) * 32 + lchunk;
    if constexpr (NH > 1) {
      // more than four entries: passes over chunks of four, ||c'||^2 carried
      // in FP64 between them (SNP effect and SE only; the full vector takes
      // the 16x16x64 kernel)
      double ccp[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) ccp[r] = 0.0;
      auto chunk = [&](auto hc) {
        constexpr int H = decltype(hc)::value, NT = (NV - 4 * H) < 4 ? (NV - 4 * H) : 4;
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int e = 0; e < 4; ++e) acc[u][e] = (v16i){};
        g32_pass<NT>(acc, smem, pa, xplane, mbp * 32, pv + 128 * 32 * H, vrows * 32, KT, afrag, bfrag);
        if (j >= t) return;
        double sc[NT];
#pragma unroll
        for (int u = 0; u < NT; ++u) sc[u] = vs[j * NV + 4 * H + u] * (1.0 / 127.0);
        const double sd = ds[j] * (1.0 / 127.0);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int64_t i = i0 + 32 * wid + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
          if (i < m_blk) {
            const double* st = sstat + i * ss;
            const double gx = st[2 * PL + 2];
            double rr = 0.0;
#pragma unroll
            for (int u = 0; u < NT; ++u) {
              const double v = g32_value(acc[u], r) * sc[u] * gx;
              if (4 * H + u < PL)
                ccp[r] += v * v;
              else
                rr = v;
            }
            if (H == NH - 1)
              schur_store_cc<PL>(ccp[r], rr, araw[g][r] * sd * gx * gx, tpar + j * trait_stride(PL), st, flags, i,
                                 j, out);
          }
          __builtin_amdgcn_sched_barrier(0);
        }
      };
      chunk(std::integral_constant<int, 0>{});
      chunk(std::integral_constant<int, 1>{});
      if constexpr (NH > 2) chunk(std::integral_constant<int, 2>{});
      continue;
    }
    g32_pass<NV>(acc, smem, pa, xplane, mbp * 32, pv, vrows * 32, KT, afrag, bfrag);
    if (j < t) {
      double sc[NV];
#pragma unroll
      for (int q = 0; q < NV; ++q) sc[q] = vs[j * NV + q] * (1.0 / 127.0);
      const double sd = ds[j] * (1.0 / 127.0);
      const double* tpj = tpar + j * trait_stride(PL);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t i = i0 + 32 * wid + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (i < m_blk) {
          const double* st = sstat + i * ss;
          const double gx = st[2 * PL + 2];  // max_k |x~_k| of SNP i
          double v[NV];
#pragma unroll
          for (int q = 0; q < NV; ++q) v[q] = g32_value(acc[q], r) * sc[q] * gx;
          schur_store<PL>(v, v[PL], araw[g][r] * sd * gx * gx, tpj, st, flags, i, j, out);
        }
        __builtin_amdgcn_sched_barrier(0);  // one cell at a time: keeps the accumulator reads from being hoisted
      }
    }
  }
}

hipError_t launch_fin_t1(const Plan& p, int64_t m_blk, const CellOut& out) {
  const Workspace& W = p.ws;
  dim3 fgrid((unsigned)((m_blk + 63) / 64));
  const int64_t nrt = p.prec == CLAK_PREC_MIXED ? p.n_pad / ROT_BM : p.n_pad / 64;
  const int pair = rot_zs_active(p) ? 1 : 0;
#define CLAK_F1(PLV)                                                                                            \
  case PLV:                                                                                                     \
    if (lin_rows(p))                                                                                            \
      k_fin_t1<PLV, 1><<<fgrid, 256, 0, p.stream>>>(nrt, m_blk, p.mb_pad, pair, W.part, W.tpar, W.sstat, p.flags, \
                                                    out);                                                       \
    else                                                                                                        \
      k_fin_t1<PLV, 0><<<fgrid, 256, 0, p.stream>>>(nrt, m_blk, p.mb_pad, 0, W.part, W.tpar, W.sstat, p.flags,    \
                                                    out);                                                       \
    break;
  switch (p.pL) {
    CLAK_F1(1) CLAK_F1(2) CLAK_F1(3) CLAK_F1(4) CLAK_F1(5) CLAK_F1(6) CLAK_F1(7) CLAK_F1(8)
    CLAK_F1(9) CLAK_F1(10) CLAK_F1(11) CLAK_F1(12) CLAK_F1(13) CLAK_F1(14) CLAK_F1(15) CLAK_F1(16)
    default:
      return hipErrorInvalidValue;
  }
#undef CLAK_F1
  return hipGetLastError();
}

hipError_t launch_grid_mixed(const Plan& p, int64_t m_blk, const CellOut& out) {
  const Workspace& W = p.ws;
  if (p.fused_t1) return launch_fin_t1(p, m_blk, out);
  // built-in for p_L <= 3: the one-pass ring kernel (k_grid.hip); grid_tt =
  // 32 or 64 selects the two-stage kernel below
  if (p.grid_tt == 0 && p.pL <= 3) return launch_grid_ring(p, m_blk, out);
  if (p.pL <= 3 || !(p.flags & CLAK_OUT_FULL)) {
    // traits per work-group: 64 unless 32 gives fewer modelled
    // dispatch rounds of 256 work-groups x traits per tile
    const int64_t ntn = (m_blk + G32_BM - 1) / G32_BM;
    int tt = 32;
    for (int c = 64; c <= 64; c *= 2) {
      const int64_t r_c = (ntn * ((p.t + c - 1) / c) + 255) / 256, r_t = (ntn * ((p.t + tt - 1) / tt) + 255) / 256;
      if (r_c * c <= r_t * tt) tt = c;
    }
    if (p.grid_tt) tt = p.grid_tt;
    const int64_t ntt = (p.t + tt - 1) / tt;
    int xt = 1;
    while (xt < 8 && 2 * xt <= ntt) xt *= 2;
    if (p.grid_xt) xt = p.grid_xt;
    const int64_t gt = (ntt + xt - 1) / xt, gs = (ntn + 8 / xt - 1) / (8 / xt);
    const dim3 g32((unsigned)(8 * gt * gs));
#define CLAK_G32(PLV, TTV)                                                                                       \
  k_grid32<PLV, TTV><<<g32, 256, 0, p.stream>>>(p.n_pad, m_blk, p.mb_pad, p.t, p.t_pad, ntn, ntt, xt, W.Xd, W.Vd, \
                                                W.Dd, W.vs, W.ds, W.tpar, W.sstat, p.flags, out)
#define CLAK_G32T(PLV)   \
  case PLV:              \
    if (tt == 32)        \
      CLAK_G32(PLV, 32); \
    else                 \
      CLAK_G32(PLV, 64); \
    break;
    switch (p.pL) {
      CLAK_G32T(1) CLAK_G32T(2) CLAK_G32T(3) CLAK_G32T(4) CLAK_G32T(5) CLAK_G32T(6) CLAK_G32T(7) CLAK_G32T(8)
      default:
        return hipErrorInvalidValue;
    }
#undef CLAK_G32T
#undef CLAK_G32
    return hipGetLastError();
  }
  dim3 grid((unsigned)((m_blk + 63) / 64), (unsigned)(p.t_pad / 16));
  const int64_t xplane = p.mb_pad * p.n_pad, vplane = p.t_pad * (p.pL + 1) * p.n_pad, dplane = p.t_pad * p.n_pad;
#define CLAK_GI8(PLV)                                                                                              \
  case PLV:                                                                                                        \
    k_grid_i8<PLV><<<grid, 256, 0, p.stream>>>(p.n_pad, m_blk, p.mb_pad, p.t, p.t_pad, W.Xd, xplane, W.Vd, vplane, \
                                               W.Dd, dplane, W.vs, W.ds, W.tpar, W.sstat, p.flags, out);           \
    break;
  switch (p.pL) {
    CLAK_GI8(4) CLAK_GI8(5) CLAK_GI8(6) CLAK_GI8(7) CLAK_GI8(8)
    default:
      return hipErrorInvalidValue;
  }
#undef CLAK_GI8
  return hipGetLastError();
}

}  // namespace clak
