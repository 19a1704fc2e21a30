// SNP block ingest: moves a caller block of genotypes into the padded int8
// staging panel of the plan and computes, per SNP, the FP64 statistics of its
// centring against the covariates (projection onto Q_L, residual norm,
// degeneracy flag).
#include <hip/hip_fp16.h>

#include <algorithm>

#include "common.hpp"

namespace clak {

// Pass 1.  A work-group takes 64 SNPs (one per lane) and the individual
// windows s, s + S, s + 2S, ... (128 individuals each; blockIdx.y = s; S from
// ingest_splits, about four windows per work-group); in a window wave w
// handles individuals [16w, 16w + 16) of every lane's SNP, and the window's
// 128 rows of Q_L are staged in LDS (read back as wave-uniform broadcasts).
// The work-group writes the int8 panel rows of its windows and one partial
// (Q_L^T g, g^T g, invalid-genotype count) per SNP, or, when S = 1, the SNP's
// statistics themselves (pass 2 is then not launched).
// ALIGN is the byte alignment shared by G and its leading dimension (u8, and
// for 2-bit rows whether 4-byte words can be read).  KIND: 0 u8, 1 f16, 2
// 2-bit codes, four individuals per byte, individual i in bits 2 (i % 4) and
// 2 (i % 4) + 1 of byte i / 4: 00 -> 2, 10 -> 1, 11 -> 0 copies of the first
// allele, 01 -> missing (an invalid genotype).
constexpr int ING_WAVES = 8;

// genotype of a 2-bit code (3 stands for missing)
// (byte c of 0x00010302 is the value of code c: 2, 3, 1, 0)
__device__ __forceinline__ uint8_t p2_value(uint32_t code) { return (uint8_t)((0x00010302u >> (8 * code)) & 0xffu); }

// Arguments of the ingest of one plan's block (S: individual windows split
// over S work-groups per 64 SNPs).
struct IngArgs {
  int64_t n, np, m_blk, m_pad, mbp;
  const void* G;
  int64_t ldg;
  const double* QL;
  int8_t* Gp;
  double* ipart;
  int S;
  const double* Rinv;  // with S = 1 the work-group writes the statistics itself
  double* sstat;
};

// The statistics of one SNP from its sums t = (Q_L^T g, g^T g, invalid
// genotype count):
//   v = Q_L^T g, gamma = R^{-1} v, ||g - Q_L v|| = sqrt(gg - ||v||^2), and
//   flag = 2 if a genotype is not in {0, 1, 2}; 1 if g lies in span(X_L)
//   (gg == 0 or ||g - Q_L v||^2 <= 1e-10 gg) or the row pads the block; else 0.
template <int PL>
__device__ __forceinline__ void snp_statistics(const double* t, bool pad, const double* __restrict__ Rinv,
                                               double* st) {
  double vv = 0.0;
#pragma unroll
  for (int a = 0; a < PL; ++a) vv += t[a] * t[a];
  const double g2 = t[PL];
  const double res = g2 - vv;
  const int flag = t[PL + 1] > 0.0 ? 2 : ((pad || !(g2 > 0.0) || !(res > 1e-10 * g2)) ? 1 : 0);
#pragma unroll
  for (int a = 0; a < PL; ++a) {
    double gam = 0.0;
#pragma unroll
    for (int c = a; c < PL; ++c) gam += Rinv[a * PL + c] * t[c];
    st[a] = flag ? 0.0 : t[a];
    st[PL + a] = flag ? 0.0 : gam;
  }
  st[2 * PL] = flag ? 1.0 : sqrt(res);
  st[2 * PL + 1] = (double)flag;
  st[2 * PL + 2] = 0.0;
}

// Work-group (bx, s0): SNPs 64 bx .., windows s0, s0 + S, ...
template <int PL, int ALIGN, int KIND>
__device__ __forceinline__ void ingest_tile(const IngArgs& ia, int64_t bx, int64_t s0) {
  const int64_t n = ia.n, np = ia.np, m_blk = ia.m_blk, m_pad = ia.m_pad, mbp = ia.mbp, ldg = ia.ldg;
  const void* __restrict__ G = ia.G;
  const double* __restrict__ QL = ia.QL;
  int8_t* __restrict__ Gp = ia.Gp;
  double* __restrict__ ipart = ia.ipart;
  constexpr int NV = PL + 2;  // v, gg, bad
  constexpr int WIN = 16 * ING_WAVES;
  __shared__ double red[ING_WAVES][64][NV + 1];
  __shared__ __attribute__((aligned(1024))) double qs[PL][WIN];
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t snp = bx * 64 + lane;
  const int64_t S = ia.S;
  double acc[PL];
#pragma unroll
  for (int a = 0; a < PL; ++a) acc[a] = 0.0;
  double gg = 0.0;
  int bad = 0;
  for (int64_t w0 = s0 * WIN; w0 < np; w0 += S * WIN) {
    __syncthreads();  // every wave is done with the previous window's Q_L rows
    // the window's Q_L rows go straight to LDS (row a by wave a % 8, 16 bytes
    // a lane), so that their latency overlaps that of the genotype loads below
    for (int a = wid; a < PL; a += ING_WAVES)
      __builtin_amdgcn_global_load_lds(QL + w0 + a * np + 2 * lane, (lds_ptr_t)&qs[a][0], 16, 0, 0);
    const int64_t i0 = w0 + 16 * wid;
    uint8_t by[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) by[e] = 0;
    if (snp < m_blk) {
      if (KIND == 2) {
        const uint8_t* row = (const uint8_t*)G + snp * ldg + i0 / 4;
        uint32_t word = 0;
        if (i0 + 16 <= n && ALIGN >= 4) {
          word = *(const uint32_t*)__builtin_assume_aligned(row, 4);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (i0 + 4 * e < n) word |= (uint32_t)row[e] << (8 * e);
        }
#pragma unroll
        for (int e = 0; e < 16; ++e) by[e] = (i0 + e < n) ? p2_value((word >> (2 * e)) & 3u) : 0;
      } else if (KIND == 1) {
        const __half* row = (const __half*)G + snp * ldg + i0;
#pragma unroll
        for (int e = 0; e < 16; ++e)
          if (i0 + e < n) {
            const float f = __half2float(row[e]);
            by[e] = (f == 0.0f || f == 1.0f || f == 2.0f) ? (uint8_t)f : 3;
          }
      } else {
        const uint8_t* row = (const uint8_t*)G + snp * ldg + i0;
        if (i0 + 16 <= n) {
          __builtin_memcpy(by, __builtin_assume_aligned(row, ALIGN), 16);
        } else {
#pragma unroll
          for (int e = 0; e < 16; ++e) by[e] = (i0 + e < n) ? row[e] : 0;
        }
      }
    }
    double gd[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      if (by[e] > 2) {
        bad = 1;
        by[e] = 0;
      }
      gd[e] = (double)by[e];
      gg += gd[e] * gd[e];
    }
    if (snp < m_pad) __builtin_memcpy(__builtin_assume_aligned(Gp + kt32(snp, i0, mbp), 16), by, 16);
    wait_vm<0>();     // this wave's Q_L rows have landed
    __syncthreads();  // and every wave's
#pragma unroll
    for (int a = 0; a < PL; ++a) {
      const double* src = &qs[a][16 * wid];
      double t0 = 0.0, t1 = 0.0;
#pragma unroll
      for (int e = 0; e < 16; e += 2) {
        t0 += src[e] * gd[e];
        t1 += src[e + 1] * gd[e + 1];
      }
      acc[a] += t0 + t1;
    }
  }
#pragma unroll
  for (int a = 0; a < PL; ++a) red[wid][lane][a] = acc[a];
  red[wid][lane][PL] = gg;
  red[wid][lane][PL + 1] = (double)bad;
  __syncthreads();
  if (wid != 0 || snp >= m_pad) return;
  double t[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    t[q] = 0.0;
    for (int w = 0; w < ING_WAVES; ++w) t[q] += red[w][lane][q];
  }
  if (S == 1) {  // the whole sums: the statistics as pass 2 forms them (0 + t is t)
    snp_statistics<PL>(t, snp >= m_blk, ia.Rinv, ia.sstat + snp * snp_stride(PL));
  } else {
#pragma unroll
    for (int q = 0; q < NV; ++q) ipart[(s0 * NV + q) * mbp + snp] = t[q];
  }
}

template <int PL, int ALIGN, int KIND>
__global__ void __launch_bounds__(64 * ING_WAVES) k_ingest(IngArgs a) {
  ingest_tile<PL, ALIGN, KIND>(a, blockIdx.x, blockIdx.y);
}

// The ingests of several plans' blocks in one launch (per plan m_pad / 64 x S
// work-groups, flattened).
template <int PL, int ALIGN, int KIND>
__global__ void __launch_bounds__(64 * ING_WAVES) k_ingest_batch(BatchArgs<IngArgs> B) {
  const int64_t b = blockIdx.x;
  const int k = batch_plan(B, b);
  const int64_t l = b - B.start[k];
  ingest_tile<PL, ALIGN, KIND>(B.a[k], l / B.a[k].S, l % B.a[k].S);
}

// Pass 2 (S > 1), one thread per SNP: sums the S partials in a fixed order
// and writes the SNP's statistics (snp_statistics).  SNP rows in
// [m_blk, m_pad) become zero SNPs with flag 1.
struct FinArgs {
  int64_t m_blk, m_pad, mbp;
  int S;
  const double* ipart;
  const double* Rinv;
  double* sstat;
};

template <int PL>
__device__ __forceinline__ void ingest_fin_tile(const FinArgs& fa, int64_t bx) {
  const int64_t m_blk = fa.m_blk, m_pad = fa.m_pad, mbp = fa.mbp;
  const int S = fa.S;
  const double* __restrict__ ipart = fa.ipart;
  const double* __restrict__ Rinv = fa.Rinv;
  double* __restrict__ sstat = fa.sstat;
  constexpr int NV = PL + 2;
  const int64_t snp = bx * 256 + threadIdx.x;
  if (snp >= m_pad || S == 1) return;  // with one split pass 1 wrote the statistics
  double t[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) t[q] = 0.0;
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int q = 0; q < NV; ++q) t[q] += ipart[(s * NV + q) * mbp + snp];
  snp_statistics<PL>(t, snp >= m_blk, Rinv, sstat + snp * snp_stride(PL));
}

template <int PL>
__global__ void __launch_bounds__(256) k_ingest_fin(FinArgs a) {
  ingest_fin_tile<PL>(a, blockIdx.x);
}

template <int PL>
__global__ void __launch_bounds__(256) k_ingest_fin_batch(BatchArgs<FinArgs> B) {
  const int64_t b = blockIdx.x;
  const int k = batch_plan(B, b);
  ingest_fin_tile<PL>(B.a[k], b - B.start[k]);
}

template <int PL>
static void ingest_dispatch(const Plan& p, int64_t m_blk, int64_t m_pad, const void* d_G, int g_dtype, int64_t ldg) {
  const int S = ingest_splits(p);
  dim3 grid((unsigned)(m_pad / 64), (unsigned)S);
  const Workspace& W = p.ws;
  const dim3 block(64 * ING_WAVES);
  const IngArgs ia{p.n, p.n_pad, m_blk, m_pad, p.mb_pad, d_G, ldg, W.QL, W.Gp, W.ipart, S, W.Rinv, W.sstat};
  if (g_dtype == CLAK_G_F16) {
    k_ingest<PL, 1, 1><<<grid, block, 0, p.stream>>>(ia);
  } else if (g_dtype == CLAK_G_P2) {
    const bool words = ((uintptr_t)d_G % 4 == 0) && (ldg % 4 == 0);
    if (words)
      k_ingest<PL, 4, 2><<<grid, block, 0, p.stream>>>(ia);
    else
      k_ingest<PL, 1, 2><<<grid, block, 0, p.stream>>>(ia);
  } else {
    // widest alignment shared by the base address and the row pitch, capped at 16
    const uint64_t bits = (uint64_t)(uintptr_t)d_G | (uint64_t)ldg | 16u;
    const int align = (int)(bits & (~bits + 1));
#define CLAK_ING(A) k_ingest<PL, A, 0><<<grid, block, 0, p.stream>>>(ia)
    if (align >= 16)
      CLAK_ING(16);
    else if (align >= 8)
      CLAK_ING(8);
    else if (align >= 4)
      CLAK_ING(4);
    else
      CLAK_ING(1);
#undef CLAK_ING
  }
  if (S > 1)  // with one split pass 1 has written the statistics
    k_ingest_fin<PL><<<dim3((unsigned)(m_pad / 256)), 256, 0, p.stream>>>(
        FinArgs{m_blk, m_pad, p.mb_pad, S, W.ipart, W.Rinv, W.sstat});
}

template <int PL>
static hipError_t ingest_batch_pl(const BatchItem* it, int count, int g_dtype, hipStream_t st) {
  BatchArgs<IngArgs> B{};
  BatchArgs<FinArgs> F{};
  B.count = F.count = count;
  int align = 16;
  bool words = true, fin = false;  // fin: some plan has more than one split
  for (int k = 0; k < count; ++k) {
    const Plan& p = *it[k].p;
    const Slot& S = p.ws.slot[it[k].slot];
    const int64_t m_pad = roundup(it[k].m_blk, SNP_PAD);
    const int sp = ingest_splits(p);
    B.a[k] = IngArgs{p.n, p.n_pad, it[k].m_blk, m_pad, p.mb_pad, it[k].G, it[k].ldg, p.ws.QL, S.Gp, S.ipart, sp,
                     p.ws.Rinv, S.sstat};
    fin = fin || sp > 1;
    F.a[k] = FinArgs{it[k].m_blk, m_pad, p.mb_pad, sp, S.ipart, p.ws.Rinv, S.sstat};
    B.start[k + 1] = B.start[k] + m_pad / 64 * sp;
    F.start[k + 1] = F.start[k] + m_pad / 256;
    const uint64_t bits = (uint64_t)(uintptr_t)it[k].G | (uint64_t)it[k].ldg | 16u;
    align = std::min(align, (int)(bits & (~bits + 1)));
    words = words && ((uintptr_t)it[k].G % 4 == 0) && (it[k].ldg % 4 == 0);
  }
  const dim3 grid((unsigned)B.start[count]), block(64 * ING_WAVES);
  if (g_dtype == CLAK_G_F16)
    k_ingest_batch<PL, 1, 1><<<grid, block, 0, st>>>(B);
  else if (g_dtype == CLAK_G_P2)
    words ? k_ingest_batch<PL, 4, 2><<<grid, block, 0, st>>>(B) : k_ingest_batch<PL, 1, 2><<<grid, block, 0, st>>>(B);
  else if (align >= 16)
    k_ingest_batch<PL, 16, 0><<<grid, block, 0, st>>>(B);
  else if (align >= 8)
    k_ingest_batch<PL, 8, 0><<<grid, block, 0, st>>>(B);
  else if (align >= 4)
    k_ingest_batch<PL, 4, 0><<<grid, block, 0, st>>>(B);
  else
    k_ingest_batch<PL, 1, 0><<<grid, block, 0, st>>>(B);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !fin) return e;
  k_ingest_fin_batch<PL><<<dim3((unsigned)F.start[count]), 256, 0, st>>>(F);
  return hipGetLastError();
}

hipError_t launch_ingest_batch(const BatchItem* it, int count, int g_dtype, hipStream_t st) {
  if (count < 1 || count > MAX_BATCH) return hipErrorInvalidValue;
  switch (it[0].p->pL) {
    case 1:
      return ingest_batch_pl<1>(it, count, g_dtype, st);
    case 2:
      return ingest_batch_pl<2>(it, count, g_dtype, st);
    case 3:
      return ingest_batch_pl<3>(it, count, g_dtype, st);
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_ingest(const Plan& p, int64_t m_blk, const void* d_G, int g_dtype, int64_t ldg) {
  const int64_t m_pad = roundup(m_blk, SNP_PAD);
  switch (p.pL) {
#define CLAK_ID(PLV)                                          \
  case PLV:                                                   \
    ingest_dispatch<PLV>(p, m_blk, m_pad, d_G, g_dtype, ldg); \
    break;
    CLAK_ID(1) CLAK_ID(2) CLAK_ID(3) CLAK_ID(4) CLAK_ID(5) CLAK_ID(6) CLAK_ID(7) CLAK_ID(8)
    CLAK_ID(9) CLAK_ID(10) CLAK_ID(11) CLAK_ID(12) CLAK_ID(13) CLAK_ID(14) CLAK_ID(15) CLAK_ID(16)
#undef CLAK_ID
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace clak
