// SNP block ingest: moves a caller block of genotypes into the padded int8
// staging panel of the plan and computes, per SNP, the FP64 statistics of its
// centring against the covariates (projection onto Q_L, residual norm,
// degeneracy flag).
#include <hip/hip_fp16.h>

#include "common.cuh"

namespace clak {

// One wave per SPW SNPs; lanes stride over the individuals.  Per SNP g:
//   v = Q_L^T g, gg = g^T g, res = gg - ||v||^2 = ||g - Q_L v||^2,
//   flag = 2 if a genotype is not in {0, 1, 2}; 1 if g lies in span(X_L)
//   (gg == 0 or res <= 1e-10 gg); else 0.
// SNP rows in [m_blk, m_pad) are written as zero SNPs with flag 1.
template <int PLMAX, int SPW, bool F16>
__global__ void __launch_bounds__(256) k_ingest(int64_t n, int64_t np, int pL, int64_t m_blk, int64_t m_pad,
                                                const void* __restrict__ G, int64_t ldg,
                                                const double* __restrict__ QL, const double* __restrict__ Rinv,
                                                int8_t* __restrict__ Gp, double* __restrict__ sstat) {
  const int lane = threadIdx.x & 63;
  const int64_t snp0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * SPW;
  if (snp0 >= m_pad) return;
  double acc[SPW][PLMAX];
  double gg[SPW];
  int bad[SPW];
#pragma unroll
  for (int s = 0; s < SPW; ++s) {
    gg[s] = 0.0;
    bad[s] = 0;
#pragma unroll
    for (int a = 0; a < PLMAX; ++a) acc[s][a] = 0.0;
  }
  for (int64_t i = lane; i < np; i += 64) {
    double q[PLMAX];
#pragma unroll
    for (int a = 0; a < PLMAX; ++a) q[a] = (a < pL) ? QL[i + a * np] : 0.0;
#pragma unroll
    for (int s = 0; s < SPW; ++s) {
      const int64_t snp = snp0 + s;
      if (snp >= m_pad) break;
      int g = 0;
      if (snp < m_blk && i < n) {
        if (F16) {
          const float f = __half2float(((const __half*)G)[snp * ldg + i]);
          g = (int)f;
          if (!(f == 0.0f || f == 1.0f || f == 2.0f)) bad[s] = 1;
        } else {
          g = ((const uint8_t*)G)[snp * ldg + i];
          if (g > 2) bad[s] = 1;
        }
        if (bad[s]) g = 0;
      }
      Gp[snp * np + i] = (int8_t)g;
      const double gd = (double)g;
      gg[s] += gd * gd;
#pragma unroll
      for (int a = 0; a < PLMAX; ++a) acc[s][a] += q[a] * gd;
    }
  }
  const int64_t ss = snp_stride(pL);
#pragma unroll
  for (int s = 0; s < SPW; ++s) {
    const int64_t snp = snp0 + s;
    double v[PLMAX];
#pragma unroll
    for (int a = 0; a < PLMAX; ++a) v[a] = wave_sum(acc[s][a]);
    const double g2 = wave_sum(gg[s]);
    int b = bad[s];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) b |= __shfl_xor(b, o, 64);
    if (lane == 0 && snp < m_pad) {
      double vv = 0.0;
      for (int a = 0; a < pL; ++a) vv += v[a] * v[a];
      const double res = g2 - vv;
      int flag = b ? 2 : ((snp >= m_blk || !(g2 > 0.0) || !(res > 1e-10 * g2)) ? 1 : 0);
      double* st = sstat + snp * ss;
      for (int a = 0; a < pL; ++a) {
        double gam = 0.0;
        for (int c = a; c < pL; ++c) gam += Rinv[a * pL + c] * v[c];
        st[a] = flag ? 0.0 : v[a];
        st[pL + a] = flag ? 0.0 : gam;
      }
      st[2 * pL] = flag ? 1.0 : sqrt(res);
      st[2 * pL + 1] = (double)flag;
      st[2 * pL + 2] = 0.0;
    }
  }
}

hipError_t launch_ingest(const Plan& p, int64_t m_blk, const void* d_G, int g_dtype, int64_t ldg) {
  const int64_t m_pad = roundup(m_blk, SNP_PAD);
  const int pL = (int)p.pL;
  const bool f16 = g_dtype == CLAK_G_F16;
#define CLAK_INGEST(PLM, SPW)                                                                                 \
  do {                                                                                                        \
    const int64_t per_block = 4 * SPW;                                                                        \
    dim3 grid((unsigned)((m_pad + per_block - 1) / per_block));                                               \
    if (f16)                                                                                                  \
      k_ingest<PLM, SPW, true><<<grid, 256, 0, p.stream>>>(p.n, p.n_pad, pL, m_blk, m_pad, d_G, ldg, p.ws.QL, \
                                                           p.ws.Rinv, p.ws.Gp, p.ws.sstat);                   \
    else                                                                                                      \
      k_ingest<PLM, SPW, false><<<grid, 256, 0, p.stream>>>(p.n, p.n_pad, pL, m_blk, m_pad, d_G, ldg,         \
                                                            p.ws.QL, p.ws.Rinv, p.ws.Gp, p.ws.sstat);         \
  } while (0)
  if (pL <= 4)
    CLAK_INGEST(4, 8);
  else if (pL <= 8)
    CLAK_INGEST(8, 4);
  else
    CLAK_INGEST(16, 2);
#undef CLAK_INGEST
  return hipGetLastError();
}

}  // namespace clak
