// Per-cell FP64 solve of the partitioned normal equations (supplementary
// notes, section 3, the multi-trait CLAK-Eig listing: S = [S_TL, *; W_R^T W_L,
// W_R^T W_R], b_ij = S^{-1} [b_T; W_R^T Y_j]), by block elimination on the
// whitened covariate block.  With S_TL = L L^T, for one (SNP, trait) cell:
//   c' = L^{-1} X~_L^T D x   (whitened cross terms, p_L values)
//   r' = x^T D e             (= W_R^T Y_j - c^T S_TL^{-1} b_T)
//   a  = x^T D x             (= W_R^T W_R)
//   s  = a - ||c'||^2        (Schur complement, = 1 / [S^{-1}]_pp)
//   b_snp = r' / s,  Var(b_snp) = 1 / s  (times s2_j under CLAK_VAR_PAPER)
//   b_cov = u - L^{-T} c' b_snp - gamma b_snp   (gamma undoes the centring)
#pragma once

#include "common.cuh"

namespace clak {

template <int PL>
__device__ __forceinline__ void schur_store(const double* c, double r, double a, const double* __restrict__ tp,
                                            const double* __restrict__ st, uint32_t flags, int64_t i, int64_t j,
                                            void* __restrict__ ob, void* __restrict__ ose, int out_f64, int64_t ldo,
                                            uint8_t* __restrict__ oflags) {
  const double nan = __builtin_nan("");
  int flag = (int)st[2 * PL + 1];
  double cc = 0.0;
#pragma unroll
  for (int l = 0; l < PL; ++l) cc += c[l] * c[l];
  const double s = a - cc;
  if (flag == 0 && !(s > 1e-10 * a)) flag = CLAK_CELL_DEGENERATE;
  double bsnp = nan, se = nan;
  if (flag == 0) {
    bsnp = r / s;
    const double var = (flags & CLAK_VAR_PAPER) ? tp[PL * PL + PL] / s : 1.0 / s;
    se = sqrt(var);
  }
  const int64_t o = i + j * ldo;
  if (flags & CLAK_OUT_FULL) {
    double bf[PL + 1];
#pragma unroll
    for (int q = 0; q < PL; ++q) {
      double lc = 0.0;
#pragma unroll
      for (int l = 0; l < PL; ++l) lc += tp[l * PL + q] * c[l];  // (L^{-T} c')_q
      bf[q] = flag ? nan : tp[PL * PL + q] - (lc + st[PL + q]) * bsnp;
    }
    bf[PL] = bsnp;
    if (out_f64) {
#pragma unroll
      for (int q = 0; q <= PL; ++q) ((double*)ob)[o * (PL + 1) + q] = bf[q];
    } else {
#pragma unroll
      for (int q = 0; q <= PL; ++q) ((float*)ob)[o * (PL + 1) + q] = (float)bf[q];
    }
  } else {
    if (out_f64)
      ((double*)ob)[o] = bsnp;
    else
      ((float*)ob)[o] = (float)bsnp;
  }
  if (out_f64)
    ((double*)ose)[o] = se;
  else
    ((float*)ose)[o] = (float)se;
  if (oflags) oflags[o] = (uint8_t)flag;
}

// The SNP-effect form of schur_store when ||c'||^2 has been accumulated in
// pieces (cc): b_snp, SE and the flag of the cell.
template <int PL>
__device__ __forceinline__ void schur_store_cc(double cc, double r, double a, const double* __restrict__ tp,
                                               const double* __restrict__ st, uint32_t flags, int64_t i, int64_t j,
                                               void* __restrict__ ob, void* __restrict__ ose, int out_f64,
                                               int64_t ldo, uint8_t* __restrict__ oflags) {
  int flag = (int)st[2 * PL + 1];
  const double s = a - cc;
  if (flag == 0 && !(s > 1e-10 * a)) flag = CLAK_CELL_DEGENERATE;
  double bsnp = __builtin_nan(""), se = __builtin_nan("");
  if (flag == 0) {
    bsnp = r / s;
    se = sqrt((flags & CLAK_VAR_PAPER) ? tp[PL * PL + PL] / s : 1.0 / s);
  }
  const int64_t o = i + j * ldo;
  if (out_f64) {
    ((double*)ob)[o] = bsnp;
    ((double*)ose)[o] = se;
  } else {
    ((float*)ob)[o] = (float)bsnp;
    ((float*)ose)[o] = (float)se;
  }
  if (oflags) oflags[o] = (uint8_t)flag;
}

}  // namespace clak
