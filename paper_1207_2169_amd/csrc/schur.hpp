// Per-cell FP64 solve of the partitioned normal equations (supplementary
// notes, section 3, the multi-trait CLAK-Eig listing: S = [S_TL, *; W_R^T W_L,
// W_R^T W_R], b_ij = S^{-1} [b_T; W_R^T Y_j]), by block elimination on the
// whitened covariate block.  With S_TL = L L^T, for one (SNP, trait) cell:
//   c' = L^{-1} X~_L^T D x   (whitened cross terms, p_L values)
//   r' = x^T D e             (= W_R^T Y_j - c^T S_TL^{-1} b_T)
//   a  = x^T D x             (= W_R^T W_R)
//   s  = a - ||c'||^2        (Schur complement, = 1 / [S^{-1}]_pp)
//   b_snp = r' / s,  Var(b_snp) = 1 / s  (times s2_j under CLAK_VAR_PAPER);
//   one reciprocal 1 / s serves both (b_snp = r' (1 / s))
//   b_cov = u - L^{-T} c' b_snp - gamma b_snp   (gamma undoes the centring)
//   z = b_snp / SE, p = erfc(|z| / sqrt 2)     (optional)
#pragma once

#include "common.hpp"

namespace clak {

// The SNP-effect outputs of one cell: b_snp, SE, the two-sided p-value of the
// Wald statistic z = b_snp / SE (P(|N(0,1)| > |z|) = erfc(|z| / sqrt 2), the
// upper tail of chi-square with one degree of freedom at z^2), and the flag.
__device__ __forceinline__ void store_snp(const CellOut& out, int64_t o, double bsnp, double se, int flag,
                                          bool write_b) {
  if (out.f64) {
    if (write_b) ((double*)out.b)[o] = bsnp;
    ((double*)out.se)[o] = se;
  } else {
    if (write_b) ((float*)out.b)[o] = (float)bsnp;
    ((float*)out.se)[o] = (float)se;
  }
  if (out.pval) {
    const double pv = flag ? __builtin_nan("") : erfc(fabs(bsnp / se) * M_SQRT1_2);
    if (out.f64)
      ((double*)out.pval)[o] = pv;
    else
      ((float*)out.pval)[o] = (float)pv;
  }
  if (out.flags) out.flags[o] = (uint8_t)flag;
}

template <int PL>
__device__ __forceinline__ void schur_store(const double* c, double r, double a, const double* __restrict__ tp,
                                            const double* __restrict__ st, uint32_t flags, int64_t i, int64_t j,
                                            const CellOut& out) {
  const double nan = __builtin_nan("");
  int flag = (int)st[2 * PL + 1];
  double cc = 0.0;
#pragma unroll
  for (int l = 0; l < PL; ++l) cc += c[l] * c[l];
  const double s = a - cc;
  if (flag == 0 && !(s > 1e-10 * a)) flag = CLAK_CELL_DEGENERATE;
  double bsnp = nan, se = nan;
  if (flag == 0) {
    const double q = 1.0 / s;
    bsnp = r * q;
    se = sqrt((flags & CLAK_VAR_PAPER) ? tp[PL * PL + PL] * q : q);
  }
  const int64_t o = i + j * out.ldo;
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
    if (out.f64) {
#pragma unroll
      for (int q = 0; q <= PL; ++q) ((double*)out.b)[o * (PL + 1) + q] = bf[q];
    } else {
#pragma unroll
      for (int q = 0; q <= PL; ++q) ((float*)out.b)[o * (PL + 1) + q] = (float)bf[q];
    }
  }
  store_snp(out, o, bsnp, se, flag, !(flags & CLAK_OUT_FULL));
}

// The SNP-effect form of schur_store when ||c'||^2 has been accumulated in
// pieces (cc).
template <int PL>
__device__ __forceinline__ void schur_store_cc(double cc, double r, double a, const double* __restrict__ tp,
                                               const double* __restrict__ st, uint32_t flags, int64_t i, int64_t j,
                                               const CellOut& out) {
  int flag = (int)st[2 * PL + 1];
  const double s = a - cc;
  if (flag == 0 && !(s > 1e-10 * a)) flag = CLAK_CELL_DEGENERATE;
  double bsnp = __builtin_nan(""), se = __builtin_nan("");
  if (flag == 0) {
    const double q = 1.0 / s;
    bsnp = r * q;
    se = sqrt((flags & CLAK_VAR_PAPER) ? tp[PL * PL + PL] * q : q);
  }
  store_snp(out, i + j * out.ldo, bsnp, se, flag, true);
}


// One cell solved into registers (for kernels that stage their outputs
// before storing them): the same arithmetic as schur_store, given ||c'||^2
// (cc), r', a, the trait's parameters and the SNP's flag.
struct CellResult {
  double b, se, pv;
  int flag;
};

__device__ __forceinline__ CellResult cell_solve(double cc, double r, double a, double s2, int snp_flag,
                                                 uint32_t flags, bool want_p) {
  const double nan = __builtin_nan("");
  CellResult o;
  o.flag = snp_flag;
  const double s = a - cc;
  if (o.flag == 0 && !(s > 1e-10 * a)) o.flag = CLAK_CELL_DEGENERATE;
  o.b = nan;
  o.se = nan;
  o.pv = nan;
  if (o.flag == 0) {
    const double q = 1.0 / s;
    o.b = r * q;
    o.se = sqrt((flags & CLAK_VAR_PAPER) ? s2 * q : q);
    if (want_p) o.pv = erfc(fabs(o.b / o.se) * M_SQRT1_2);
  }
  return o;
}

}  // namespace clak
