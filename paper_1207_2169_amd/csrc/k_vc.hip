// Variance components of the reduced model (the first step of the two-step
// analysis, supplementary notes, section 1; its cost is discussed with the
// parameter estimation in section 4): for each trait, y ~ N(X_L beta,
// s2 (h2 Phi + (1 - h2) I)).  With Phi = Z W Z^T, H = h2 Phi + (1 - h2) I has
// eigenvalues h2 w_k + 1 - h2, so for rotated data y~ = Z^T y, X~ = Z^T X_L and
// delta_k = 1 / (h2 w_k + 1 - h2) every profile quantity is a sum over k:
//   A = X~^T D X~,  b = X~^T D y~,  c = y~^T D y~,  log det H = -sum log delta_k,
//   RSS = c - b^T A^-1 b,  ML: s2 = RSS / n,  REML: s2 = RSS / (n - p),
//   ML  : l = -1/2 [n (log(2 pi s2) + 1) + log det H]
//   REML: l = -1/2 [(n - p)(log(2 pi s2) + 1) + log det H + log det A - log det(X^T X)].
// h2 maximises l over [0, 1]: the 101 points 0, 0.01, ..., 1, then a golden-
// section search on the bracket around the best of them (ties to the smaller
// h2) down to a width of 1e-7, keeping the better of its midpoint and the
// best grid point.  One work-group per trait, FP64 throughout.
#include "common.hpp"

namespace clak {

constexpr int VC_THREADS = 256, VC_CHUNK = 16, VC_GRID = 100;
constexpr double VC_TOL = 1e-7;

// Sum over the work-group of NV values per thread; every thread receives the sums.
template <int NV>
__device__ __forceinline__ void block_sum_vec(double (&v)[NV], double (*red)[NV]) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = wave_sum(v[q]);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NV; ++q) red[wid][q] = v[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double s = 0.0;
    for (int u = 0; u < VC_THREADS / 64; ++u) s += red[u][q];
    v[q] = s;
  }
  __syncthreads();
}

template <int REML>
__global__ void __launch_bounds__(VC_THREADS) k_vc(int64_t n, int64_t np, int pL, const double* __restrict__ w,
                                                   const double* __restrict__ XLt, const double* __restrict__ Yt,
                                                   double* __restrict__ h2o, double* __restrict__ s2o,
                                                   double* __restrict__ llo, int* __restrict__ dstat) {
  __shared__ double red[VC_THREADS / 64][VC_CHUNK];
  __shared__ double S[MAX_PL * MAX_PL];  // X~^T D X~ (upper), its Cholesky factor (lower, diagonal)
  __shared__ double bv[MAX_PL];          // X~^T D y~, then L^-1 of it
  __shared__ unsigned char pa[MAX_PL * (MAX_PL + 1) / 2], pb[MAX_PL * (MAX_PL + 1) / 2];
  __shared__ double cc, ldh, out_ll, out_s2, logdet_xx;
  __shared__ int bad;
  const int64_t j = blockIdx.x;
  const double* y = Yt + j * np;
  const int npair = pL * (pL + 1) / 2, nval = npair + pL + 2;  // A, b, c, log det H
  if (threadIdx.x == 0) {
    bad = 0;
    logdet_xx = 0.0;
    for (int a = 0, v = 0; a < pL; ++a)
      for (int b = a; b < pL; ++b, ++v) pa[v] = (unsigned char)a, pb[v] = (unsigned char)b;
  }
  __syncthreads();

  // Profile log-likelihood at h.  h < 0 stands for unit weights and only
  // records log det(X^T X) (= log det of X~^T X~, Z being orthogonal).
  auto eval = [&](double h) -> double {
    bool nonpos = false;
    for (int c0 = 0; c0 < nval; c0 += VC_CHUNK) {
      double acc[VC_CHUNK];
#pragma unroll
      for (int q = 0; q < VC_CHUNK; ++q) acc[q] = 0.0;
      for (int64_t k = threadIdx.x; k < n; k += VC_THREADS) {
        const double e = h < 0.0 ? 1.0 : h * w[k] + (1.0 - h);
        if (!(e > 0.0)) nonpos = true;
        const double d = 1.0 / e, yk = y[k];
#pragma unroll
        for (int q = 0; q < VC_CHUNK; ++q) {
          const int v = c0 + q;
          if (v < npair)
            acc[q] += XLt[k + pa[v] * np] * d * XLt[k + pb[v] * np];
          else if (v < npair + pL)
            acc[q] += XLt[k + (v - npair) * np] * d * yk;
          else if (v == npair + pL)
            acc[q] += yk * d * yk;
          else if (v == npair + pL + 1)
            acc[q] += log(e);
        }
      }
      block_sum_vec<VC_CHUNK>(acc, red);
      if (threadIdx.x == 0)
        for (int q = 0; q < VC_CHUNK && c0 + q < nval; ++q) {
          const int v = c0 + q;
          if (v < npair)
            S[pa[v] * MAX_PL + pb[v]] = acc[q];
          else if (v < npair + pL)
            bv[v - npair] = acc[q];
          else if (v == npair + pL)
            cc = acc[q];
          else
            ldh = acc[q];
        }
    }
    if (nonpos) atomicOr(&bad, 1);
    __syncthreads();
    if (threadIdx.x == 0) {
      // Cholesky of A (read from the upper triangle, factor written to the
      // lower one), log det A, then RSS = c - ||L^-1 b||^2.
      bool spd = !(bad & 1);
      double ldet = 0.0;
      for (int a = 0; a < pL && spd; ++a)
        for (int b = 0; b <= a; ++b) {
          double s = S[b * MAX_PL + a];
          for (int c = 0; c < b; ++c) s -= S[a * MAX_PL + c] * S[b * MAX_PL + c];
          if (a == b) {
            if (!(s > 0.0)) {
              spd = false;
              break;
            }
            ldet += log(s);
            S[a * MAX_PL + a] = sqrt(s);
          } else {
            S[a * MAX_PL + b] = s / S[b * MAX_PL + b];
          }
        }
      // the factor overwrote the diagonal of A; the next evaluation rebuilds A
      double ll = -INFINITY, s2 = NAN;
      if (spd && h < 0.0) {
        logdet_xx = ldet;
      } else if (spd) {
        double q2 = 0.0;
        for (int a = 0; a < pL; ++a) {
          double s = bv[a];
          for (int c = 0; c < a; ++c) s -= S[a * MAX_PL + c] * bv[c];
          bv[a] = s / S[a * MAX_PL + a];
          q2 += bv[a] * bv[a];
        }
        const double dof = REML ? (double)(n - pL) : (double)n;
        s2 = (cc - q2) / dof;
        if (s2 > 0.0) {
          ll = -0.5 * (dof * (log(2.0 * M_PI * s2) + 1.0) + ldh);
          if (REML) ll -= 0.5 * (ldet - logdet_xx);
        }
      } else if (!(bad & 1)) {
        bad |= 2;  // X~^T D X~ not positive definite: the covariates are (numerically) rank deficient
      }
      out_ll = ll;
      out_s2 = s2;
      bad &= ~1;  // a non-positive H only rules out this h
    }
    __syncthreads();
    return out_ll;
  };

  bool nonfin = false;
  for (int64_t k = threadIdx.x; k < n; k += VC_THREADS)
    if (!isfinite(y[k])) nonfin = true;
  if (nonfin) atomicOr(&bad, 4);
  __syncthreads();
  if (bad & 4) {
    if (threadIdx.x == 0) {
      atomicAdd(dstat + DS_TRAIT_ARG, 1);
      h2o[j] = s2o[j] = NAN;
      if (llo) llo[j] = NAN;
    }
    return;
  }
  if (REML) eval(-1.0);
  int best = 0;
  double lbest = -INFINITY;
  for (int i = 0; i <= VC_GRID; ++i) {
    const double l = eval((double)i / VC_GRID);
    if (l > lbest) lbest = l, best = i;
  }
  const double g = 0.5 * (sqrt(5.0) - 1.0);
  double a = (double)(best > 0 ? best - 1 : 0) / VC_GRID, b = (double)(best < VC_GRID ? best + 1 : VC_GRID) / VC_GRID;
  double c = b - g * (b - a), d = a + g * (b - a);
  double fc = eval(c), fd = eval(d);
  while (b - a > VC_TOL) {
    if (fc >= fd) {
      b = d;
      d = c;
      fd = fc;
      c = b - g * (b - a);
      fc = eval(c);
    } else {
      a = c;
      c = d;
      fc = fd;
      d = a + g * (b - a);
      fd = eval(d);
    }
  }
  const double x = 0.5 * (a + b);
  const double h2 = eval(x) > lbest ? x : (double)best / VC_GRID;
  const double ll = eval(h2);
  if (threadIdx.x == 0) {
    if (bad & 2) atomicAdd(dstat + DS_TRAIT_COV, 1);
    h2o[j] = h2;
    s2o[j] = out_s2;
    if (llo) llo[j] = ll;
  }
}

hipError_t launch_vc(const Plan& p, int method, double* h2, double* s2, double* ll) {
  const Workspace& W = p.ws;
  if (method == CLAK_VC_REML)
    k_vc<1><<<dim3((unsigned)p.t), VC_THREADS, 0, p.stream>>>(p.n, p.n_pad, (int)p.pL, W.w, W.XLt, W.Yt, h2, s2,
                                                              ll, W.dstat);
  else
    k_vc<0><<<dim3((unsigned)p.t), VC_THREADS, 0, p.stream>>>(p.n, p.n_pad, (int)p.pL, W.w, W.XLt, W.Yt, h2, s2,
                                                              ll, W.dstat);
  return hipGetLastError();
}

}  // namespace clak
