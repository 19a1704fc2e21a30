// Set-up kernels of the CLAK-Eig path, run once per cohort (kinship,
// covariates) or once per set of traits: eigenpair validation, the int8 digit
// planes of Z^T, the orthonormal basis of X_L, and the per-trait quantities of
// the loop over traits in the multi-trait CLAK-Eig listing (D, S_TL, b_T and
// the operand of the grid contraction).
#include "common.hpp"

namespace clak {

// ---------------------------------------------------------------- eigenpairs

__global__ void k_check_eigen(int64_t n, int64_t np, const double* __restrict__ Zt, const double* __restrict__ w,
                              int* dstat) {
  const int64_t k = blockIdx.x;
  bool bad = false;
  if (threadIdx.x == 0 && !isfinite(w[k])) bad = true;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x)
    if (!isfinite(Zt[k * np + i])) bad = true;
  if (bad) atomicAdd(dstat + DS_EIGVAL, 1);
}

hipError_t launch_check_eigen(const Plan& p) {
  k_check_eigen<<<dim3((unsigned)p.n), dim3(256), 0, p.stream>>>(p.n, p.n_pad, p.ws.Zt, p.ws.w, p.ws.dstat);
  return hipGetLastError();
}

// Row k of Z^T (eigenvector k) is stored as four int8 planes with one scale
// per row: Z^T[k][i] ~= zs[k] * sum_p Zd[p][k][i] * 256^(3-p), zs[k] =
// max_i |Z^T[k][i]| / QMAX.  Rounding error <= 0.5 zs[k] per entry.
// Rows r0 + blockIdx.x of a layout of zr rows.  Rows below n and from zl on
// (the U^T rows of a single-trait mixed plan) carry data, the rows between are
// zero padding, and every row is zero beyond n.
__global__ void k_split_digits(int64_t n, int64_t np, int64_t zr, int64_t zl, int64_t r0,
                               const double* __restrict__ Zt, int8_t* __restrict__ Zd, double* __restrict__ zs) {
  __shared__ double red[16];
  const int64_t k = r0 + blockIdx.x;
  const bool live = k < n || k >= zl;
  const double* row = Zt + k * np;
  double mx = 0.0;
  if (live)
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) mx = fmax(mx, fabs(row[i]));
  mx = block_max(mx, red);
  const double inv = mx > 0.0 ? 1.0 / mx : 0.0;
  const int64_t plane = zr * np;
  for (int64_t i = threadIdx.x; i < np; i += blockDim.x) {
    int8_t d[4] = {0, 0, 0, 0};
    if (live && i < n) digits4(quantize(row[i], inv), d);
#pragma unroll
    for (int q = 0; q < 4; ++q) Zd[q * plane + kt32(k, i, zr)] = d[q];
  }
  if (threadIdx.x == 0) zs[k] = mx / QMAX;
}

// Replaces rows [r0, r1) of the rotation operand by the values their digit
// planes encode (zs[k] * sum_p d_p 256^(3-p)).  Used for the single-trait
// rows U^T: C = Q_L^T U is then formed from the matrix the int8 rotation
// multiplies by, so the centring of those rows cancels their digit rounding.
__global__ void k_dequant_rows(int64_t np, int64_t zr, int64_t r0, const int8_t* __restrict__ Zd,
                               const double* __restrict__ zs, double* __restrict__ Zt) {
  const int64_t k = r0 + blockIdx.x;
  const int64_t plane = zr * np;
  const double sc = zs[k];
  for (int64_t i = threadIdx.x; i < np; i += blockDim.x) {
    const int64_t o = kt32(k, i, zr);
    const int q = (((int)Zd[o] * 256 + (int)Zd[plane + o]) * 256 + (int)Zd[2 * plane + o]) * 256 +
                  (int)Zd[3 * plane + o];
    Zt[k * np + i] = sc * (double)q;
  }
}

// The centring rotation of the mixed path, Qt = Z_q^T Q_L with Z_q the values
// the digit planes of Z^T encode (one work-group per row k; FP64).  A rotated
// SNP is x~ = Z_q^T g - Qt v: with the same Z_q on both sides, the centring
// cancels the digit rounding of Z_q^T g up to FP64 rounding, so the error of
// x~ is relative to the centred SNP g - Q_L v, not to g (which matters for
// SNPs close to span(X_L)).  X_L, Y and everything else are rotated by the
// FP64 Z; the two differ by the digit rounding, about 2^-31 of each row.
template <int PL>
__global__ void __launch_bounds__(256) k_qt_digits(int64_t n, int64_t np, int64_t zr, const int8_t* __restrict__ Zd,
                                                   const double* __restrict__ zs, const double* __restrict__ QL,
                                                   double* __restrict__ Qt) {
  __shared__ double red[8];
  const int64_t k = blockIdx.x;
  const int64_t plane = zr * np;
  double acc[PL];
#pragma unroll
  for (int a = 0; a < PL; ++a) acc[a] = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const int64_t o = kt32(k, i, zr);
    const double z = (double)((((int)Zd[o] * 256 + (int)Zd[plane + o]) * 256 + (int)Zd[2 * plane + o]) * 256 +
                              (int)Zd[3 * plane + o]);
#pragma unroll
    for (int a = 0; a < PL; ++a) acc[a] += z * QL[i + a * np];
  }
  const double sc = zs[k];
#pragma unroll
  for (int a = 0; a < PL; ++a) {
    const double v = block_sum(acc[a], red);
    if (threadIdx.x == 0) Qt[k + a * np] = sc * v;
  }
}

hipError_t launch_qt_digits(const Plan& p) {
  const Workspace& W = p.ws;
  const dim3 grid((unsigned)p.n_pad);
  switch (p.pL) {
#define CLAK_QT(PLV)                                                                                          \
  case PLV:                                                                                                   \
    k_qt_digits<PLV><<<grid, 256, 0, p.stream>>>(p.n, p.n_pad, p.zrows, W.Zd, W.zs, W.QL, W.Qt); \
    break;
    CLAK_QT(1) CLAK_QT(2) CLAK_QT(3) CLAK_QT(4) CLAK_QT(5) CLAK_QT(6) CLAK_QT(7) CLAK_QT(8)
#undef CLAK_QT
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_dequant_rows(const Plan& p, int64_t r0, int64_t r1) {
  if (r1 <= r0) return hipSuccess;
  k_dequant_rows<<<dim3((unsigned)(r1 - r0)), dim3(256), 0, p.stream>>>(p.n_pad, p.zrows, r0, p.ws.Zd, p.ws.zs,
                                                                          p.ws.Zt);
  return hipGetLastError();
}

hipError_t launch_split_digits(const Plan& p, int64_t r0, int64_t r1) {
  if (r1 <= r0) return hipSuccess;
  k_split_digits<<<dim3((unsigned)(r1 - r0)), dim3(256), 0, p.stream>>>(p.n, p.n_pad, p.zrows, p.zlin, r0, p.ws.Zt,
                                                                          p.ws.Zd, p.ws.zs);
  return hipGetLastError();
}

// ---------------------------------------------------------------- covariates

// X_L = Q_L R by classical Gram-Schmidt applied twice per column, FP64, one
// work-group.  Q_L (n_pad x pL, zero padded) spans the covariates; it is the
// basis against which every SNP is centred before the rotation.
__global__ void __launch_bounds__(1024) k_covariates(int64_t n, int64_t np, int pL, const double* __restrict__ XL,
                                                     int64_t ld, double* __restrict__ QL, double* __restrict__ Rm,
                                                     double* __restrict__ Rinv, int* dstat) {
  __shared__ double red[16];
  __shared__ double R[MAX_PL * MAX_PL];
  __shared__ double coef[MAX_PL];
  __shared__ int flag;
  if (threadIdx.x == 0) flag = 0;
  for (int i = threadIdx.x; i < MAX_PL * MAX_PL; i += blockDim.x) R[i] = 0.0;
  __syncthreads();
  for (int l = 0; l < pL; ++l)
    for (int64_t i = threadIdx.x; i < np; i += blockDim.x) {
      double v = i < n ? XL[i + l * ld] : 0.0;
      if (!isfinite(v)) flag = 1;
      QL[i + l * np] = v;
    }
  __syncthreads();
  if (flag) {
    if (threadIdx.x == 0) dstat[DS_COV] = 1;
    return;
  }
  for (int l = 0; l < pL; ++l) {
    double* ql = QL + l * np;
    double nrm0 = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) nrm0 += ql[i] * ql[i];
    nrm0 = block_sum(nrm0, red);
    for (int pass = 0; pass < 2; ++pass) {
      for (int a = 0; a < l; ++a) {
        double s = 0.0;
        for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += QL[i + a * np] * ql[i];
        s = block_sum(s, red);
        if (threadIdx.x == 0) coef[a] = s;
      }
      __syncthreads();
      for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        double v = ql[i];
        for (int a = 0; a < l; ++a) v -= coef[a] * QL[i + a * np];
        ql[i] = v;
      }
      if (threadIdx.x == 0)
        for (int a = 0; a < l; ++a) R[a * MAX_PL + l] += coef[a];
      __syncthreads();
    }
    double nrm = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) nrm += ql[i] * ql[i];
    nrm = block_sum(nrm, red);
    if (!(nrm > 1e-20 * nrm0) || !(nrm0 > 0.0)) {
      if (threadIdx.x == 0) dstat[DS_COV] = 2;
      return;
    }
    nrm = sqrt(nrm);
    if (threadIdx.x == 0) R[l * MAX_PL + l] = nrm;
    const double inv = 1.0 / nrm;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) ql[i] *= inv;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    // R^{-1} of the upper-triangular R, column by column (back substitution)
    double Ri[MAX_PL * MAX_PL];
    for (int c = 0; c < pL; ++c)
      for (int r = pL - 1; r >= 0; --r) {
        double s = (r == c) ? 1.0 : 0.0;
        for (int k = r + 1; k < pL; ++k) s -= R[r * MAX_PL + k] * Ri[k * MAX_PL + c];
        Ri[r * MAX_PL + c] = s / R[r * MAX_PL + r];
      }
    for (int r = 0; r < pL; ++r)
      for (int c = 0; c < pL; ++c) {
        Rm[r * pL + c] = R[r * MAX_PL + c];
        Rinv[r * pL + c] = (c >= r) ? Ri[r * MAX_PL + c] : 0.0;
      }
  }
}

hipError_t launch_covariates(const Plan& p, const double* d_XL, int64_t ld) {
  k_covariates<<<1, 1024, 0, p.stream>>>(p.n, p.n_pad, (int)p.pL, d_XL, ld, p.ws.QL, p.ws.Rm, p.ws.Rinv,
                                          p.ws.dstat);
  return hipGetLastError();
}

// ---------------------------------------------------------------- traits

// Everything the loop over traits of the multi-trait CLAK-Eig listing computes
// once per trait, FP64, one work-group per trait j:
//   d_k    = 1 / (s2_j (h2_j w_k + 1 - h2_j))          (the diagonal D_j)
//   S_TL   = X~_L^T D_j X~_L,  b_T = X~_L^T D_j y~_j,  S_TL = L L^T
//   u      = S_TL^{-1} b_T,    e = y~_j - X~_L u
// and the per-trait operand of the grid contraction, one column per entry:
//   column l < pL : D_j X~_L L^{-T}   (whitened covariates)
//   column pL     : D_j e             (weighted residual)
//   D column      : d
// so that for a rotated SNP x the cell sums are c' = (D X~_L L^{-T})^T x,
// r' = (D e)^T x and a = d^T (x o x).
template <bool MIXED>
__global__ void __launch_bounds__(256) k_traits(int64_t n, int64_t np, int pL, int64_t t, int64_t tp,
                                                const double* __restrict__ w, const double* __restrict__ XLt,
                                                const double* __restrict__ Yt, double* __restrict__ tpar,
                                                double* __restrict__ V64, double* __restrict__ D64,
                                                int8_t* __restrict__ Vd, int8_t* __restrict__ Dd,
                                                double* __restrict__ vs, double* __restrict__ ds, int* dstat) {
  __shared__ double red[8];
  __shared__ double S[MAX_PL * MAX_PL];
  __shared__ double bT[MAX_PL];
  __shared__ double Li[MAX_PL * MAX_PL];
  __shared__ double u[MAX_PL];
  __shared__ double cmax[MAX_PL + 2];
  __shared__ int fl;
  const int64_t j = blockIdx.x;
  const int ncol = pL + 1;
  const int64_t ts = trait_stride(pL);
  const int64_t vplane = tp * ncol * np, dplane = tp * np;

  auto zero_fill = [&]() {
    for (int64_t k = threadIdx.x; k < np; k += blockDim.x) {
      for (int l = 0; l < ncol; ++l) {
        if (Vd)
          for (int q = 0; q < 4; ++q) Vd[q * vplane + kt32(vrow(j, l, ncol), k, tp * ncol)] = 0;
        if (V64) V64[(j * ncol + l) * np + k] = 0.0;
      }
      if (Dd)
        for (int q = 0; q < 4; ++q) Dd[q * dplane + kt32(j, k, tp)] = 0;
      if (D64) D64[j * np + k] = 0.0;
    }
    if (threadIdx.x == 0) {
      if (vs) {
        for (int l = 0; l < ncol; ++l) vs[j * ncol + l] = 0.0;
        ds[j] = 0.0;
      }
      for (int64_t q = 0; q < ts - 2; ++q) tpar[j * ts + q] = 0.0;
    }
  };

  if (j >= t) {
    zero_fill();
    return;
  }
  const double s2 = tpar[j * ts + pL * pL + pL];
  const double h2 = tpar[j * ts + pL * pL + pL + 1];
  if (threadIdx.x == 0) fl = 0;
  __syncthreads();
  if (!(h2 >= 0.0 && h2 <= 1.0) || !(s2 > 0.0) || !isfinite(s2)) {
    if (threadIdx.x == 0) atomicAdd(dstat + DS_TRAIT_ARG, 1);
    zero_fill();
    return;
  }
  const double* y = Yt + j * np;
  // S_TL (upper triangle) and b_T, in chunks of 16 values
  const int npair = pL * (pL + 1) / 2, nval = npair + pL;
  bool nspd = false, nonfin = false;
  for (int c0 = 0; c0 < nval; c0 += 16) {
    double acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.0;
    for (int64_t k = threadIdx.x; k < n; k += blockDim.x) {
      const double del = h2 * w[k] + (1.0 - h2);
      if (!(del > 0.0)) nspd = true;
      const double d = 1.0 / (s2 * del);
      if (!isfinite(y[k])) nonfin = true;
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int v = c0 + q;
        if (v < npair) {
          // v -> (a, b), a <= b, row-major upper triangle
          int a = 0, rem = v;
          while (rem >= pL - a) {
            rem -= pL - a;
            ++a;
          }
          const int b = a + rem;
          acc[q] += XLt[k + a * np] * d * XLt[k + b * np];
        } else if (v < nval) {
          acc[q] += XLt[k + (v - npair) * np] * d * y[k];
        }
      }
    }
    for (int q = 0; q < 16 && c0 + q < nval; ++q) {
      const double s = block_sum(acc[q], red);
      const int v = c0 + q;
      if (threadIdx.x == 0) {
        if (v < npair) {
          int a = 0, rem = v;
          while (rem >= pL - a) {
            rem -= pL - a;
            ++a;
          }
          S[a * MAX_PL + a + rem] = s;
          S[(a + rem) * MAX_PL + a] = s;
        } else {
          bT[v - npair] = s;
        }
      }
    }
  }
  if (nspd) atomicOr(&fl, 1);
  if (nonfin) atomicOr(&fl, 4);
  __syncthreads();
  if (threadIdx.x == 0 && fl == 0) {
    // Cholesky S_TL = L L^T (row-major lower in Li first, then inverted)
    double L[MAX_PL * MAX_PL];
    for (int a = 0; a < pL; ++a)
      for (int b = 0; b <= a; ++b) {
        double s = S[a * MAX_PL + b];
        for (int k = 0; k < b; ++k) s -= L[a * MAX_PL + k] * L[b * MAX_PL + k];
        if (a == b) {
          if (!(s > 1e-13 * S[a * MAX_PL + a])) {
            fl |= 2;
            s = 1.0;
          }
          L[a * MAX_PL + a] = sqrt(s);
        } else {
          L[a * MAX_PL + b] = s / L[b * MAX_PL + b];
        }
      }
    // L^{-1} (lower) by forward substitution on the identity
    for (int c = 0; c < pL; ++c)
      for (int r = 0; r < pL; ++r) {
        double s = (r == c) ? 1.0 : 0.0;
        for (int k = c; k < r; ++k) s -= L[r * MAX_PL + k] * Li[k * MAX_PL + c];
        Li[r * MAX_PL + c] = (r >= c) ? s / L[r * MAX_PL + r] : 0.0;
      }
    // u = L^{-T} L^{-1} b_T
    double z[MAX_PL];
    for (int r = 0; r < pL; ++r) {
      double s = 0.0;
      for (int k = 0; k <= r; ++k) s += Li[r * MAX_PL + k] * bT[k];
      z[r] = s;
    }
    for (int r = 0; r < pL; ++r) {
      double s = 0.0;
      for (int k = r; k < pL; ++k) s += Li[k * MAX_PL + r] * z[k];
      u[r] = s;
    }
    for (int r = 0; r < pL; ++r) {
      for (int c = 0; c < pL; ++c) tpar[j * ts + r * pL + c] = Li[r * MAX_PL + c];
      tpar[j * ts + pL * pL + r] = u[r];
    }
  }
  __syncthreads();
  if (fl) {
    if (threadIdx.x == 0) {
      if (fl & 4) atomicAdd(dstat + DS_TRAIT_ARG, 1);
      else if (fl & 1) atomicAdd(dstat + DS_TRAIT_SPD, 1);
      else atomicAdd(dstat + DS_TRAIT_COV, 1);
    }
    zero_fill();
    return;
  }

  // the operand columns at row k: out[0..pL) whitened covariates, out[pL]
  // weighted residual, out[pL+1] = d
  auto column_values = [&](int64_t k, double* out) {
    if (k >= n) {
      for (int l = 0; l < pL + 2; ++l) out[l] = 0.0;
      return;
    }
    const double d = 1.0 / (s2 * (h2 * w[k] + (1.0 - h2)));
    double xl[MAX_PL];
    double e = y[k];
    for (int a = 0; a < pL; ++a) {
      xl[a] = XLt[k + a * np];
      e -= xl[a] * u[a];
    }
    for (int l = 0; l < pL; ++l) {
      double s = 0.0;
      for (int a = 0; a <= l; ++a) s += xl[a] * Li[l * MAX_PL + a];
      out[l] = d * s;
    }
    out[pL] = d * e;
    out[pL + 1] = d;
  };

  if (!MIXED) {
    for (int64_t k = threadIdx.x; k < np; k += blockDim.x) {
      double v[MAX_PL + 2];
      column_values(k, v);
      for (int l = 0; l < ncol; ++l) V64[(j * ncol + l) * np + k] = v[l];
      D64[j * np + k] = v[ncol];
    }
  } else if (Vd) {
    // column maxima, then the digit planes of every column
    for (int l = 0; l < ncol + 1; ++l) {
      double mx = 0.0;
      for (int64_t k = threadIdx.x; k < n; k += blockDim.x) {
        double v[MAX_PL + 2];
        column_values(k, v);
        mx = fmax(mx, fabs(v[l]));
      }
      mx = block_max(mx, red);
      if (threadIdx.x == 0) cmax[l] = mx;
    }
    __syncthreads();
    for (int64_t k = threadIdx.x; k < np; k += blockDim.x) {
      double v[MAX_PL + 2];
      column_values(k, v);
      for (int l = 0; l < ncol + 1; ++l) {
        int8_t d[4];
        const double inv = cmax[l] > 0.0 ? 1.0 / cmax[l] : 0.0;
        digits4(quantize(v[l], inv), d);
        for (int q = 0; q < 4; ++q) {
          if (l < ncol)
            Vd[q * vplane + kt32(vrow(j, l, ncol), k, tp * ncol)] = d[q];
          else
            Dd[q * dplane + kt32(j, k, tp)] = d[q];
        }
      }
    }
    if (threadIdx.x == 0) {
      for (int l = 0; l < ncol; ++l) vs[j * ncol + l] = cmax[l] / QMAX;
      ds[j] = cmax[ncol] / QMAX;
    }
  }
  if (MIXED && V64) {  // FP64 copy for the fused single-trait kernel
    for (int64_t k = threadIdx.x; k < np; k += blockDim.x) {
      double v[MAX_PL + 2];
      column_values(k, v);
      for (int l = 0; l < ncol; ++l) V64[(j * ncol + l) * np + k] = v[l];
      D64[j * np + k] = v[ncol];
    }
  }
}

// Single trait, mixed path: the trait operand carried back to the genotype
// side.  The rotation forms x~ = Z^T (g - Q_L v) (Z^T: the rows of Zt, the
// eigenvectors, or U^-T under CLAK-Chol); the linear cell sums of section 3's
// inner loop, W^T x~ for the p_L + 1 operand columns W of the trait (c' and r'),
// equal U^T (g - Q_L v) with U = Z W.  The columns of U become rows zl + q of
// Zt, so the rotation yields them too, centred by C = Q_L^T U.
// k_uproj: one thread per individual i, U[i][q] summed over the n eigen rows
// in order (W is zero beyond n); rows zl + q for q > p_L up to zr are zero.
__global__ void __launch_bounds__(256) k_uproj(int64_t n, int64_t np, int64_t zl, int64_t zr, int ncol,
                                               const double* __restrict__ V64, double* __restrict__ Zt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  for (int64_t q = 0; q < zr - zl; ++q) {
    double acc = 0.0;
    if (q < ncol && i < n) {
      const double* wq = V64 + q * np;
      for (int64_t k = 0; k < n; ++k) acc += Zt[k * np + i] * wq[k];
    }
    Zt[(zl + q) * np + i] = acc;
  }
}

// C[a][q] = sum_i Q_L[i][a] U[i][q], one thread per entry.
__global__ void __launch_bounds__(256) k_cproj(int64_t np, int64_t zl, int pL, const double* __restrict__ QL,
                                               const double* __restrict__ Zt, double* __restrict__ Cq) {
  const int ncol = pL + 1;
  for (int e = threadIdx.x; e < pL * ncol; e += blockDim.x) {
    const int a = e / ncol, q = e % ncol;
    const double* u = Zt + (zl + q) * np;
    double acc = 0.0;
    for (int64_t i = 0; i < np; ++i) acc += QL[i + a * np] * u[i];
    Cq[e] = acc;
  }
}

// U = Z W into rows zlin .. of Z^T, their digit planes, the rows replaced by
// the values the digits encode, then C = Q_L^T U of those values.
hipError_t launch_uproj(const Plan& p) {
  const Workspace& W = p.ws;
  k_uproj<<<dim3((unsigned)((p.n_pad + 255) / 256)), 256, 0, p.stream>>>(p.n, p.n_pad, p.zlin, p.zrows,
                                                                         (int)p.pL + 1, W.V64, W.Zt);
  hipError_t e = launch_split_digits(p, p.zlin, p.zrows);
  if (e == hipSuccess) e = launch_dequant_rows(p, p.zlin, p.zrows);
  if (e != hipSuccess) return e;
  k_cproj<<<1, 256, 0, p.stream>>>(p.n_pad, p.zlin, (int)p.pL, W.QL, W.Zt, W.Cq);
  return hipGetLastError();
}

hipError_t launch_traits(const Plan& p) {
  const Workspace& W = p.ws;
  if (p.prec == CLAK_PREC_MIXED)
    k_traits<true><<<dim3((unsigned)p.t_pad), 256, 0, p.stream>>>(p.n, p.n_pad, (int)p.pL, p.t, p.t_pad, W.w, W.XLt,
                                                                  W.Yt, W.tpar, W.V64, W.D64, W.Vd, W.Dd, W.vs,
                                                                  W.ds, W.dstat);
  else
    k_traits<false><<<dim3((unsigned)p.t_pad), 256, 0, p.stream>>>(p.n, p.n_pad, (int)p.pL, p.t, p.t_pad, W.w,
                                                                   W.XLt, W.Yt, W.tpar, W.V64, W.D64, nullptr,
                                                                   nullptr, nullptr, nullptr, W.dstat);
  return hipGetLastError();
}

}  // namespace clak
