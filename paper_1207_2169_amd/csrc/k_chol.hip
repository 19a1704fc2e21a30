// Set-up of the single-trait CLAK-Chol route (supplementary notes, section 2):
// M = s2 H with H = h2 Phi + (1 - h2) I = U^T U (upper Cholesky factor), so
// X^T M^{-1} X = (U^-T X)^T (U^-T X) / s2.  The per-block path is then the one
// of CLAK-Eig with U^-T in place of Z^T and unit weights w_k = 1 (every
// diagonal weight becomes 1 / s2).  U^-T is lower triangular: row k of the
// rotation has nonzeros in columns 0..k only.
//
// Layout: the rotation matrix is kept as Z^T rows, i.e. the column-major
// n_pad x n_pad array whose column k is row k of the rotation.  The column-
// major upper-triangular U^-1 written by the triangular inversion is exactly
// that array for U^-T once its strictly lower part (left over from H) and the
// padding are cleared.
#include "common.hpp"

namespace clak {

// Phi must be finite in its lower triangle (the part that is read).
__global__ void __launch_bounds__(256) k_chol_check(int64_t n, int64_t np, const double* __restrict__ Phi,
                                                    int* dstat) {
  const int64_t c = blockIdx.x;
  bool bad = false;
  for (int64_t r = c + threadIdx.x; r < n; r += 256)
    if (!isfinite(Phi[c * np + r])) bad = true;
  if (bad) atomicAdd(dstat + DS_EIGVAL, 1);
}

// H = h2 Phi + (1 - h2) I, full symmetric from the lower triangle of Phi,
// zero in the padding.  An h2 outside [0, 1] (or NaN) counts as a bad trait
// argument and leaves H untouched.
__global__ void __launch_bounds__(256) k_chol_build(int64_t n, int64_t np, const double* __restrict__ Phi,
                                                    const double* __restrict__ h2p, double* __restrict__ H,
                                                    int* dstat) {
  const double h2 = *h2p;
  if (!(h2 >= 0.0 && h2 <= 1.0)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(dstat + DS_TRAIT_ARG, 1);
    return;
  }
  const int64_t c = blockIdx.x;
  for (int64_t r = threadIdx.x; r < np; r += 256) {
    double v = 0.0;
    if (r < n && c < n) {
      const double phi = r >= c ? Phi[c * np + r] : Phi[r * np + c];
      v = h2 * phi + (r == c ? 1.0 - h2 : 0.0);
    }
    H[c * np + r] = v;
  }
}

// After the factorisation and the triangular inversion (upper, in place):
// clear the strictly lower part and the padding, unit weights for k < n.
__global__ void __launch_bounds__(256) k_chol_fix(int64_t n, int64_t np, double* __restrict__ Zt,
                                                  double* __restrict__ w) {
  const int64_t c = blockIdx.x;
  for (int64_t r = threadIdx.x; r < np; r += 256)
    if (r > c || r >= n || c >= n) Zt[c * np + r] = 0.0;
  if (threadIdx.x == 0) w[c] = c < n ? 1.0 : 0.0;
}

hipError_t launch_chol_check(const Plan& p) {
  k_chol_check<<<dim3((unsigned)p.n), 256, 0, p.stream>>>(p.n, p.n_pad, p.ws.Phi, p.ws.dstat);
  return hipGetLastError();
}

hipError_t launch_chol_build(const Plan& p, const double* d_h2) {
  k_chol_build<<<dim3((unsigned)p.n_pad), 256, 0, p.stream>>>(p.n, p.n_pad, p.ws.Phi, d_h2, p.ws.Zt, p.ws.dstat);
  return hipGetLastError();
}

hipError_t launch_chol_fix(const Plan& p) {
  k_chol_fix<<<dim3((unsigned)p.n_pad), 256, 0, p.stream>>>(p.n, p.n_pad, p.ws.Zt, p.ws.w);
  return hipGetLastError();
}

}  // namespace clak
