// Device helpers shared by the HIP translation units of libclak.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "clak_internal.hpp"

namespace clak {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Sum of v over the work-group, returned to every thread.  smem must hold
// blockDim.x / 64 doubles; contains two barriers.
__device__ __forceinline__ double block_sum(double v, double* smem) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) smem[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; ++i) s += smem[i];
  return s;
}

__device__ __forceinline__ double block_max(double v, double* smem) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_max(v);
  __syncthreads();
  if (lane == 0) smem[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; ++i) s = fmax(s, smem[i]);
  return s;
}

// Four base-256 digits of an integer |q| <= 127 * 2^24, most significant
// first: q = d0 * 2^24 + d1 * 2^16 + d2 * 2^8 + d3, d1..d3 in [-128, 127],
// |d0| <= 127.  Packed little-endian into the four bytes of the result in the
// order d0, d1, d2, d3.
__device__ __forceinline__ void digits4(int q, int8_t* d) {
  int l3 = ((q + 128) & 255) - 128;
  q = (q - l3) >> 8;
  int l2 = ((q + 128) & 255) - 128;
  q = (q - l2) >> 8;
  int l1 = ((q + 128) & 255) - 128;
  q = (q - l1) >> 8;
  d[0] = (int8_t)q;
  d[1] = (int8_t)l1;
  d[2] = (int8_t)l2;
  d[3] = (int8_t)l3;
}

// Offset of byte k of row `row` in a K-tiled digit plane of `rows` rows: the
// n_pad bytes of each row are cut into 32-byte slices and slice s of every row
// is stored contiguously (s * 32 rows + 32 row + k % 32), so one 32-deep stage
// of a tile of consecutive rows is a single contiguous run.
__host__ __device__ __forceinline__ int64_t kt32(int64_t row, int64_t k, int64_t rows) {
  return (k >> 5) * rows * 32 + row * 32 + (k & 31);
}

// Row of operand entry q of trait j in the per-trait operand planes: traits
// are grouped by 32 and, within a group, stored entry by entry, so the 32
// traits of a group have each entry in 32 consecutive rows.
__host__ __device__ __forceinline__ int64_t vrow(int64_t j, int64_t q, int64_t nent) {
  return (j >> 5) * 32 * nent + q * 32 + (j & 31);
}

// rint(v * inv_scale * QMAX) clamped to [-QMAX, QMAX].
__device__ __forceinline__ int quantize(double v, double inv_scale) {
  double q = rint(v * inv_scale * QMAX);
  q = fmin(fmax(q, -QMAX), QMAX);
  return (int)q;
}

}  // namespace clak
