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

// v_mfma_i32_32x32x32_i8 lane layout (gfx950): lane l supplies 16 bytes of row
// l%32 of A and of column l%32 of B, the same 16 values of the 32-deep
// contraction (half l/32); result register r holds C[8(r/4) + 4(l/32) + r%4][l%32].
__device__ __forceinline__ v16i mfma32_i8(v4i a, v4i b, v16i c) {
  return __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0);
}

// Encoded s_waitcnt immediate that waits until at most N vector memory
// operations of the wave are outstanding (expcnt and lgkmcnt not waited on).
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

typedef __attribute__((address_space(3))) void* lds_ptr_t;

// Work-group barrier for the direct-load ring: the wave's LDS reads complete
// (lgkmcnt 0), then s_barrier.  Unlike __syncthreads it does not wait for
// the wave's outstanding global-to-LDS loads; the caller waits for the ones
// it needs (wait_vm) before the barrier.  The memory clobbers keep the
// compiler from moving memory accesses across it.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Value of four digit-weight accumulators (weights 256^3 .. 1) at register
// r, exact in FP64 (|sum| < 2^53 for the sizes the mixed path accepts).
__device__ __forceinline__ double g32_value(const v16i (&acc)[4], int r) {
  return (((double)acc[0][r] * 256.0 + (double)acc[1][r]) * 256.0 + (double)acc[2][r]) * 256.0 + (double)acc[3][r];
}


// Several plans' launches of one kernel as one grid: plan k takes work-groups
// [start[k], start[k + 1]) of the flattened grid (its own grid, flattened,
// after the plans before it; every range a multiple of 8 where the kernel's
// tile map is XCD-aware, so that a work-group's XCD is its local index mod 8).
template <class A>
struct BatchArgs {
  int count;
  int64_t start[MAX_BATCH + 1];
  A a[MAX_BATCH];
};

// The plan that work-group b of a batched grid belongs to.
template <class A>
__device__ __forceinline__ int batch_plan(const BatchArgs<A>& B, int64_t b) {
  int k = 0;
  for (int q = 1; q < B.count; ++q) k += (b >= B.start[q]) ? 1 : 0;
  return k;
}

}  // namespace clak
