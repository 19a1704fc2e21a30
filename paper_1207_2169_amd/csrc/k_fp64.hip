// FP64 MFMA kernels: the rotations by Z^T (fixed operands X_L, Q_L, Y in both
// precisions; the SNP blocks in the FP64 path) and the FP64 grid contraction
// with its fused Schur-complement epilogue.
#include "common.hpp"
#include "schur.hpp"

namespace clak {

// v_mfma_f64_16x16x4f64 lane layout (gfx950): lane l supplies A[l%16][l/16]
// and B[l/16][l%16]; result register r holds C[4r + l/16][l%16].

// C = Z^T B over the padded eigen index, 64 x 64 tiles, BK = 16.
//   MODE 0: B real FP64, column-major (ldb), rows >= n and columns >= ncols
//           read as zero; out[k + col * ldo] = C[k][col] for col < ncols.
//   MODE 1: B = int8 SNP panel Gp (ldb SNP rows, K-tiled); the centring
//           x = C[k][col] - sum_a (Z^T Q_L)[k][a] v_a(col) is fused and the
//           result stored SNP-major: out[col * np + k].
//   MODE 2: as MODE 1, but with a single trait the cell sums of the tile's
//           64 rows (c' against the whitened covariate columns, r' against
//           D e, a = d^T (x o x)) are formed in FP64 and written as one partial
//           per (row tile, SNP), part[(blockIdx.x * (pL+2) + q) * mbp + col];
//           the rotated SNPs are not stored.
template <int MODE>
__global__ void __launch_bounds__(256) k_rot64(int64_t n, int64_t np, int pL, const double* __restrict__ Zt,
                                               const void* __restrict__ B, int64_t ldb, int64_t ncols,
                                               double* __restrict__ out, int64_t ldo, const double* __restrict__ Qt,
                                               const double* __restrict__ sstat, const double* __restrict__ V,
                                               const double* __restrict__ Dv, double* __restrict__ part,
                                               int64_t mbp, int tri) {
  constexpr int BM = 64, BN = 64, BK = 16, NPM = MAX_PL + 2;
  __shared__ double As[BK][BM + 1];
  __shared__ double Bs[BK][BN + 1];
  __shared__ double Ps[MODE == 2 ? 2 * BN * NPM : 1];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  const int64_t m0 = (int64_t)blockIdx.x * BM, n0 = (int64_t)blockIdx.y * BN;
  v4d acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (v4d){0.0, 0.0, 0.0, 0.0};
  const int lr = tid >> 2, lk = (tid & 3) * 4;
  const int64_t kend = tri ? min(np, m0 + BM) : np;  // lower-triangular Z^T: K tiles up to the diagonal
  for (int64_t k0 = 0; k0 < kend; k0 += BK) {
    {
      const double* src = Zt + (m0 + lr) * np + k0 + lk;
#pragma unroll
      for (int q = 0; q < 4; ++q) As[lk + q][lr] = src[q];
    }
    if (MODE == 0) {
      const double* Bd = (const double*)B;
      const int64_t col = n0 + lr;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t k = k0 + lk + q;
        Bs[lk + q][lr] = (col < ncols && k < n) ? Bd[k + col * ldb] : 0.0;
      }
    } else {
      const int8_t* Gp = (const int8_t*)B;
      const int32_t packed = *(const int32_t*)(Gp + kt32(n0 + lr, k0 + lk, ldb));  // ldb: rows of the panel
#pragma unroll
      for (int q = 0; q < 4; ++q) Bs[lk + q][lr] = (double)(int8_t)(packed >> (8 * q));
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      double a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[4 * kk + (lane >> 4)][32 * wr + 16 * i + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[4 * kk + (lane >> 4)][32 * wc + 16 * j + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  const int64_t ss = snp_stride(pL);
  if (MODE == 2) {
    const int NP = pL + 2;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int cl = 32 * wc + 16 * j + (lane & 15);
      const double* st = sstat + (n0 + cl) * ss;
      double ps[NPM];
#pragma unroll
      for (int q = 0; q < NPM; ++q) ps[q] = 0.0;
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = m0 + 32 * wr + 16 * i + 4 * r + (lane >> 4);
          double x = acc[i][j][r];
          for (int a = 0; a < pL; ++a) x -= Qt[row + a * np] * st[a];
#pragma unroll
          for (int q = 0; q < NPM - 1; ++q)
            if (q <= pL) ps[q] += V[q * np + row] * x;
          ps[NPM - 1] += Dv[row] * x * x;
        }
#pragma unroll
      for (int q = 0; q < NPM; ++q) {
        double v = ps[q] + __shfl_xor(ps[q], 16, 64);
        v += __shfl_xor(v, 32, 64);
        const int qq = (q == NPM - 1) ? NP - 1 : q;
        if ((lane >> 4) == 0 && (q <= pL || q == NPM - 1)) Ps[(wr * BN + cl) * NPM + qq] = v;
      }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < BN * NP; e += 256) {
      const int cl = e % BN, q = e / BN;
      part[((int64_t)blockIdx.x * NP + q) * mbp + n0 + cl] = Ps[cl * NPM + q] + Ps[(BN + cl) * NPM + q];
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int64_t col = n0 + 32 * wc + 16 * j + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = m0 + 32 * wr + 16 * i + 4 * r + (lane >> 4);
        double x = acc[i][j][r];
        if (MODE == 0) {
          if (col < ncols) out[row + col * ldo] = x;
        } else {
          if (col < ncols) {
            const double* st = sstat + col * ss;
            for (int a = 0; a < pL; ++a) x -= Qt[row + a * np] * st[a];
            out[col * np + row] = x;
          }
        }
      }
    }
}

hipError_t launch_rotate_real(const Plan& p, const double* B, int64_t ldb, int64_t ncols, double* out,
                              int64_t ldo) {
  dim3 grid((unsigned)(p.n_pad / 64), (unsigned)((ncols + 63) / 64));
  k_rot64<0><<<grid, 256, 0, p.stream>>>(p.n, p.n_pad, (int)p.pL, p.ws.Zt, B, ldb, ncols, out, ldo, nullptr,
                                         nullptr, nullptr, nullptr, nullptr, 0, (p.flags & CLAK_CHOL) ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_rotate_snps_fp64(const Plan& p, int64_t m_blk) {
  const int64_t m_pad = roundup(m_blk, 64);
  dim3 grid((unsigned)(p.n_pad / 64), (unsigned)(m_pad / 64));
  const Workspace& W = p.ws;
  const int tri = (p.flags & CLAK_CHOL) ? 1 : 0;
  if (p.fused_t1)
    k_rot64<2><<<grid, 256, 0, p.stream>>>(p.n, p.n_pad, (int)p.pL, W.Zt, W.Gp, p.mb_pad, m_pad, nullptr, 0, W.Qt,
                                           W.sstat, W.V64, W.D64, W.part, p.mb_pad, tri);
  else
    k_rot64<1><<<grid, 256, 0, p.stream>>>(p.n, p.n_pad, (int)p.pL, W.Zt, W.Gp, p.mb_pad, m_pad, W.X64, p.n_pad,
                                           W.Qt, W.sstat, nullptr, nullptr, nullptr, 0, tri);
  return hipGetLastError();
}

// Grid contraction in FP64: a work-group takes 64 SNPs x 16 traits.  B holds
// the 16 (PL+1) operand columns of those traits followed by their 16 d
// columns; the x columns multiply the former, x o x the latter.  The p_L + 2
// sums of each cell then meet in LDS for the Schur-complement solve.
template <int PL>
__global__ void __launch_bounds__(256) k_grid64(int64_t np, int64_t m_blk, int64_t t, const double* __restrict__ X,
                                                const double* __restrict__ V, const double* __restrict__ Dm,
                                                const double* __restrict__ tpar, const double* __restrict__ sstat,
                                                uint32_t flags, CellOut out) {
  constexpr int NCV = 16 * (PL + 1), NC = NCV + 16, NCT = NC / 16, BK = 16;
  __shared__ double As[BK][64 + 1];
  __shared__ double Bs[BK][NC + 1];
  __shared__ double Cs[16][NC + 1];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int64_t i0 = (int64_t)blockIdx.x * 64, j0 = (int64_t)blockIdx.y * 16;
  v4d acc[NCT];
#pragma unroll
  for (int c = 0; c < NCT; ++c) acc[c] = (v4d){0.0, 0.0, 0.0, 0.0};
  const int lr = tid >> 2, lk = (tid & 3) * 4;
  for (int64_t k0 = 0; k0 < np; k0 += BK) {
    {
      const double* src = X + (i0 + lr) * np + k0 + lk;
#pragma unroll
      for (int q = 0; q < 4; ++q) As[lk + q][lr] = src[q];
    }
    for (int e = tid; e < NC * BK; e += 256) {
      const int c = e / BK, kk = e % BK;
      const double* src = (c < NCV) ? V + (j0 * (PL + 1) + c) * np : Dm + (j0 + c - NCV) * np;
      Bs[kk][c] = src[k0 + kk];
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      const double a = As[4 * kk + (lane >> 4)][16 * wid + (lane & 15)];
      const double a2 = a * a;
#pragma unroll
      for (int c = 0; c < NCT; ++c) {
        const double b = Bs[4 * kk + (lane >> 4)][16 * c + (lane & 15)];
        acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(c < PL + 1 ? a : a2, b, acc[c], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // epilogue: one wave's 16 SNPs at a time through LDS, one cell per thread
  for (int w = 0; w < 4; ++w) {
    if (wid == w) {
#pragma unroll
      for (int c = 0; c < NCT; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r) Cs[4 * r + (lane >> 4)][16 * c + (lane & 15)] = acc[c][r];
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
        schur_store<PL>(c, r, a, tpar + j * trait_stride(PL), sstat + i * snp_stride(PL), flags, i, j, out);
      }
    }
    __syncthreads();
  }
}

hipError_t launch_grid_fp64(const Plan& p, int64_t m_blk, const CellOut& out) {
  if (p.fused_t1) return launch_fin_t1(p, m_blk, out);
  dim3 grid((unsigned)((m_blk + 63) / 64), (unsigned)(p.t_pad / 16));
  const Workspace& W = p.ws;
#define CLAK_G64(PLV)                                                                                             \
  case PLV:                                                                                                       \
    k_grid64<PLV><<<grid, 256, 0, p.stream>>>(p.n_pad, m_blk, p.t, W.X64, W.V64, W.D64, W.tpar, W.sstat, p.flags, \
                                              out);                                                               \
    break;
  switch (p.pL) {
    CLAK_G64(1) CLAK_G64(2) CLAK_G64(3) CLAK_G64(4) CLAK_G64(5) CLAK_G64(6) CLAK_G64(7) CLAK_G64(8)
    CLAK_G64(9) CLAK_G64(10) CLAK_G64(11) CLAK_G64(12) CLAK_G64(13) CLAK_G64(14) CLAK_G64(15) CLAK_G64(16)
    default:
      return hipErrorInvalidValue;
  }
#undef CLAK_G64
  return hipGetLastError();
}

hipError_t launch_rotate_snps_mixed(const Plan& p, int64_t m_blk);
hipError_t launch_grid_mixed(const Plan& p, int64_t m_blk, const CellOut& out);

hipError_t launch_rotate_snps(const Plan& p, int64_t m_blk) {
  return p.prec == CLAK_PREC_MIXED ? launch_rotate_snps_mixed(p, m_blk) : launch_rotate_snps_fp64(p, m_blk);
}

hipError_t launch_grid(const Plan& p, int64_t m_blk, const CellOut& out) {
  return p.prec == CLAK_PREC_MIXED ? launch_grid_mixed(p, m_blk, out) : launch_grid_fp64(p, m_blk, out);
}

}  // namespace clak
