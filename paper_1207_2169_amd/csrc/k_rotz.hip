// Z-resident SNP rotation of the mixed path (rotation configuration 10), for
// n_pad <= 1024 and the plain (non-triangular) operand.
//
// The same product as k_rot_i8, X~ = Z^T G with fused centring (multi-trait
// CLAK-Eig, supplementary notes, section 3), organised the other way round: a
// work-group keeps one 32-row slice of Z^T, all four digit planes over the
// whole contraction (4 x 32 x n_pad bytes, 128 KB at n_pad = 1024), in LDS for
// its lifetime, and its eight waves stream genotype fragments from global
// memory straight into registers, two 32-SNP tiles at a time, four K steps
// ahead.  The K loop has no barrier and no LDS store: per 32-deep step a wave
// reads four 1 KB fragments of Z^T from LDS (ds_read_b128, conflict-free) and
// issues eight MFMAs (v_mfma_i32_32x32x32_i8), so the LDS carries half the
// bytes per MFMA of the staged kernels and the waves never wait for each
// other.  Two waves share a SIMD, so one wave's epilogue (FP64) overlaps the
// other's MFMAs.
//
// Work map: work-group b runs on XCD b % 8; XCD x owns the x-th eighth of the
// block's 32-SNP tiles, and its work-groups take (slice s, SNP sub-range j),
// s fastest, so that at n_pad = 1024 its 32 CUs hold the 32 slices of Z^T
// and read each genotype tile of the XCD's range from its L2.  Within a
// work-group the tiles go to the waves in pairs, pair i to wave i % 8: a
// SIMD's two waves share its pairs between them.
//
// Per element the planes are recombined, scaled and centred exactly as in
// k_rot_i8, and the per-SNP results are bitwise the same: EPI 0 stores x~ and
// raises the SNP's max |x~_k|; EPI 1 (single trait) writes the partial of
// a = d^T (x~ o x~) over the slice's 32 rows (the per-wave-row partial of
// k_rot_i8), which the single-trait finish adds in pairs to form the 64-row
// partials of the other configurations before summing them in their order,
// and the U^T rows go to the SNP's statistics.
#include "common.hpp"

namespace clak {

constexpr int ZR_KS = 32;    // 32-deep K steps the LDS slice holds: n_pad <= 1024
constexpr int ZR_D = 4;      // genotype fragments in flight per wave, in K steps (n_pad / 32 is a multiple)
constexpr int ZR_WAVES = 8;  // waves per work-group (two per SIMD)
constexpr int ZR_PL_MAX = 4;
static_assert(KPAD % (32 * ZR_D) == 0, "K steps per item must be a multiple of the prefetch depth");

struct ZRotArgs {
  int64_t np, nz, zl, mb, mbp, ntl;  // ntl: 32-SNP tiles of the block
  int S, q;                          // slices (nz / 32), SNP sub-ranges per XCD
  const int8_t* Zd;
  const double* zs;
  const int8_t* Gp;
  const double* Qt;
  const double* Cq;
  double* sstat;
  double* X;
  const double* Dv;
  double* part;
};

template <int PL, int EPI>
__global__ void __launch_bounds__(64 * ZR_WAVES, 1) k_rot_zs(ZRotArgs a) {
  __shared__ __attribute__((aligned(1024))) int8_t zsl[ZR_KS * 4 * 1024];  // fragment (k, p) at (4 k + p) KB
  __shared__ double Qs[32 * PL], zS[32], Vs[32];
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t bid = blockIdx.x, xcd = bid % 8, idx = bid / 8;
  const int64_t s = idx % a.S, j = idx / a.S;
  const int64_t T8 = (a.ntl + 7) / 8, xb = xcd * T8, xe = min(a.ntl, xb + T8);
  const int64_t Tq = (T8 + a.q - 1) / a.q, tb = xb + j * Tq, te = min(xe, tb + Tq);
  if (j >= a.q || tb >= te) return;  // uniform over the work-group
  const int64_t np = a.np, nz = a.nz, mbp = a.mbp, m0 = 32 * s, zl = a.zl;
  const int KS = (int)(np / 32);
  const int loff = 32 * (lane & 31) + 16 * (lane >> 5);  // MFMA operand bytes of this lane in a 1 KB fragment

  // the slice of Z^T: every fragment by a direct global-to-LDS load (lane l's
  // 16 bytes land at byte 16 l of the fragment, the order of the operand reads)
  {
    const int8_t* za = a.Zd + m0 * 32 + loff;
    const int64_t zplane = nz * np;
    for (int f = w; f < 4 * KS; f += ZR_WAVES) {
      const int k = f >> 2, p = f & 3;
      __builtin_amdgcn_global_load_lds(za + p * zplane + (int64_t)k * nz * 32, (lds_ptr_t)(zsl + f * 1024), 16, 0,
                                       0);
    }
  }
  // epilogue tables of the slice's rows: centring rows (Z^T Q_L, or C for the
  // U^T rows), digit scales, d (EPI 1)
  for (int e = tid; e < 32 * PL; e += 64 * ZR_WAVES) {
    const int64_t row = m0 + e / PL;
    const int c = e % PL;
    Qs[e] = (row >= zl && row <= zl + PL) ? a.Cq[c * (PL + 1) + (row - zl)] : (row < np ? a.Qt[row + c * np] : 0.0);
  }
  if (tid < 32) {
    zS[tid] = a.zs[m0 + tid];
    Vs[tid] = (EPI == 1 && m0 + tid < np) ? a.Dv[m0 + tid] : 0.0;
  }
  wait_vm<0>();
  __syncthreads();

  // this wave's tile pairs: pair i of the work-group is tiles tb + 2 i, +1
  const int64_t P = (te - tb + 1) / 2;
  const int NI = P > w ? (int)((P - w + ZR_WAVES - 1) / ZR_WAVES) : 0;
  if (NI == 0) return;  // no barrier follows
  auto tile = [&](int i, int ct) -> int64_t { return tb + 2 * (w + (int64_t)ZR_WAVES * i) + ct; };
  // fragment source of (item i, K step k, tile ct); a second tile past the
  // range repeats the range's last tile (in bounds, its results are dropped)
  const int8_t* gb = a.Gp + loff;
  auto bsrc = [&](int i, int k, int ct) -> const v4i* {
    const int64_t t = min(tile(i, ct), te - 1);
    return (const v4i*)(gb + ((int64_t)k * mbp + 32 * t) * 32);
  };
  const int64_t ss = snp_stride(PL);

  v4i bq[ZR_D][2];
#pragma unroll
  for (int u = 0; u < ZR_D; ++u) {
    bq[u][0] = *bsrc(0, u, 0);
    bq[u][1] = *bsrc(0, u, 1);
  }
  // next fragment to fetch: (pi, pk), D steps ahead over the wave's items;
  // past the last item it repeats the last step (every step has the same
  // loads, so the outstanding-load count is the same on every path)
  int pi = ZR_D / KS, pk = ZR_D % KS;  // KS >= ZR_D
  for (int i = 0; i < NI; ++i) {
    double v[2][PL];
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      const int64_t col = 32 * min(tile(i, ct), te - 1) + (lane & 31);
#pragma unroll
      for (int c = 0; c < PL; ++c) v[ct][c] = a.sstat[col * ss + c];
    }
    v16i acc[2][4];
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
      for (int p = 0; p < 4; ++p) acc[ct][p] = (v16i){};
    for (int k0 = 0; k0 < KS; k0 += ZR_D) {
#pragma unroll
      for (int u = 0; u < ZR_D; ++u) {
        const int8_t* as = zsl + (4 * (k0 + u)) * 1024 + 16 * lane;
        v4i af[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) af[p] = *(const v4i*)(as + p * 1024);
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          acc[0][p] = mfma32_i8(af[p], bq[u][0], acc[0][p]);
          acc[1][p] = mfma32_i8(af[p], bq[u][1], acc[1][p]);
        }
        // the slot's next fragments are fetched after its MFMAs are issued,
        // into the same registers (a load hoisted above them would need other
        // registers and a copy that waits for the load at the loop's end)
        __builtin_amdgcn_sched_barrier(0);
        const int fi = pi < NI ? pi : NI - 1, fk = pi < NI ? pk : KS - 1;
        bq[u][0] = *bsrc(fi, fk, 0);
        bq[u][1] = *bsrc(fi, fk, 1);
        if (++pk == KS) {
          pk = 0;
          ++pi;
        }
      }
    }

    // epilogue (as k_rot_i8): the planes of both tiles paired exactly in
    // int32 first, which frees half the accumulator registers, then one tile
    // at a time recombined and scaled in FP64 and centred
    int hp[2][16], lp[2][16];
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        hp[ct][e] = acc[ct][0][e] * 256 + acc[ct][1][e];
        lp[ct][e] = acc[ct][2][e] * 256 + acc[ct][3][e];
      }
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      __builtin_amdgcn_sched_barrier(0);
      const int64_t t = tile(i, ct);
      if (t >= te) continue;
      const int64_t col = 32 * t + (lane & 31);
      const int* hc = hp[ct];
      const int* lc = lp[ct];
      double pa = 0.0, mx = 0.0;
#pragma unroll
      for (int gq = 0; gq < 4; ++gq) {
        const int rb0 = 8 * gq + 4 * (lane >> 5);
        double xs[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int rr = rb0 + r, e = 4 * gq + r;
          double x = fma((double)hc[e], 65536.0, (double)lc[e]) * zS[rr];
#pragma unroll
          for (int c = 0; c < PL; ++c) x -= Qs[rr * PL + c] * v[ct][c];
          xs[r] = x;
          if (EPI == 0) {
            mx = fmax(mx, fabs(x));
          } else {
            const int64_t row = m0 + rr;
            if (row >= zl && row <= zl + PL)
              a.sstat[col * ss + 2 * PL + 3 + (row - zl)] = x;
            else
              pa += Vs[rr] * x * x;
          }
        }
        if (EPI == 0) *(v4d*)(a.X + col * np + m0 + rb0) = (v4d){xs[0], xs[1], xs[2], xs[3]};
        __builtin_amdgcn_sched_barrier(0);
      }
      if (EPI == 0) {
        const double m = fmax(mx, __shfl_xor(mx, 32, 64));
        if ((lane >> 5) == 0 && col < a.mb)
          atomicMax((unsigned long long*)(a.sstat + col * ss + 2 * PL + 2),
                    (unsigned long long)__double_as_longlong(m));
      } else {
        const double sq = pa + __shfl_xor(pa, 32, 64);
        if ((lane >> 5) == 0 && m0 < np) a.part[s * mbp + col] = sq;
      }
    }
  }
}

bool rot_zs_applicable(const Plan& p) {
  return p.prec == CLAK_PREC_MIXED && p.n_pad <= 32 * ZR_KS && !(p.flags & CLAK_CHOL) && p.pL <= ZR_PL_MAX &&
         p.zrows % 32 == 0;
}

hipError_t launch_rotate_zs(const Plan& p, int64_t m_blk) {
  const Workspace& W = p.ws;
  const int S = (int)(p.zrows / 32);
  const int q = S >= 32 ? 1 : (32 + S / 2) / S;  // about one work-group per CU (32 CUs per XCD)
  const int64_t ntl = roundup(m_blk, SNP_PAD) / 32;
  dim3 grid((unsigned)(8 * (int64_t)S * q)), block(64 * ZR_WAVES);
  const bool t1 = p.fused_t1;
  const ZRotArgs args{p.n_pad, p.zrows, p.zlin, m_blk, p.mb_pad, ntl, S, q, W.Zd, W.zs, W.Gp, W.Qt, W.Cq, W.sstat,
                      t1 ? nullptr : W.X64, t1 ? W.D64 : nullptr, t1 ? W.part : nullptr};
#define CLAK_ZR(PLV)                                                                  \
  case PLV:                                                                           \
    if (t1)                                                                           \
      k_rot_zs<PLV, 1><<<grid, block, 0, p.stream>>>(args);                           \
    else                                                                              \
      k_rot_zs<PLV, 0><<<grid, block, 0, p.stream>>>(args);                           \
    break;
  switch (p.pL) {
    CLAK_ZR(1) CLAK_ZR(2) CLAK_ZR(3) CLAK_ZR(4)
    default:
      return hipErrorInvalidValue;
  }
#undef CLAK_ZR
  return hipGetLastError();
}

}  // namespace clak
