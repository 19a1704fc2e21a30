// Grid contraction of the multi-trait CLAK-Eig listing (section 3, the inner
// loop over (SNP, trait) cells: W_R^T W_L, W_R^T Y_j and W_R^T W_R per cell)
// in one or two passes over the individuals, on v_mfma_i32_32x32x32_i8.
//
// For a rotated, centred SNP x and trait j the cell needs p_L + 2 sums over
// the n eigen indices k (the operand columns built by the trait kernel):
//   c'_q = V_q^T x  (q < p_L, whitened covariates),  r' = (D e)^T x,
//   a    = d^T (x o x).
// Every operand is four int8 digit planes with one FP64 scale; a sum is the
// ten digit products of total weight 256^-g, g <= 3, accumulated exactly in
// four int32 accumulators (one per g).
//
// A work-group takes 128 SNPs x 32 traits with four waves, one per SIMD; wave
// w owns the 32 x 32 cells of SNP rows 32 w .. 32 w + 31 and keeps every sum
// of them in its accumulators: p_L + 2 MFMA tiles of 32 x 32, 64 registers
// each.  For p_L <= 2 they fit the 256 accumulation registers and one pass
// over K forms them all.  For p_L = 3 (320 registers) the quadratic sum a
// takes a first pass over the x o x and d planes and is parked in LDS, and the
// p_L + 1 linear sums (256 registers) a second pass over the x and operand
// planes: held in one pass, the compiler kept part of the sums in the
// architectural registers and moved them through the accumulation registers
// around the MFMAs (some 200 register moves per 50 MFMAs).  (p_L <= 3; larger
// p_L take the two-stage kernel of k_mixed.hip.)
//
// Staging: a ring of three 32-deep K slices, two in flight while one is
// multiplied.  The trait operand fragments, which all four waves read, go to
// LDS by direct global-to-LDS loads (global_load_lds_dwordx4) of whole 1 KB
// MFMA fragments (32 rows x 32 bytes of K, the kt32 layout of every digit
// plane), wave w loading plane w of every operand tile of the pass; no LDS
// stores by the waves.  The x (and x o x) fragments of a wave's own SNP rows,
// which no other wave reads, go straight into its registers (three sets), so
// the LDS carries only the shared operand.
//
// Work-groups go round-robin over the 8 XCDs.  XCD x owns a contiguous range
// of the block's SNP tiles and walks all trait groups for sg of them at a
// time, so that the work-groups resident on one XCD share those SNP tiles'
// digits and the trait groups' operand in its L2.
//
// Epilogue: per cell the Schur solve in FP64 (cell_solve, the arithmetic of
// schur_store), then each wave stages its 32 x 32 results per output array in
// LDS and writes them trait row by trait row, 32 consecutive SNPs per
// half-wave store, with the p-value formed from the staged b and SE when it
// is asked for.
#include "common.hpp"
#include "schur.hpp"

namespace clak {

// The tiles of a cell with p_L = PL <= 3: entries c'_0 .. c'_{p_L-1}, r'
// (against x) and a (against x o x), p_L + 2 <= 5 tiles, 320 accumulator
// registers at most, formed in one or two passes over K.  (Larger p_L would
// need more passes; the two-stage kernel of k_mixed.hip serves them.)
template <int PL>
struct GridTiles {
  static constexpr int NT = PL + 2;
  // LDS fragments per slice at most: 4 planes of each trait operand tile (the
  // SNP tiles' x and x o x planes go to registers)
  static constexpr int FB = 4 * NT;
  static_assert(PL >= 1 && PL <= 3, "the ring kernel takes p_L <= 3");
};

constexpr int GR_SLOT = 52 * 1024;  // a ring slot; after the K loop the epilogue's stages and the parked sums
constexpr int GR_STAGE = 32 * 33;   // per-wave epilogue staging: 32 traits x (32 SNPs + 1)

// Arguments of the grid contraction of one plan's block (see grid_tile).
struct GridArgs {
  int64_t np, m_blk, mbp, t, tp, ns, ng;
  int sg;
  const int8_t* Xd;
  const int8_t* Vd;
  const int8_t* Dd;
  const double* vs;
  const double* ds;
  const double* tpar;
  const double* sstat;
  uint32_t flags;
  CellOut out;
};

// A pass over K through a three-slot ring: step s takes the SPS consecutive
// 32-deep slices SPS s .. SPS s + SPS - 1.  The trait operand fragments, which
// the four waves share, go through LDS slot s % 3: the LPW fragments of wave w
// for sub-slice h sit at LDS fragment (h LPW + q) 4 + w (source src(q, slice):
// a wave-uniform base plus the lane's offset loff into the fragment).  The
// XPW fragments of the wave's own SNP tile go straight into registers, one
// set per slot (source xs(q, slice)), so they cost no LDS bandwidth.  As the
// rotation's ring: wait for this wave's loads of step s (the next step's stay
// in flight), barrier (every wave's loads of s have landed, every wave is done
// with step s - 1), load step s + 2 into the slot and register set of s - 1,
// multiply step s (body, once per sub-slice h, given the lane's address in
// the slot, the sub-slice's registers and h).  Past the last slice the loads repeat
// slice KT - 1 into a slot that is not read again (in bounds).  Ends with no
// load in flight and a barrier.  KT must be a multiple of SPS.
template <int LPW, int XPW, int SPS, class Src, class XSrc, class Body>
__device__ __forceinline__ void grid_kloop(int KT, int w, int lane, uint32_t loff, int8_t* s0, int8_t* s1, int8_t* s2,
                                           Src src, XSrc xs, Body body) {
  int8_t* const slots[3] = {s0, s1, s2};
  v4i xr[3][SPS * XPW];
  const int NS = KT / SPS;
  auto issue = [&](int u, int s) {
    int8_t* dst = slots[u];
#pragma unroll
    for (int h = 0; h < SPS; ++h)
#pragma unroll
      for (int q = 0; q < LPW; ++q)
        __builtin_amdgcn_global_load_lds(src(q, min(SPS * s + h, KT - 1)) + loff,
                                         (lds_ptr_t)(dst + ((h * LPW + q) * 4 + w) * 1024), 16, 0, 0);
#pragma unroll
    for (int h = 0; h < SPS; ++h)
#pragma unroll
      for (int q = 0; q < XPW; ++q) xr[u][h * XPW + q] = *(const v4i*)(xs(q, min(SPS * s + h, KT - 1)) + loff);
  };
  auto step = [&](int u, int s) {
    wait_vm<(LPW + XPW) * SPS>();
    lds_barrier();
    issue((u + 2) % 3, s + 2);
#pragma unroll
    for (int h = 0; h < SPS; ++h)
      body((const int8_t*)(slots[u] + h * LPW * 4 * 1024 + 16 * lane), (const v4i*)&xr[u][h * XPW], h);
  };
  issue(0, 0);
  issue(1, 1);
  int s = 0;
  for (; s + 3 <= NS; s += 3) {
    step(0, s);
    step(1, s + 1);
    step(2, s + 2);
  }
  if (s < NS) step(0, s);
  if (s + 1 < NS) step(1, s + 1);
  wait_vm<0>();     // no load is left in flight
  __syncthreads();  // the ring is free for the next pass or the epilogue
}

// Work-group bid of the grid of one plan's block.
template <int PL, bool FULL>
__device__ __forceinline__ void grid_tile(const GridArgs& ga, int64_t bid) {
  const int64_t np = ga.np, m_blk = ga.m_blk, mbp = ga.mbp, t = ga.t, tp = ga.tp, ns = ga.ns, ng = ga.ng;
  const int sg = ga.sg;
  const int8_t* __restrict__ Xd = ga.Xd;
  const int8_t* __restrict__ Vd = ga.Vd;
  const int8_t* __restrict__ Dd = ga.Dd;
  const double* __restrict__ vs = ga.vs;
  const double* __restrict__ ds = ga.ds;
  const double* __restrict__ tpar = ga.tpar;
  const double* __restrict__ sstat = ga.sstat;
  const uint32_t flags = ga.flags;
  const CellOut& out = ga.out;
  using GT = GridTiles<PL>;
  constexpr int NV = PL + 1, NT = GT::NT;
  static_assert(GR_SLOT >= GT::FB * 1024, "slot size");
  __shared__ __attribute__((aligned(1024))) int8_t smem0[GR_SLOT];
  __shared__ __attribute__((aligned(1024))) int8_t smem1[GR_SLOT];
  __shared__ __attribute__((aligned(1024))) int8_t smem2[GR_SLOT];
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);

  // work-group -> (SNP tile, trait group): XCD x owns SNP tiles [x gs, x gs + gs)
  const int64_t xcd = bid % 8, idx = bid / 8, gs = (ns + 7) / 8;
  const int64_t c = idx / (sg * ng), base = c * sg * ng, cs = min((int64_t)sg, gs - c * sg);
  if (cs <= 0) return;
  const int64_t rem = idx - base, tg = rem / cs, sl = c * sg + rem % cs, st = xcd * gs + sl;
  if (tg >= ng || sl >= gs || st >= ns) return;
  const int64_t i0 = st * 128, j0 = tg * 32;
  const int64_t xplane = mbp * np, vplane = tp * NV * np, dplane = tp * np;
  const int KT = (int)(np / 32);
  const uint32_t loff = 32 * (lane & 31) + 16 * (lane >> 5);
  const int64_t vgrp = (j0 >> 5) * 32 * NV;  // first operand row of the trait group

  // One pass over K holds every sum of a cell (p_L + 2 tiles x four weight
  // groups) in the accumulators when they fit the 256 accumulation registers
  // (p_L <= 2).  For p_L = 3 (320 registers) the compiler would keep part of
  // them in the architectural registers and shuttle them through the
  // accumulation registers around every MFMA, so the quadratic sum a goes
  // first, in a pass of its own over the x o x and d planes, and is parked in
  // LDS (16 doubles per lane); the linear sums follow in a second pass.
  constexpr bool TWO = NT * 64 > 256;
  constexpr int NTB = TWO ? NV : NT;  // tiles of the main pass
  v16i acc[NTB][4];
#pragma unroll
  for (int q = 0; q < NTB; ++q)
#pragma unroll
    for (int g = 0; g < 4; ++g) acc[q][g] = (v16i){};
  // the quadratic sums parked between the passes: [r][lane] doubles per wave,
  // waves 0, 1 past byte ASAVE_OFF of slot 0, waves 2, 3 of slot 1 (free of
  // the second pass's 16 KB slices and of the epilogue's 33.8 KB stages)
  constexpr int ASAVE_OFF = 36 * 1024;
  static_assert(!TWO || (ASAVE_OFF + 2 * 16 * 64 * 8 <= GR_SLOT && ASAVE_OFF >= 8 * GR_STAGE * 4 &&
                         ASAVE_OFF >= NV * 4 * 1024),
                "parked sums must not overlap the ring or the stages");
  double* asave = (double*)((w < 2 ? smem0 : smem1) + ASAVE_OFF) + (w & 1) * 16 * 64 + lane;

  // The ten digit products of total weight g = a + b <= 3 of one slice into
  // the four weight-group accumulators A[g].
  auto products = [](const v4i* a, const v4i* b, v16i(&A)[4]) {
    A[0] = mfma32_i8(a[0], b[0], A[0]);
    A[1] = mfma32_i8(a[0], b[1], A[1]);
    A[2] = mfma32_i8(a[0], b[2], A[2]);
    A[3] = mfma32_i8(a[0], b[3], A[3]);
    A[1] = mfma32_i8(a[1], b[0], A[1]);
    A[2] = mfma32_i8(a[1], b[1], A[2]);
    A[3] = mfma32_i8(a[1], b[2], A[3]);
    A[2] = mfma32_i8(a[2], b[0], A[2]);
    A[3] = mfma32_i8(a[2], b[1], A[3]);
    A[3] = mfma32_i8(a[3], b[0], A[3]);
  };

  // source of digit plane p of the x (xq: x o x) fragments of this wave's SNP tile
  auto xsrc = [&](int p, int s) { return Xd + p * xplane + ((int64_t)s * mbp + i0 + 32 * w) * 32; };
  // plane w of trait operand entry e (d for e = PL + 1)
  auto tsrc = [&](int e, int s) {
    return e <= PL ? Vd + w * vplane + ((int64_t)s * tp * NV + vgrp + 32 * e) * 32
                   : Dd + w * dplane + ((int64_t)s * tp + j0) * 32;
  };

  if constexpr (TWO) {
    // pass A: a = d^T (x o x), two slices per ring step (ten MFMAs per slice
    // would not cover the loads' latency), each slice of a step into its own
    // set of the four accumulators (two independent MFMA chains per weight
    // group; the sets are added exactly in int32 at the end); LDS fragments
    // per slice: the d planes; registers: the wave's x o x planes
    v16i accA[2][4];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int g = 0; g < 4; ++g) accA[h][g] = (v16i){};
    grid_kloop<1, 4, 2>(KT, w, lane, loff, smem0, smem1, smem2, [&](int, int s) { return tsrc(PL + 1, s); },
          [&](int q, int s) { return xsrc(4 + q, s); },
          [&](const int8_t* sp, const v4i* xq, int h) {
            v4i b[4];
#pragma unroll
            for (int p = 0; p < 4; ++p) b[p] = *(const v4i*)(sp + p * 1024);
            products(xq, b, accA[h]);
          });
#pragma unroll
    for (int g = 0; g < 4; ++g) accA[0][g] += accA[1][g];
#pragma unroll
    for (int r = 0; r < 16; ++r) asave[r * 64] = g32_value(accA[0], r);
    // pass B: the linear sums; LDS fragments: operand entry e plane p at 4 e + p; registers: the x planes
    grid_kloop<NV, 4, 1>(KT, w, lane, loff, smem0, smem1, smem2, [&](int q, int s) { return tsrc(q, s); },
          [&](int q, int s) { return xsrc(q, s); },
          [&](const int8_t* sp, const v4i* xa, int) {
            // the next entry's operand fragments are read while this entry's
            // MFMAs run (two register sets), so an LDS read latency is exposed
            // once per slice, not once per entry
            v4i b[2][4];
#pragma unroll
            for (int p = 0; p < 4; ++p) b[0][p] = *(const v4i*)(sp + p * 1024);
#pragma unroll
            for (int tt = 0; tt < NV; ++tt) {
              if (tt + 1 < NV)
#pragma unroll
                for (int p = 0; p < 4; ++p) b[(tt + 1) & 1][p] = *(const v4i*)(sp + (4 * (tt + 1) + p) * 1024);
              products(xa, b[tt & 1], acc[tt]);
            }
          });
  } else {
    // one pass; LDS fragments: tile tt plane p at 4 tt + p; registers: the x, then the x o x planes
    grid_kloop<NT, 8, 1>(KT, w, lane, loff, smem0, smem1, smem2, [&](int q, int s) { return tsrc(q, s); },
          [&](int q, int s) { return xsrc(q, s); },
          [&](const int8_t* sp, const v4i* xr, int) {
#pragma unroll
            for (int tt = 0; tt < NT; ++tt) {
              v4i b[4];
#pragma unroll
              for (int p = 0; p < 4; ++p) b[p] = *(const v4i*)(sp + (4 * tt + p) * 1024);
              products(tt == NT - 1 ? xr + 4 : xr, b, acc[tt]);
            }
          });
  }

  // per-lane trait (column lane % 32 of every tile) and its parameters
  const int64_t j = j0 + (lane & 31);
  const bool jok = j < t;
  const int64_t jj = jok ? j : 0;
  const double* tpj = tpar + jj * trait_stride(PL);

  // ---- epilogue.  LDS after the K loop: slot 0 stages b, slot 1 SE, slot 2
  // the flags and the work-group's per-SNP tables; wave w owns [32 traits][33]
  // of each stage, so the stages need no work-group barrier.
  constexpr int FLG_BYTES = 4 * GR_STAGE;
  static_assert(FLG_BYTES + 128 * (2 + PL) * 8 <= GR_SLOT, "stage size");
  double* gxT = (double*)(smem2 + FLG_BYTES);  // [128] max |x~| of the SNP
  double* flT = gxT + 128;                     // [128] SNP flag
  double* gmT = flT + 128;                     // [128][PL] centring coefficients (full vector)
  const int64_t ss = snp_stride(PL);
  if (tid < 128) {
    const int64_t i = i0 + tid;
    const bool iok = i < m_blk;
    gxT[tid] = iok ? sstat[i * ss + 2 * PL + 2] : 0.0;
    flT[tid] = iok ? sstat[i * ss + 2 * PL + 1] : 0.0;
    if constexpr (FULL)
#pragma unroll
      for (int q = 0; q < PL; ++q) gmT[tid * PL + q] = iok ? sstat[i * ss + PL + q] : 0.0;
  }
  __syncthreads();

  // trait parameters of this lane
  double sc[NT];
#pragma unroll
  for (int tt = 0; tt < NT; ++tt) sc[tt] = (tt <= PL ? vs[jj * NV + tt] : ds[jj]) * (1.0 / 127.0);
  const double s2 = tpj[PL * PL + PL];
  const bool want_p = out.pval != nullptr;
  double* sb = (double*)smem0 + w * GR_STAGE;
  double* sse = (double*)smem1 + w * GR_STAGE;
  uint8_t* sfl = (uint8_t*)smem2 + w * GR_STAGE;  // [32][33] bytes per wave
  const int64_t iw = i0 + 32 * w;

  // cell r of this lane: SNP row 8 (r / 4) + 4 (lane / 32) + r % 4 of the
  // wave's tile, trait j; solved in FP64 and staged
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int rw = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3), rl = 32 * w + rw;
    const double gx = gxT[rl];
    double cc = 0.0, rr = 0.0, a = 0.0;
    double cv[FULL ? PL : 1];
#pragma unroll
    for (int e = 0; e < NT; ++e) {
      double raw;
      if constexpr (TWO)
        raw = (e == NT - 1 ? asave[r * 64] : g32_value(acc[e < NTB ? e : 0], r)) * sc[e];
      else
        raw = g32_value(acc[e < NTB ? e : 0], r) * sc[e];
      if (e < PL) {
        const double v = raw * gx;
        cc += v * v;
        if constexpr (FULL) cv[e] = v;
      } else if (e == PL) {
        rr = raw * gx;
      } else {
        a = raw * gx * gx;
      }
    }
    const CellResult res = cell_solve(cc, rr, a, s2, (int)flT[rl], flags, false);
    const int so = (lane & 31) * 33 + rw;
    sb[so] = res.b;
    sse[so] = res.se;
    sfl[so] = (uint8_t)res.flag;
    if constexpr (FULL) {
      // b_cov = u - (L^{-T} c' + gamma) b_snp (the last term undoes the
      // centring), written in place (the full vector is not staged)
      const int64_t i = iw + rw;
      if (jok && i < m_blk) {
        const int64_t o = (i + j * out.ldo) * (PL + 1);
#pragma unroll
        for (int q = 0; q < PL; ++q) {
          double lc = 0.0;
#pragma unroll
          for (int l = 0; l < PL; ++l) lc += tpj[l * PL + q] * cv[l];
          const double bq = res.flag ? __builtin_nan("") : tpj[PL * PL + q] - (lc + gmT[rl * PL + q]) * res.b;
          if (out.f64) ((double*)out.b)[o + q] = bq;
          else ((float*)out.b)[o + q] = (float)bq;
        }
      }
    }
    __builtin_amdgcn_sched_barrier(0);  // one cell at a time
  }
  __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): this wave's stage writes are done
  __builtin_amdgcn_wave_barrier();

  // stores, trait row by trait row: half-wave h writes 32 consecutive SNPs of trait 2 it + h
  const int64_t bstride = FULL ? PL + 1 : 1, boff = FULL ? PL : 0;
#pragma unroll 4
  for (int it = 0; it < 16; ++it) {
    const int tr = 2 * it + (lane >> 5), sn = lane & 31;
    const int64_t i = iw + sn, jt = j0 + tr;
    if (i < m_blk && jt < t) {
      const int64_t o = i + jt * out.ldo;
      const int so = tr * 33 + sn;
      const double bv = sb[so], sv = sse[so];
      const uint8_t fv = sfl[so];
      if (out.f64) {
        ((double*)out.b)[o * bstride + boff] = bv;
        ((double*)out.se)[o] = sv;
      } else {
        ((float*)out.b)[o * bstride + boff] = (float)bv;
        ((float*)out.se)[o] = (float)sv;
      }
      if (want_p) {  // the p-value as store_snp forms it, from the staged b and SE
        const double pv = fv ? __builtin_nan("") : erfc(fabs(bv / sv) * M_SQRT1_2);
        if (out.f64)
          ((double*)out.pval)[o] = pv;
        else
          ((float*)out.pval)[o] = (float)pv;
      }
      if (out.flags) out.flags[o] = fv;
    }
  }
}

template <int PL, bool FULL>
__global__ void __launch_bounds__(256, 1) k_grid_ring(GridArgs a) {
  grid_tile<PL, FULL>(a, blockIdx.x);
}

// The grid contractions of several plans' blocks in one launch.
template <int PL, bool FULL>
__global__ void __launch_bounds__(256, 1) k_grid_ring_batch(BatchArgs<GridArgs> B) {
  const int64_t b = blockIdx.x;
  const int k = batch_plan(B, b);
  grid_tile<PL, FULL>(B.a[k], b - B.start[k]);
}

// Work-groups of the ring grid kernel for a block of m_blk SNPs: 128-SNP
// tiles spread over the 8 XCDs in contiguous ranges, sg of them walked
// together over every 32-trait group.
hipError_t launch_grid_ring(const Plan& p, int64_t m_blk, const CellOut& out) {
  const Workspace& W = p.ws;
  const int64_t ns = (m_blk + 127) / 128, ng = (p.t + 31) / 32, gs = (ns + 7) / 8;
  const int sg = p.grid_xt ? p.grid_xt : 4;
  const dim3 grid((unsigned)(8 * gs * ng));
  const bool full = (p.flags & CLAK_OUT_FULL) != 0;
  const GridArgs ga{p.n_pad, m_blk, p.mb_pad, p.t, p.t_pad, ns, ng, sg, W.Xd, W.Vd, W.Dd, W.vs, W.ds, W.tpar, W.sstat,
                    p.flags, out};
#define CLAK_GR(PLV, F) k_grid_ring<PLV, F><<<grid, 256, 0, p.stream>>>(ga)
#define CLAK_GRP(PLV)     \
  case PLV:               \
    if (full)             \
      CLAK_GR(PLV, true); \
    else                  \
      CLAK_GR(PLV, false); \
    break;
  switch (p.pL) {
    CLAK_GRP(1) CLAK_GRP(2) CLAK_GRP(3)
    default:
      return hipErrorInvalidValue;
  }
#undef CLAK_GRP
#undef CLAK_GR
  return hipGetLastError();
}

// Plans whose blocks can share batched launches.  A batched round always
// takes the ring grid kernel and the built-in rotation tiles of multi-trait
// plans (each plan keeps its XCD groupings); every launch variant computes
// the same bits, so a plan's tuned variants need not match.
bool batch_compatible(const Plan& a, const Plan& b) {
  auto ok = [](const Plan& p) {
    return p.prec == CLAK_PREC_MIXED && !p.fused_t1 && p.pL <= 3 && !(p.flags & CLAK_STAGE_GENOTYPES);
  };
  return ok(a) && ok(b) && a.pL == b.pL && (a.flags & CLAK_OUT_FULL) == (b.flags & CLAK_OUT_FULL) &&
         a.device == b.device;
}

hipError_t launch_grid_batch(const BatchItem* it, int count, hipStream_t st) {
  if (count < 1 || count > MAX_BATCH) return hipErrorInvalidValue;
  BatchArgs<GridArgs> B{};
  B.count = count;
  for (int k = 0; k < count; ++k) {
    const Plan& p = *it[k].p;
    const Workspace& W = p.ws;
    const Slot& S = W.slot[it[k].slot];
    const int64_t ns = (it[k].m_blk + 127) / 128, ng = (p.t + 31) / 32, gs = (ns + 7) / 8;
    const int sg = (p.grid_tt == 0 && p.grid_xt) ? p.grid_xt : 4;  // grid_xt means sg only for the ring kernel
    B.a[k] = GridArgs{p.n_pad, it[k].m_blk, p.mb_pad, p.t, p.t_pad, ns, ng, sg, S.Xd, W.Vd, W.Dd, W.vs, W.ds, W.tpar,
                      S.sstat, p.flags, it[k].out};
    B.start[k + 1] = B.start[k] + 8 * gs * ng;
  }
  const dim3 grid((unsigned)B.start[count]);
  const bool full = (it[0].p->flags & CLAK_OUT_FULL) != 0;
  switch (it[0].p->pL) {
#define CLAK_GB(PLV)                                                                                  \
  case PLV:                                                                                           \
    full ? k_grid_ring_batch<PLV, true><<<grid, 256, 0, st>>>(B) : k_grid_ring_batch<PLV, false><<<grid, 256, 0, st>>>(B); \
    break;
    CLAK_GB(1) CLAK_GB(2) CLAK_GB(3)
#undef CLAK_GB
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace clak
