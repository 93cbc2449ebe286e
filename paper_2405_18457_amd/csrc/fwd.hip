// Fused matrix-free kernel-matrix product  out = scale * M(X1, X2) V (+ noise * V1).
//
// M is the Matern-3/2 kernel without its a^2 factor, evaluated in registers and
// never stored (the paper's regularised kernel matrix, Sec. 2; App. B counts
// one "epoch" as computing every entry once).  Work split:
//
//   * one workgroup = 4 waves; every wave owns RS row sub-tiles of 16 rows
//     (RS = 4 for up to 80 columns, 2 above: more rows per wave reuse every
//     loaded V tile and coordinate more often, which keeps the vector-L1
//     load traffic well below its throughput) and streams the kernel columns
//     j in steps of 32;
//   * per step each lane evaluates 8 kernel values of one row i (lane % 16)
//     against 8 consecutive columns j (8 * (lane / 16) + e) with direct
//     coordinate differences in FP32 (no norm expansion, so no cancellation),
//     one v_sqrt_f32 and one v_exp_f32 per entry;
//   * those 8 values are exactly the A operand a lane supplies to
//     v_mfma_f32_16x16x32_bf16 (row = lane % 16, k = 8 (lane / 16) + e), so
//     the tile goes from the VALU straight into the matrix core with no LDS
//     round trip; V arrives pre-packed in the matching B-operand order
//     (16 columns x 32 rows per 1 KiB tile, column-major), one 16-byte load
//     per lane per tile;
//   * BF16X3 splits both operands into bf16 hi + lo and accumulates
//     hi*hi + hi*lo + lo*hi in FP32 (Henry, Tang & Heinecke 2019), which keeps
//     the product within ~1e-5 of FP32; BF16 uses hi*hi only;
//   * FP32 mode uses v_mfma_f32_16x16x4_f32 with the kernel value as a scalar
//     A operand (row = lane % 16, k = lane / 16) and V in a 32x16 tile order
//     that gives each lane 8 consecutive floats per step.
//
// Software pipeline.  The VALU (distances, sqrt, exp2) and the matrix cores
// are separate units; one wave keeps both busy by interleaving, in every
// half-step, the MFMAs of one row sub-tile with the VALU work that produces
// the next sub-tile's A operand:
//     sub-tile r < RS-1:  VALU A(r+1, step k)   ||  MFMA  acc[r] += A(r, k) B(k)
//     sub-tile RS-1:      VALU A(0, step k+1)   ||  MFMA  acc[RS-1] += A(RS-1, k) B(k)
// The step loop is unrolled by two with swapped register buffers (no register
// copies); the next step's coordinates are loaded at the start of a step and
// each V tile is reloaded for the next step right after its last MFMA use.
// The direct kernels pin the MFMA/VALU alternation with scheduling groups; the
// cross-term kernel leaves the order inside a half-step to the compiler, which
// measured 2.8 % faster at d = 3 than groups of 1 MFMA : 4 VALU.
//
// Accuracy: a fresh accumulator per chunk of kChunk column steps is folded
// into a running total (two-level summation keeps FP32 chains short at large n).
// For small n the column range is split over S workgroups per row block and a
// second kernel sums the S partial tiles in a fixed order (deterministic).
#include "gpk.h"

namespace gpk {

namespace {

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

constexpr int kChunk = 64;  // column steps (x 32 columns) per partial accumulator

// sched_group_barrier masks
constexpr int kMaskVALU = 0x002;
constexpr int kMaskMFMA = 0x008;
constexpr int kMaskVMEMRead = 0x020;

template <int D>
__device__ __forceinline__ float sqdist(const float (&xi)[D], const float (&xj)[D]) {
  float r2 = 0.f;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const float t = xi[k] - xj[k];
    r2 = __builtin_fmaf(t, t, r2);
  }
  return r2;
}

// m(rho) = (1 + ln2 rho) 2^-rho with rho^2 = r2 in pre-scaled units.
__device__ __forceinline__ float matern_r2(float r2) {
  const float rho = __builtin_amdgcn_sqrtf(r2);
  const float e = __builtin_amdgcn_exp2f(-rho);
  return __builtin_fmaf(rho, kLn2, 1.0f) * e;
}

// 2^-rho * dhat_k^2 : the length-scale derivative kernel up to a constant factor.
template <int D>
__device__ __forceinline__ float dlen_val(const float (&xi)[D], const float (&xj)[D], int kd) {
  float r2 = 0.f, dk = 0.f;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const float t = xi[k] - xj[k];
    r2 = __builtin_fmaf(t, t, r2);
    dk = (k == kd) ? t : dk;
  }
  const float e = __builtin_amdgcn_exp2f(-__builtin_amdgcn_sqrtf(r2));
  return e * dk * dk;
}

template <int D>
__device__ __forceinline__ void load_point(const float* __restrict__ p, float (&x)[D]) {
  constexpr int DP = (D + 3) & ~3;
#pragma unroll
  for (int q = 0; q < DP / 4; ++q) {
    const float4 v = *reinterpret_cast<const float4*>(p + 4 * q);
    if (4 * q + 0 < D) x[4 * q + 0] = v.x;
    if (4 * q + 1 < D) x[4 * q + 1] = v.y;
    if (4 * q + 2 < D) x[4 * q + 2] = v.z;
    if (4 * q + 3 < D) x[4 * q + 3] = v.w;
  }
}

// A operand of one 16 x 32 kernel tile: the lane's row against its 8 columns,
// rounded to bf16 (hi, RNE) and, for BF16X3, the bf16 rounding of the remainder.
template <int MODE, int D>
__device__ __forceinline__ void tile_a(const float (&xi)[D], const float (&xj)[8][D], bf16x8& ah,
                                       bf16x8& al) {
#pragma unroll
  for (int e = 0; e < 8; e += 2) {
    const float m0 = matern_r2(sqdist<D>(xi, xj[e]));
    const float m1 = matern_r2(sqdist<D>(xi, xj[e + 1]));
    const bf16x2 h = __builtin_convertvector((f32x2){m0, m1}, bf16x2);
    ah[e] = h[0];
    ah[e + 1] = h[1];
    if (MODE == P_BF16X3) {
      const uint32_t hb = __builtin_bit_cast(uint32_t, h);
      const float h0 = __builtin_bit_cast(float, hb << 16);
      const float h1 = __builtin_bit_cast(float, hb & 0xffff0000u);
      const bf16x2 l = __builtin_convertvector((f32x2){m0 - h0, m1 - h1}, bf16x2);
      al[e] = l[0];
      al[e + 1] = l[1];
    }
  }
}

// acc[ct] += A B[ct] for all column tiles; for BF16X3 the three partial products
// (lo*hi, hi*lo, hi*hi; small terms first) are issued as three passes over the
// tiles so that dependent accumulations into one tile are CT instructions apart.
template <int MODE, int CT>
__device__ __forceinline__ void mfma_tiles(f32x4 (&acc)[CT], const bf16x8& ah, const bf16x8& al,
                                           const bf16x8 (&bh)[CT], const bf16x8 (&bl)[CT]) {
  if (MODE == P_BF16X3) {
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
      acc[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[ct], acc[ct], 0, 0, 0);
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
      acc[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[ct], acc[ct], 0, 0, 0);
  }
#pragma unroll
  for (int ct = 0; ct < CT; ++ct)
    acc[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[ct], acc[ct], 0, 0, 0);
}

// Interleave NMFMA MFMAs with the VALU work of the same scheduling region.
template <int NMFMA, int NVALU>
__device__ __forceinline__ void interleave() {
#pragma unroll
  for (int i = 0; i < NMFMA; ++i) {
    __builtin_amdgcn_sched_group_barrier(kMaskMFMA, 1, 0);
    __builtin_amdgcn_sched_group_barrier(kMaskVALU, NVALU, 0);
  }
}

// One column step of the bf16 pipeline (see file comment).  xc/bh/bl/a0 hold
// step k; xn receives step k+1's coordinates, n0 the A operand of sub-tile 0
// for step k+1, and bh/bl are refilled with step k+1's V tiles.
template <int MODE, int D, int CT, int RS>
__device__ __forceinline__ void bf16_step(const float (&xi)[RS][D], const float (&xc)[8][D],
                                          float (&xn)[8][D], bf16x8 (&bh)[CT], bf16x8 (&bl)[CT],
                                          const bf16x8& a0h, const bf16x8& a0l, bf16x8& n0h,
                                          bf16x8& n0l, f32x4 (&acc)[RS][CT],
                                          const float* __restrict__ xnext,
                                          const uint16_t* __restrict__ vh_next,
                                          const uint16_t* __restrict__ vl_next) {
  constexpr int DP = (D + 3) & ~3;
  constexpr int NM = (MODE == P_BF16X3 ? 3 : 1) * CT;
  constexpr int NV = (MODE == P_BF16X3 ? 6 : 12);
#pragma unroll
  for (int e = 0; e < 8; ++e) load_point<D>(xnext + e * DP, xn[e]);
  // sub-tiles 0..RS-2: A(r+1, k) on the VALU while acc[r] accumulates
  bf16x8 ah = a0h, al = a0l;
#pragma unroll
  for (int r = 0; r + 1 < RS; ++r) {
    bf16x8 nh, nl;
    tile_a<MODE, D>(xi[r + 1], xc, nh, nl);
    mfma_tiles<MODE, CT>(acc[r], ah, al, bh, bl);
    if (r == 0) __builtin_amdgcn_sched_group_barrier(kMaskVMEMRead, 2 * D, 0);
    interleave<NM, NV>();
    __builtin_amdgcn_sched_barrier(0);
    ah = nh;
    al = nl;
  }
  // last sub-tile: A(0, k+1) on the VALU while acc[RS-1] accumulates; V refilled
  tile_a<MODE, D>(xi[0], xn, n0h, n0l);
  if (MODE == P_BF16X3) {
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
      acc[RS - 1][ct] =
          __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[ct], acc[RS - 1][ct], 0, 0, 0);
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      acc[RS - 1][ct] =
          __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[ct], acc[RS - 1][ct], 0, 0, 0);
      bl[ct] = *reinterpret_cast<const bf16x8*>(vl_next + ct * 512);
    }
  }
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    acc[RS - 1][ct] =
        __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[ct], acc[RS - 1][ct], 0, 0, 0);
    bh[ct] = *reinterpret_cast<const bf16x8*>(vh_next + ct * 512);
  }
  interleave<NM, NV>();
  __builtin_amdgcn_sched_barrier(0);
}

template <int CT, int RS>
__device__ __forceinline__ void epilogue(const f32x4 (&acc)[RS][CT], int64_t row0, int l16, int g,
                                         int64_t n1, int64_t n1_pad, int c, int S, int64_t sp,
                                         float* __restrict__ out, int64_t ldo,
                                         float* __restrict__ part, float scale,
                                         const float* __restrict__ vn, int64_t ldv,
                                         float noise) {
#pragma unroll
  for (int rs = 0; rs < RS; ++rs)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t row = row0 + rs * 16 + 4 * g + q;
        const int col = ct * 16 + l16;
        if (S == 1) {
          if (row < n1 && col < c) {
            float v = scale * acc[rs][ct][q];
            if (vn) v = __builtin_fmaf(noise, vn[row * ldv + col], v);
            out[row * ldo + col] = v;
          }
        } else {
          part[(sp * n1_pad + row) * (16 * CT) + col] = acc[rs][ct][q];
        }
      }
}

template <int CT, int RS>
__device__ __forceinline__ void zero(f32x4 (&a)[RS][CT]) {
#pragma unroll
  for (int rs = 0; rs < RS; ++rs)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) a[rs][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
}

// Running totals of the two-level summation live in a wave-private LDS slice
// ([RS * CT * 4 values][64 lanes], lane-contiguous, so no bank conflicts and no
// barriers) instead of 4*RS*CT extra VGPRs, which keeps occupancy up.
template <int CT, int RS>
__device__ __forceinline__ void fold(float* __restrict__ tl, f32x4 (&acc)[RS][CT], int lane) {
#pragma unroll
  for (int rs = 0; rs < RS; ++rs)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        tl[((rs * CT + ct) * 4 + q) * 64 + lane] += acc[rs][ct][q];
        acc[rs][ct][q] = 0.f;
      }
}

template <int CT, int RS>
__device__ __forceinline__ void tot_init(float* __restrict__ tl, int lane) {
#pragma unroll
  for (int k = 0; k < RS * CT * 4; ++k) tl[k * 64 + lane] = 0.f;
}

template <int CT, int RS>
__device__ __forceinline__ void tot_read(const float* __restrict__ tl, f32x4 (&tot)[RS][CT],
                                         int lane) {
#pragma unroll
  for (int rs = 0; rs < RS; ++rs)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int q = 0; q < 4; ++q) tot[rs][ct][q] = tl[((rs * CT + ct) * 4 + q) * 64 + lane];
}

template <int MODE, int D, int CT, int RS>
__global__ __launch_bounds__(256, 2) void kfwd_bf16(
    const float* __restrict__ xp1, const float* __restrict__ xp2,
    const uint16_t* __restrict__ vhi, const uint16_t* __restrict__ vlo, int64_t n1,
    int64_t n1_pad, int64_t steps, int S, float* __restrict__ out, int64_t ldo, int c,
    float* __restrict__ part, float scale, const float* __restrict__ vn, int64_t ldv,
    float noise) {
  constexpr int DP = (D + 3) & ~3;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int l16 = lane & 15;
  const int g = lane >> 4;
  const int64_t rb = blockIdx.x / S;
  const int64_t sp = blockIdx.x % S;
  const int64_t row0 = rb * (64 * RS) + wave * (16 * RS);
  const int64_t s0 = steps * sp / S;
  const int64_t s1 = steps * (sp + 1) / S;

  float xi[RS][D];
#pragma unroll
  for (int rs = 0; rs < RS; ++rs) load_point<D>(xp1 + (row0 + rs * 16 + l16) * DP, xi[rs]);

  __shared__ float tot_lds[4][RS * CT * 4 * 64];
  float* tl = tot_lds[wave];
  tot_init<CT, RS>(tl, lane);
  f32x4 acc[RS][CT];
  zero<CT, RS>(acc);

  if (s0 < s1) {
    // per-lane offsets: coordinates of columns 8g..8g+7, V tile element (col l16, rows 8g..)
    const float* xb = xp2 + 8 * g * DP;
    const int64_t voff = l16 * 32 + 8 * g;
    const int64_t tstride = (int64_t)CT * 512;
    float X0[8][D], X1[8][D];
    bf16x8 bh[CT], bl[CT];
    bf16x8 A0h, A0l, A1h, A1l;
#pragma unroll
    for (int e = 0; e < 8; ++e) load_point<D>(xb + (s0 * kJStep + e) * DP, X0[e]);
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      bh[ct] = *reinterpret_cast<const bf16x8*>(vhi + s0 * tstride + voff + ct * 512);
      if (MODE == P_BF16X3)
        bl[ct] = *reinterpret_cast<const bf16x8*>(vlo + s0 * tstride + voff + ct * 512);
    }
    tile_a<MODE, D>(xi[0], X0, A0h, A0l);
    int64_t st = s0;
    int left = kChunk;
    while (true) {
      int64_t nx = st + 1 < s1 ? st + 1 : st;
      bf16_step<MODE, D, CT, RS>(xi, X0, X1, bh, bl, A0h, A0l, A1h, A1l, acc,
                             xb + nx * kJStep * DP, vhi + nx * tstride + voff,
                             vlo + nx * tstride + voff);
      if (++st >= s1) break;
      if (--left == 0) {
        fold<CT, RS>(tl, acc, lane);
        left = kChunk;
      }
      nx = st + 1 < s1 ? st + 1 : st;
      bf16_step<MODE, D, CT, RS>(xi, X1, X0, bh, bl, A1h, A1l, A0h, A0l, acc,
                             xb + nx * kJStep * DP, vhi + nx * tstride + voff,
                             vlo + nx * tstride + voff);
      if (++st >= s1) break;
      if (--left == 0) {
        fold<CT, RS>(tl, acc, lane);
        left = kChunk;
      }
    }
    fold<CT, RS>(tl, acc, lane);
  }
  f32x4 tot[RS][CT];
  tot_read<CT, RS>(tl, tot, lane);
  epilogue<CT, RS>(tot, row0, l16, g, n1, n1_pad, c, S, sp, out, ldo, part, scale, vn, ldv, noise);
}

// ---------------------------------------------------------------------------
// Cross-term path (bf16 modes, any d with every scaled point's |x^|^2 bounded).
// Points are packed chunk-major, xt[q][i][0..3] for q < NK = ceil((d+1)/4):
// coordinates in slots 0..d-1, |x^|^2 in the last slot 4NK-1, zeros between.
// With A'[j] = [-2 x^_j, |x^_j|^2] and B'[i] = [x^_i, 1], NK chained
// v_mfma_f32_16x16x4_f32 with |x^_i|^2 as the accumulator input give r^2 for a
// 16 x 16 block, so the VALU only evaluates the Matern function and splits it,
// each lane loads NK scalars per 16 columns (coalesced: lanes of a chunk read 64
// consecutive floats), and no coordinates are held in registers beyond the NK
// operands of the lane's rows.  The product's output layout gives each lane rows
// j = 4g..4g+3 (and 16 + 4g..) of one column i, so the V tiles are packed with the
// matching row permutation (xt_j_of_k in vec.hip).  The FP32 cancellation error
// in r^2 grows with |x^|^2; the library uses this path only while the norms stay
// within the bounds of gpk.h (kXTMaxNorm2 and its companions) and otherwise the
// direct path.
template <int MODE, int NK>
__device__ __forceinline__ void tile_a_xt(const float (&bx)[NK], float ni, const float (&ajl)[NK],
                                          const float (&ajh)[NK], bf16x8& ah, bf16x8& al) {
  // |x^_i|^2 enters as the accumulator input; a slightly negative r^2 left by
  // cancellation is taken by magnitude (a free source modifier), which perturbs
  // m by the same O(|r^2 error|) as clamping at zero would
  f32x4 d0 = {ni, ni, ni, ni};
  f32x4 d1 = d0;
#pragma unroll
  for (int q = 0; q < NK; ++q) {
    d0 = __builtin_amdgcn_mfma_f32_16x16x4f32(ajl[q], bx[q], d0, 0, 0, 0);
    d1 = __builtin_amdgcn_mfma_f32_16x16x4f32(ajh[q], bx[q], d1, 0, 0, 0);
  }
  float r2[8];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    r2[q] = __builtin_fabsf(d0[q]);
    r2[4 + q] = __builtin_fabsf(d1[q]);
  }
#pragma unroll
  for (int e = 0; e < 8; e += 2) {
    const float m0 = matern_r2(r2[e]);
    const float m1 = matern_r2(r2[e + 1]);
    const bf16x2 h = __builtin_convertvector((f32x2){m0, m1}, bf16x2);
    ah[e] = h[0];
    ah[e + 1] = h[1];
    if (MODE == P_BF16X3) {
      const uint32_t hb = __builtin_bit_cast(uint32_t, h);
      const float h0 = __builtin_bit_cast(float, hb << 16);
      const float h1 = __builtin_bit_cast(float, hb & 0xffff0000u);
      const bf16x2 l = __builtin_convertvector((f32x2){m0 - h0, m1 - h1}, bf16x2);
      al[e] = l[0];
      al[e + 1] = l[1];
    }
  }
}

// A' operand of column rows j (lane's j = l%16 of each half) for the NK chunks,
// scaled by -2 except in the norm slot.
template <int NK>
__device__ __forceinline__ void load_cols_xt(const float* __restrict__ xb, int64_t cstride,
                                             int g, float (&jl)[NK], float (&jh)[NK]) {
#pragma unroll
  for (int q = 0; q < NK; ++q) {
    const float mult = (q == NK - 1 && g == 3) ? 1.f : -2.f;
    jl[q] = xb[q * cstride] * mult;
    jh[q] = xb[q * cstride + 16 * 4] * mult;
  }
}

template <int MODE, int CT, int RS, int NK>
__device__ __forceinline__ void bf16_step_xt(const float (&bx)[RS][NK], const float (&ni)[RS],
                                             const float (&ajl)[NK], const float (&ajh)[NK],
                                             float (&njl)[NK], float (&njh)[NK],
                                             bf16x8 (&bh)[CT], bf16x8 (&bl)[CT],
                                             const bf16x8& a0h, const bf16x8& a0l, bf16x8& n0h,
                                             bf16x8& n0l, f32x4 (&acc)[RS][CT],
                                             const float* __restrict__ xnext, int64_t cstride,
                                             int g, const uint16_t* __restrict__ vh_next,
                                             const uint16_t* __restrict__ vl_next) {
  float rl[NK], rh[NK];
  load_cols_xt<NK>(xnext, cstride, g, rl, rh);
  bf16x8 ah = a0h, al = a0l;
#pragma unroll
  for (int r = 0; r + 1 < RS; ++r) {
    bf16x8 nh, nl;
    tile_a_xt<MODE, NK>(bx[r + 1], ni[r + 1], ajl, ajh, nh, nl);
    mfma_tiles<MODE, CT>(acc[r], ah, al, bh, bl);
    __builtin_amdgcn_sched_barrier(0);
    ah = nh;
    al = nl;
  }
#pragma unroll
  for (int q = 0; q < NK; ++q) {
    njl[q] = rl[q];
    njh[q] = rh[q];
  }
  tile_a_xt<MODE, NK>(bx[0], ni[0], njl, njh, n0h, n0l);
  if (MODE == P_BF16X3) {
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
      acc[RS - 1][ct] =
          __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[ct], acc[RS - 1][ct], 0, 0, 0);
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      acc[RS - 1][ct] =
          __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[ct], acc[RS - 1][ct], 0, 0, 0);
      bl[ct] = *reinterpret_cast<const bf16x8*>(vl_next + ct * 512);
    }
  }
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    acc[RS - 1][ct] =
        __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[ct], acc[RS - 1][ct], 0, 0, 0);
    bh[ct] = *reinterpret_cast<const bf16x8*>(vh_next + ct * 512);
  }
  __builtin_amdgcn_sched_barrier(0);
}

template <int MODE, int CT, int RS, int NK>
__global__ __launch_bounds__(256, 2) void kfwd_bf16_xt(
    const float* __restrict__ xt1, const float* __restrict__ xt2, int64_t n2_pad,
    const uint16_t* __restrict__ vhi, const uint16_t* __restrict__ vlo, int64_t n1,
    int64_t n1_pad, int64_t steps, int S, float* __restrict__ out, int64_t ldo, int c,
    float* __restrict__ part, float scale, const float* __restrict__ vn, int64_t ldv,
    float noise) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int l16 = lane & 15;
  const int g = lane >> 4;
  const int64_t rb = blockIdx.x / S;
  const int64_t sp = blockIdx.x % S;
  const int64_t row0 = rb * (64 * RS) + wave * (16 * RS);
  const int64_t s0 = steps * sp / S;
  const int64_t s1 = steps * (sp + 1) / S;
  const int64_t rstride = n1_pad * 4;  // floats per chunk of the row points
  const int64_t cstride = n2_pad * 4;  // floats per chunk of the column points

  // B' operand (k = g of every chunk) and |x^_i|^2 of this lane's row in every sub-tile
  float bx[RS][NK], ni[RS];
#pragma unroll
  for (int rs = 0; rs < RS; ++rs) {
    const float* pi = xt1 + (row0 + rs * 16 + l16) * 4;
#pragma unroll
    for (int q = 0; q < NK; ++q) bx[rs][q] = (q == NK - 1 && g == 3) ? 1.f : pi[q * rstride + g];
    ni[rs] = pi[(NK - 1) * rstride + 3];
  }

  __shared__ float tot_lds[4][RS * CT * 4 * 64];
  float* tl = tot_lds[wave];
  tot_init<CT, RS>(tl, lane);
  f32x4 acc[RS][CT];
  zero<CT, RS>(acc);

  if (s0 < s1) {
    const float* xb = xt2 + l16 * 4 + g;  // column j = 32 st + l16 (+16), slot g of each chunk
    const int64_t voff = l16 * 32 + 8 * g;
    const int64_t tstride = (int64_t)CT * 512;
    float J0l[NK], J0h[NK], J1l[NK], J1h[NK];
    bf16x8 bh[CT], bl[CT];
    bf16x8 A0h, A0l, A1h, A1l;
    load_cols_xt<NK>(xb + s0 * kJStep * 4, cstride, g, J0l, J0h);
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      bh[ct] = *reinterpret_cast<const bf16x8*>(vhi + s0 * tstride + voff + ct * 512);
      if (MODE == P_BF16X3)
        bl[ct] = *reinterpret_cast<const bf16x8*>(vlo + s0 * tstride + voff + ct * 512);
    }
    tile_a_xt<MODE, NK>(bx[0], ni[0], J0l, J0h, A0h, A0l);
    int64_t st = s0;
    int left = kChunk;
    while (true) {
      int64_t nx = st + 1 < s1 ? st + 1 : st;
      bf16_step_xt<MODE, CT, RS, NK>(bx, ni, J0l, J0h, J1l, J1h, bh, bl, A0h, A0l, A1h, A1l, acc,
                                     xb + nx * kJStep * 4, cstride, g, vhi + nx * tstride + voff,
                                     vlo + nx * tstride + voff);
      if (++st >= s1) break;
      if (--left == 0) {
        fold<CT, RS>(tl, acc, lane);
        left = kChunk;
      }
      nx = st + 1 < s1 ? st + 1 : st;
      bf16_step_xt<MODE, CT, RS, NK>(bx, ni, J1l, J1h, J0l, J0h, bh, bl, A1h, A1l, A0h, A0l, acc,
                                     xb + nx * kJStep * 4, cstride, g, vhi + nx * tstride + voff,
                                     vlo + nx * tstride + voff);
      if (++st >= s1) break;
      if (--left == 0) {
        fold<CT, RS>(tl, acc, lane);
        left = kChunk;
      }
    }
    fold<CT, RS>(tl, acc, lane);
  }
  f32x4 tot[RS][CT];
  tot_read<CT, RS>(tl, tot, lane);
  epilogue<CT, RS>(tot, row0, l16, g, n1, n1_pad, c, S, sp, out, ldo, part, scale, vn, ldv,
                   noise);
}

// FP32 pipeline: same structure with 8 scalar A operands per row sub-tile and
// 8 K=4 MFMAs per 16-column tile per step.
template <int D, int FN>
__device__ __forceinline__ void f32_vals(const float (&xi)[D], const float (&xj)[8][D], int fd,
                                         float (&m)[8]) {
#pragma unroll
  for (int kk = 0; kk < 8; ++kk)
    m[kk] = (FN == FN_MATERN) ? matern_r2(sqdist<D>(xi, xj[kk])) : dlen_val<D>(xi, xj[kk], fd);
}

template <int D, int CT, int FN, int RS>
__device__ __forceinline__ void f32_step(const float (&xi)[RS][D], const float (&xc)[8][D],
                                         float (&xn)[8][D], float (&b)[CT][8],
                                         const float (&a0)[8], float (&n0)[8],
                                         f32x4 (&acc)[RS][CT], int fd,
                                         const float* __restrict__ xnext,
                                         const float* __restrict__ vnext) {
  constexpr int DP = (D + 3) & ~3;
#pragma unroll
  for (int kk = 0; kk < 8; ++kk) load_point<D>(xnext + 4 * kk * DP, xn[kk]);
  float a[8];
#pragma unroll
  for (int kk = 0; kk < 8; ++kk) a[kk] = a0[kk];
#pragma unroll
  for (int r = 0; r + 1 < RS; ++r) {
    float nx[8];
    f32_vals<D, FN>(xi[r + 1], xc, fd, nx);
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int kk = 0; kk < 8; ++kk)
        acc[r][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[kk], b[ct][kk], acc[r][ct], 0, 0, 0);
    if (r == 0) __builtin_amdgcn_sched_group_barrier(kMaskVMEMRead, 2 * D, 0);
    interleave<8 * CT, 2>();
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) a[kk] = nx[kk];
  }
  f32_vals<D, FN>(xi[0], xn, fd, n0);
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
#pragma unroll
    for (int kk = 0; kk < 8; ++kk)
      acc[RS - 1][ct] =
          __builtin_amdgcn_mfma_f32_16x16x4f32(a[kk], b[ct][kk], acc[RS - 1][ct], 0, 0, 0);
    const float4 lo4 = *reinterpret_cast<const float4*>(vnext + ct * 512);
    const float4 hi4 = *reinterpret_cast<const float4*>(vnext + ct * 512 + 4);
    b[ct][0] = lo4.x; b[ct][1] = lo4.y; b[ct][2] = lo4.z; b[ct][3] = lo4.w;
    b[ct][4] = hi4.x; b[ct][5] = hi4.y; b[ct][6] = hi4.z; b[ct][7] = hi4.w;
  }
  interleave<8 * CT, 2>();
  __builtin_amdgcn_sched_barrier(0);
}

template <int D, int CT, int FN, int RS>
__global__ __launch_bounds__(256, 2) void kfwd_f32(
    const float* __restrict__ xp1, const float* __restrict__ xp2, const float* __restrict__ vf,
    int64_t n1, int64_t n1_pad, int64_t steps, int S, float* __restrict__ out, int64_t ldo,
    int c, float* __restrict__ part, float scale, const float* __restrict__ vn, int64_t ldv,
    float noise, int fn_dim) {
  constexpr int DP = (D + 3) & ~3;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int l16 = lane & 15;
  const int g = lane >> 4;
  const int64_t rb = blockIdx.x / S;
  const int64_t sp = blockIdx.x % S;
  const int64_t row0 = rb * (64 * RS) + wave * (16 * RS);
  const int64_t s0 = steps * sp / S;
  const int64_t s1 = steps * (sp + 1) / S;

  float xi[RS][D];
#pragma unroll
  for (int rs = 0; rs < RS; ++rs) load_point<D>(xp1 + (row0 + rs * 16 + l16) * DP, xi[rs]);

  __shared__ float tot_lds[4][RS * CT * 4 * 64];
  float* tl = tot_lds[wave];
  tot_init<CT, RS>(tl, lane);
  f32x4 acc[RS][CT];
  zero<CT, RS>(acc);

  if (s0 < s1) {
    // per-lane offsets: columns g + 4 kk, V tile element (col l16, rows g + 4 kk)
    const float* xb = xp2 + g * DP;
    const int64_t voff = (l16 * 4 + g) * 8;
    const int64_t tstride = (int64_t)CT * 512;
    float X0[8][D], X1[8][D];
    float b[CT][8];
    float A0[8], A1[8];
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) load_point<D>(xb + (s0 * kJStep + 4 * kk) * DP, X0[kk]);
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const float* p = vf + s0 * tstride + voff + ct * 512;
      const float4 lo4 = *reinterpret_cast<const float4*>(p);
      const float4 hi4 = *reinterpret_cast<const float4*>(p + 4);
      b[ct][0] = lo4.x; b[ct][1] = lo4.y; b[ct][2] = lo4.z; b[ct][3] = lo4.w;
      b[ct][4] = hi4.x; b[ct][5] = hi4.y; b[ct][6] = hi4.z; b[ct][7] = hi4.w;
    }
    f32_vals<D, FN>(xi[0], X0, fn_dim, A0);
    int64_t st = s0;
    int left = kChunk;
    while (true) {
      int64_t nx = st + 1 < s1 ? st + 1 : st;
      f32_step<D, CT, FN, RS>(xi, X0, X1, b, A0, A1, acc, fn_dim, xb + nx * kJStep * DP,
                              vf + nx * tstride + voff);
      if (++st >= s1) break;
      if (--left == 0) {
        fold<CT, RS>(tl, acc, lane);
        left = kChunk;
      }
      nx = st + 1 < s1 ? st + 1 : st;
      f32_step<D, CT, FN, RS>(xi, X1, X0, b, A1, A0, acc, fn_dim, xb + nx * kJStep * DP,
                              vf + nx * tstride + voff);
      if (++st >= s1) break;
      if (--left == 0) {
        fold<CT, RS>(tl, acc, lane);
        left = kChunk;
      }
    }
    fold<CT, RS>(tl, acc, lane);
  }
  f32x4 tot[RS][CT];
  tot_read<CT, RS>(tl, tot, lane);
  epilogue<CT, RS>(tot, row0, l16, g, n1, n1_pad, c, S, sp, out, ldo, part, scale, vn, ldv,
                   noise);
}

// Direct FP32 kernel for wide points (D >= 8): the same arithmetic as kfwd_f32
// (identical kernel values and MFMA order), but the 32 column points of a step
// are staged once per workgroup in LDS (three buffers: the current step, the
// next one, whose sub-tile-0 operand is computed at the end of the current step,
// and the one being filled) instead of eight points per lane in registers, and
// two row sub-tiles per wave; at d = 12 that removes the register spills of the
// register-resident form and leaves LDS for three workgroups per CU.
template <int D, int FN>
__device__ __forceinline__ void f32_vals_lds(const float (&xi)[D], const float* xs, int g, int fd,
                                             float (&m)[8]) {
  constexpr int DP = (D + 3) & ~3;
#pragma unroll
  for (int kk = 0; kk < 8; ++kk) {
    float xj[D];
    const float* p = xs + (g + 4 * kk) * DP;
#pragma unroll
    for (int q = 0; q < DP / 4; ++q) {
      const float4 v = *reinterpret_cast<const float4*>(p + 4 * q);
      if (4 * q + 0 < D) xj[4 * q + 0] = v.x;
      if (4 * q + 1 < D) xj[4 * q + 1] = v.y;
      if (4 * q + 2 < D) xj[4 * q + 2] = v.z;
      if (4 * q + 3 < D) xj[4 * q + 3] = v.w;
    }
    m[kk] = (FN == FN_MATERN) ? matern_r2(sqdist<D>(xi, xj)) : dlen_val<D>(xi, xj, fd);
  }
}

template <int D, int CT, int FN, int RS>
__device__ __forceinline__ void f32_step_lds(const float (&xi)[RS][D], const float* xc,
                                             const float* xn, int g, float (&b)[CT][8],
                                             const float (&a0)[8], float (&n0)[8],
                                             f32x4 (&acc)[RS][CT], int fd,
                                             const float* __restrict__ vnext) {
  float a[8];
#pragma unroll
  for (int kk = 0; kk < 8; ++kk) a[kk] = a0[kk];
#pragma unroll
  for (int r = 0; r + 1 < RS; ++r) {
    float nx[8];
    f32_vals_lds<D, FN>(xi[r + 1], xc, g, fd, nx);
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int kk = 0; kk < 8; ++kk)
        acc[r][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[kk], b[ct][kk], acc[r][ct], 0, 0, 0);
    interleave<8 * CT, 2>();
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) a[kk] = nx[kk];
  }
  f32_vals_lds<D, FN>(xi[0], xn, g, fd, n0);
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
#pragma unroll
    for (int kk = 0; kk < 8; ++kk)
      acc[RS - 1][ct] =
          __builtin_amdgcn_mfma_f32_16x16x4f32(a[kk], b[ct][kk], acc[RS - 1][ct], 0, 0, 0);
    const float4 lo4 = *reinterpret_cast<const float4*>(vnext + ct * 512);
    const float4 hi4 = *reinterpret_cast<const float4*>(vnext + ct * 512 + 4);
    b[ct][0] = lo4.x; b[ct][1] = lo4.y; b[ct][2] = lo4.z; b[ct][3] = lo4.w;
    b[ct][4] = hi4.x; b[ct][5] = hi4.y; b[ct][6] = hi4.z; b[ct][7] = hi4.w;
  }
  interleave<8 * CT, 2>();
  __builtin_amdgcn_sched_barrier(0);
}

template <int D, int CT, int FN, int RS>
__global__ __launch_bounds__(256, 2) void kfwd_f32_lds(
    const float* __restrict__ xp1, const float* __restrict__ xp2, const float* __restrict__ vf,
    int64_t n1, int64_t n1_pad, int64_t steps, int S, float* __restrict__ out, int64_t ldo,
    int c, float* __restrict__ part, float scale, const float* __restrict__ vn, int64_t ldv,
    float noise, int fn_dim) {
  constexpr int DP = (D + 3) & ~3;
  constexpr int NV4 = 8 * DP;                     // float4s of one step's 32 points
  constexpr int NPF = (NV4 + 255) / 256;          // of them per thread
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int l16 = lane & 15;
  const int g = lane >> 4;
  const int64_t rb = blockIdx.x / S;
  const int64_t sp = blockIdx.x % S;
  const int64_t row0 = rb * (64 * RS) + wave * (16 * RS);
  const int64_t s0 = steps * sp / S;
  const int64_t s1 = steps * (sp + 1) / S;

  float xi[RS][D];
#pragma unroll
  for (int rs = 0; rs < RS; ++rs) load_point<D>(xp1 + (row0 + rs * 16 + l16) * DP, xi[rs]);

  __shared__ float tot_lds[4][RS * CT * 4 * 64];
  __shared__ __align__(16) float pts[3][32 * DP];
  float* tl = tot_lds[wave];
  tot_init<CT, RS>(tl, lane);
  f32x4 acc[RS][CT];
  zero<CT, RS>(acc);

  if (s0 < s1) {
    const int64_t voff = (l16 * 4 + g) * 8;
    const int64_t tstride = (int64_t)CT * 512;
    const float4* src = reinterpret_cast<const float4*>(xp2);  // step st: NV4 float4s from st * NV4
    // steps s0 and s0 + 1 into buffers 0 and 1, step s0 + 2 into the prefetch registers
    float4 pf[NPF];
#pragma unroll
    for (int u = 0; u < NPF; ++u) {
      const int e = tid + 256 * u;
      if (e < NV4) {
        reinterpret_cast<float4*>(pts[0])[e] = src[s0 * NV4 + e];
        if (s0 + 1 < s1) reinterpret_cast<float4*>(pts[1])[e] = src[(s0 + 1) * NV4 + e];
        if (s0 + 2 < s1) pf[u] = src[(s0 + 2) * NV4 + e];
      }
    }
    float b[CT][8];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const float* p = vf + s0 * tstride + voff + ct * 512;
      const float4 lo4 = *reinterpret_cast<const float4*>(p);
      const float4 hi4 = *reinterpret_cast<const float4*>(p + 4);
      b[ct][0] = lo4.x; b[ct][1] = lo4.y; b[ct][2] = lo4.z; b[ct][3] = lo4.w;
      b[ct][4] = hi4.x; b[ct][5] = hi4.y; b[ct][6] = hi4.z; b[ct][7] = hi4.w;
    }
    __syncthreads();
    float A0[8], A1[8];
    f32_vals_lds<D, FN>(xi[0], pts[0], g, fn_dim, A0);
    int64_t st = s0;
    int cur = 0;
    int left = kChunk;
    while (true) {
      // every wave is done with step st - 1: its buffer takes step st + 2
      __syncthreads();
      const int nxt = cur == 2 ? 0 : cur + 1;
      const int fil = nxt == 2 ? 0 : nxt + 1;
      if (st + 2 < s1) {
#pragma unroll
        for (int u = 0; u < NPF; ++u) {
          const int e = tid + 256 * u;
          if (e < NV4) {
            reinterpret_cast<float4*>(pts[fil])[e] = pf[u];
            if (st + 3 < s1) pf[u] = src[(st + 3) * NV4 + e];
          }
        }
      }
      const int64_t nx = st + 1 < s1 ? st + 1 : st;
      // the last step computes its successor's operand from its own points (unused)
      const float* xn = st + 1 < s1 ? pts[nxt] : pts[cur];
      if ((st - s0) & 1)
        f32_step_lds<D, CT, FN, RS>(xi, pts[cur], xn, g, b, A1, A0, acc, fn_dim,
                                    vf + nx * tstride + voff);
      else
        f32_step_lds<D, CT, FN, RS>(xi, pts[cur], xn, g, b, A0, A1, acc, fn_dim,
                                    vf + nx * tstride + voff);
      if (++st >= s1) break;
      cur = nxt;
      if (--left == 0) {
        fold<CT, RS>(tl, acc, lane);
        left = kChunk;
      }
    }
    fold<CT, RS>(tl, acc, lane);
  }
  f32x4 tot[RS][CT];
  tot_read<CT, RS>(tl, tot, lane);
  epilogue<CT, RS>(tot, row0, l16, g, n1, n1_pad, c, S, sp, out, ldo, part, scale, vn, ldv,
                   noise);
}

// FP32 cross-term kernel: r^2 as in kfwd_bf16_xt, then 8 K=4 FP32 MFMAs per
// 16-column tile and step with the lane's 8 kernel values as scalar A operands
// in the order the cross-term output leaves them (k = g of step kk holds column
// j = 4g + kk for kk < 4 and 16 + 4g + kk - 4 after), so the FP32 V tiles are
// packed with that row permutation.  Used under a tighter norm bound than the
// bf16 modes (the FP32 product's own error is smaller).
template <int NK>
__device__ __forceinline__ void f32_tile_xt(const float (&bx)[NK], float ni, const float (&ajl)[NK],
                                            const float (&ajh)[NK], float (&m)[8]) {
  f32x4 d0 = {ni, ni, ni, ni};
  f32x4 d1 = d0;
#pragma unroll
  for (int q = 0; q < NK; ++q) {
    d0 = __builtin_amdgcn_mfma_f32_16x16x4f32(ajl[q], bx[q], d0, 0, 0, 0);
    d1 = __builtin_amdgcn_mfma_f32_16x16x4f32(ajh[q], bx[q], d1, 0, 0, 0);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    m[q] = matern_r2(__builtin_fabsf(d0[q]));
    m[4 + q] = matern_r2(__builtin_fabsf(d1[q]));
  }
}

template <int CT, int RS, int NK>
__device__ __forceinline__ void f32_step_xt(const float (&bx)[RS][NK], const float (&ni)[RS],
                                            const float (&ajl)[NK], const float (&ajh)[NK],
                                            float (&njl)[NK], float (&njh)[NK], float (&b)[CT][8],
                                            const float (&a0)[8], float (&n0)[8],
                                            f32x4 (&acc)[RS][CT],
                                            const float* __restrict__ xnext, int64_t cstride,
                                            int g, const float* __restrict__ vnext) {
  float rl[NK], rh[NK];
  load_cols_xt<NK>(xnext, cstride, g, rl, rh);
  float a[8];
#pragma unroll
  for (int kk = 0; kk < 8; ++kk) a[kk] = a0[kk];
#pragma unroll
  for (int r = 0; r + 1 < RS; ++r) {
    float nx[8];
    f32_tile_xt<NK>(bx[r + 1], ni[r + 1], ajl, ajh, nx);
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int kk = 0; kk < 8; ++kk)
        acc[r][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[kk], b[ct][kk], acc[r][ct], 0, 0, 0);
    interleave<8 * CT + 2 * NK, 2>();
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) a[kk] = nx[kk];
  }
#pragma unroll
  for (int q = 0; q < NK; ++q) {
    njl[q] = rl[q];
    njh[q] = rh[q];
  }
  f32_tile_xt<NK>(bx[0], ni[0], njl, njh, n0);
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
#pragma unroll
    for (int kk = 0; kk < 8; ++kk)
      acc[RS - 1][ct] =
          __builtin_amdgcn_mfma_f32_16x16x4f32(a[kk], b[ct][kk], acc[RS - 1][ct], 0, 0, 0);
    const float4 lo4 = *reinterpret_cast<const float4*>(vnext + ct * 512);
    const float4 hi4 = *reinterpret_cast<const float4*>(vnext + ct * 512 + 4);
    b[ct][0] = lo4.x; b[ct][1] = lo4.y; b[ct][2] = lo4.z; b[ct][3] = lo4.w;
    b[ct][4] = hi4.x; b[ct][5] = hi4.y; b[ct][6] = hi4.z; b[ct][7] = hi4.w;
  }
  interleave<8 * CT + 2 * NK, 2>();
  __builtin_amdgcn_sched_barrier(0);
}

template <int CT, int RS, int NK>
__global__ __launch_bounds__(256, 2) void kfwd_f32_xt(
    const float* __restrict__ xt1, const float* __restrict__ xt2, int64_t n2_pad,
    const float* __restrict__ vf, int64_t n1, int64_t n1_pad, int64_t steps, int S,
    float* __restrict__ out, int64_t ldo, int c, float* __restrict__ part, float scale,
    const float* __restrict__ vn, int64_t ldv, float noise) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int l16 = lane & 15;
  const int g = lane >> 4;
  const int64_t rb = blockIdx.x / S;
  const int64_t sp = blockIdx.x % S;
  const int64_t row0 = rb * (64 * RS) + wave * (16 * RS);
  const int64_t s0 = steps * sp / S;
  const int64_t s1 = steps * (sp + 1) / S;
  const int64_t rstride = n1_pad * 4;
  const int64_t cstride = n2_pad * 4;

  float bx[RS][NK], ni[RS];
#pragma unroll
  for (int rs = 0; rs < RS; ++rs) {
    const float* pi = xt1 + (row0 + rs * 16 + l16) * 4;
#pragma unroll
    for (int q = 0; q < NK; ++q) bx[rs][q] = (q == NK - 1 && g == 3) ? 1.f : pi[q * rstride + g];
    ni[rs] = pi[(NK - 1) * rstride + 3];
  }

  __shared__ float tot_lds[4][RS * CT * 4 * 64];
  float* tl = tot_lds[wave];
  tot_init<CT, RS>(tl, lane);
  f32x4 acc[RS][CT];
  zero<CT, RS>(acc);

  if (s0 < s1) {
    const float* xb = xt2 + l16 * 4 + g;
    const int64_t voff = (l16 * 4 + g) * 8;
    const int64_t tstride = (int64_t)CT * 512;
    float J0l[NK], J0h[NK], J1l[NK], J1h[NK];
    float b[CT][8];
    float A0[8], A1[8];
    load_cols_xt<NK>(xb + s0 * kJStep * 4, cstride, g, J0l, J0h);
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const float* p = vf + s0 * tstride + voff + ct * 512;
      const float4 lo4 = *reinterpret_cast<const float4*>(p);
      const float4 hi4 = *reinterpret_cast<const float4*>(p + 4);
      b[ct][0] = lo4.x; b[ct][1] = lo4.y; b[ct][2] = lo4.z; b[ct][3] = lo4.w;
      b[ct][4] = hi4.x; b[ct][5] = hi4.y; b[ct][6] = hi4.z; b[ct][7] = hi4.w;
    }
    f32_tile_xt<NK>(bx[0], ni[0], J0l, J0h, A0);
    int64_t st = s0;
    int left = kChunk;
    while (true) {
      int64_t nx = st + 1 < s1 ? st + 1 : st;
      f32_step_xt<CT, RS, NK>(bx, ni, J0l, J0h, J1l, J1h, b, A0, A1, acc, xb + nx * kJStep * 4,
                              cstride, g, vf + nx * tstride + voff);
      if (++st >= s1) break;
      if (--left == 0) {
        fold<CT, RS>(tl, acc, lane);
        left = kChunk;
      }
      nx = st + 1 < s1 ? st + 1 : st;
      f32_step_xt<CT, RS, NK>(bx, ni, J1l, J1h, J0l, J0h, b, A1, A0, acc, xb + nx * kJStep * 4,
                              cstride, g, vf + nx * tstride + voff);
      if (++st >= s1) break;
      if (--left == 0) {
        fold<CT, RS>(tl, acc, lane);
        left = kChunk;
      }
    }
    fold<CT, RS>(tl, acc, lane);
  }
  f32x4 tot[RS][CT];
  tot_read<CT, RS>(tl, tot, lane);
  epilogue<CT, RS>(tot, row0, l16, g, n1, n1_pad, c, S, sp, out, ldo, part, scale, vn, ldv,
                   noise);
}

template <int D, int CT>
hipError_t launch(const FwdArgs& a, hipStream_t st) {
  if (a.xt && a.prec == P_FP32 && a.fn == FN_MATERN) {
    constexpr int NK = xt_chunks(D);
    constexpr int RX = fwd_xt_row_subtiles(CT, NK);
    if (a.n1_pad % (64 * RX) || !a.xt1 || !a.xt2) return hipErrorInvalidValue;
    const dim3 gx((unsigned)(a.n1_pad / (64 * RX) * a.S));
    hipLaunchKernelGGL((kfwd_f32_xt<CT, RX, NK>), gx, dim3(256), 0, st, a.xt1, a.xt2, a.n2_pad,
                       (const float*)a.vhi, a.n1, a.n1_pad, a.steps, a.S, a.out, a.ldo, a.c,
                       a.part, a.scale, a.vn, a.ldv, a.noise);
    return hipGetLastError();
  }
  if (a.xt && a.prec != P_FP32) {
    constexpr int NK = xt_chunks(D);
    constexpr int RX = fwd_xt_row_subtiles(CT, NK);
    if (a.n1_pad % (64 * RX) || !a.xt1 || !a.xt2) return hipErrorInvalidValue;
    const dim3 gx((unsigned)(a.n1_pad / (64 * RX) * a.S));
    if (a.prec == P_BF16X3)
      hipLaunchKernelGGL((kfwd_bf16_xt<P_BF16X3, CT, RX, NK>), gx, dim3(256), 0, st, a.xt1, a.xt2,
                         a.n2_pad, (const uint16_t*)a.vhi, (const uint16_t*)a.vlo, a.n1,
                         a.n1_pad, a.steps, a.S, a.out, a.ldo, a.c, a.part, a.scale, a.vn,
                         a.ldv, a.noise);
    else
      hipLaunchKernelGGL((kfwd_bf16_xt<P_BF16, CT, RX, NK>), gx, dim3(256), 0, st, a.xt1, a.xt2,
                         a.n2_pad, (const uint16_t*)a.vhi, (const uint16_t*)a.vhi, a.n1,
                         a.n1_pad, a.steps, a.S, a.out, a.ldo, a.c, a.part, a.scale, a.vn,
                         a.ldv, a.noise);
    return hipGetLastError();
  }
  constexpr int RS = fwd_row_subtiles(CT);
  if (a.n1_pad % (64 * RS)) return hipErrorInvalidValue;
  const dim3 grid((unsigned)(a.n1_pad / (64 * RS) * a.S));
  if (a.prec == P_BF16X3) {
    hipLaunchKernelGGL((kfwd_bf16<P_BF16X3, D, CT, RS>), grid, dim3(256), 0, st, a.xp1, a.xp2,
                       (const uint16_t*)a.vhi, (const uint16_t*)a.vlo, a.n1, a.n1_pad, a.steps,
                       a.S, a.out, a.ldo, a.c, a.part, a.scale, a.vn, a.ldv, a.noise);
  } else if (a.prec == P_BF16) {
    hipLaunchKernelGGL((kfwd_bf16<P_BF16, D, CT, RS>), grid, dim3(256), 0, st, a.xp1, a.xp2,
                       (const uint16_t*)a.vhi, (const uint16_t*)a.vhi, a.n1, a.n1_pad, a.steps,
                       a.S, a.out, a.ldo, a.c, a.part, a.scale, a.vn, a.ldv, a.noise);
  } else if (D >= 8) {
    constexpr int RL = 2;
    if (a.n1_pad % (64 * RL)) return hipErrorInvalidValue;
    const dim3 gl((unsigned)(a.n1_pad / (64 * RL) * a.S));
    if (a.fn == FN_MATERN)
      hipLaunchKernelGGL((kfwd_f32_lds<D, CT, FN_MATERN, RL>), gl, dim3(256), 0, st, a.xp1, a.xp2,
                         (const float*)a.vhi, a.n1, a.n1_pad, a.steps, a.S, a.out, a.ldo, a.c,
                         a.part, a.scale, a.vn, a.ldv, a.noise, a.fn_dim);
    else
      hipLaunchKernelGGL((kfwd_f32_lds<D, CT, FN_DLEN, RL>), gl, dim3(256), 0, st, a.xp1, a.xp2,
                         (const float*)a.vhi, a.n1, a.n1_pad, a.steps, a.S, a.out, a.ldo, a.c,
                         a.part, a.scale, a.vn, a.ldv, a.noise, a.fn_dim);
  } else if (a.fn == FN_MATERN) {
    hipLaunchKernelGGL((kfwd_f32<D, CT, FN_MATERN, RS>), grid, dim3(256), 0, st, a.xp1, a.xp2,
                       (const float*)a.vhi, a.n1, a.n1_pad, a.steps, a.S, a.out, a.ldo, a.c,
                       a.part, a.scale, a.vn, a.ldv, a.noise, a.fn_dim);
  } else {
    hipLaunchKernelGGL((kfwd_f32<D, CT, FN_DLEN, RS>), grid, dim3(256), 0, st, a.xp1, a.xp2,
                       (const float*)a.vhi, a.n1, a.n1_pad, a.steps, a.S, a.out, a.ldo, a.c,
                       a.part, a.scale, a.vn, a.ldv, a.noise, a.fn_dim);
  }
  return hipGetLastError();
}

template <int D>
hipError_t dispatch_ct(const FwdArgs& a, hipStream_t st) {
  switch (a.CT) {
    case 1: return launch<D, 1>(a, st);
    case 2: return launch<D, 2>(a, st);
    case 3: return launch<D, 3>(a, st);
    case 5: return launch<D, 5>(a, st);
    case 8: return launch<D, 8>(a, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

// This file is compiled once per template dimension (GPK_D = 1, 2, 3, 4, 8,
// 12, 16, 24, 32, 64) so that the instantiations build in parallel; the
// dispatcher that picks one lives in dispatch.hip.
#ifndef GPK_D
#error "compile with -DGPK_D=<dimension>"
#endif
#define GPK_CAT2(a, b) a##b
#define GPK_CAT(a, b) GPK_CAT2(a, b)
hipError_t GPK_CAT(fwd_d, GPK_D)(const FwdArgs& a, hipStream_t st) {
  return dispatch_ct<GPK_D>(a, st);
}

}  // namespace gpk
