// Fused matrix-free kernel-matrix product  out = scale * M(X1, X2) V (+ noise * V1).
//
// M is the Matern-3/2 kernel without its a^2 factor, evaluated in registers and
// never stored (the paper's regularised kernel matrix, Sec. 2; App. B counts
// one "epoch" as computing every entry once).  Work split:
//
//   * one workgroup = 4 waves = 128 output rows; every wave owns 2 row
//     sub-tiles of 16 rows and streams the kernel columns j in steps of 32;
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
// For small n the column range is split over S workgroups per row block and a
// second kernel sums the S partial tiles in a fixed order (deterministic).
#include "gpk.h"

namespace gpk {

namespace {

typedef float f32x8 __attribute__((ext_vector_type(8)));

constexpr int kChunk = 64;  // column steps (x 32 columns) per partial accumulator

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

template <int CT>
__device__ __forceinline__ void epilogue(const f32x4 (&acc)[2][CT], int64_t row0, int l16, int g,
                                         int64_t n1, int64_t n1_pad, int c, int S, int64_t sp,
                                         float* __restrict__ out, int64_t ldo,
                                         float* __restrict__ part, float scale,
                                         const float* __restrict__ vn, int64_t ldv,
                                         float noise) {
#pragma unroll
  for (int rs = 0; rs < 2; ++rs)
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

template <int MODE, int D, int CT>
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
  const int64_t row0 = rb * kFwdRowsPerWG + wave * 32;
  const int64_t s0 = steps * sp / S;
  const int64_t s1 = steps * (sp + 1) / S;

  float xi[2][D];
#pragma unroll
  for (int rs = 0; rs < 2; ++rs) load_point<D>(xp1 + (row0 + rs * 16 + l16) * DP, xi[rs]);

  f32x4 tot[2][CT], acc[2][CT];
#pragma unroll
  for (int rs = 0; rs < 2; ++rs)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) tot[rs][ct] = f32x4{0.f, 0.f, 0.f, 0.f};

  // Two-level summation: a fresh accumulator per chunk of kChunk column steps,
  // folded into the running total, keeps FP32 chains short at large n.
  for (int64_t c0 = s0; c0 < s1; c0 += kChunk) {
  const int64_t c1 = c0 + kChunk < s1 ? c0 + kChunk : s1;
#pragma unroll
  for (int rs = 0; rs < 2; ++rs)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[rs][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int64_t st = c0; st < c1; ++st) {
    float xj[8][D];
    const float* xb = xp2 + (st * kJStep + 8 * g) * DP;
#pragma unroll
    for (int e = 0; e < 8; ++e) load_point<D>(xb + e * DP, xj[e]);
    const int64_t toff = st * CT * 512 + l16 * 32 + 8 * g;
    bf16x8 bh[CT], bl[CT];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      bh[ct] = *reinterpret_cast<const bf16x8*>(vhi + toff + ct * 512);
      if (MODE == P_BF16X3) bl[ct] = *reinterpret_cast<const bf16x8*>(vlo + toff + ct * 512);
    }
#pragma unroll
    for (int rs = 0; rs < 2; ++rs) {
      f32x8 m;
#pragma unroll
      for (int e = 0; e < 8; ++e) m[e] = matern_r2(sqdist<D>(xi[rs], xj[e]));
      const bf16x8 ah = __builtin_convertvector(m, bf16x8);
      bf16x8 al;
      if (MODE == P_BF16X3) al = __builtin_convertvector(m - __builtin_convertvector(ah, f32x8), bf16x8);
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        if (MODE == P_BF16X3) {
          acc[rs][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[ct], acc[rs][ct], 0, 0, 0);
          acc[rs][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[ct], acc[rs][ct], 0, 0, 0);
        }
        acc[rs][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[ct], acc[rs][ct], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int rs = 0; rs < 2; ++rs)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) tot[rs][ct] += acc[rs][ct];
  }
  epilogue<CT>(tot, row0, l16, g, n1, n1_pad, c, S, sp, out, ldo, part, scale, vn, ldv, noise);
}

template <int D, int CT, int FN>
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
  const int64_t row0 = rb * kFwdRowsPerWG + wave * 32;
  const int64_t s0 = steps * sp / S;
  const int64_t s1 = steps * (sp + 1) / S;

  float xi[2][D];
#pragma unroll
  for (int rs = 0; rs < 2; ++rs) load_point<D>(xp1 + (row0 + rs * 16 + l16) * DP, xi[rs]);

  f32x4 tot[2][CT], acc[2][CT];
#pragma unroll
  for (int rs = 0; rs < 2; ++rs)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) tot[rs][ct] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int64_t c0 = s0; c0 < s1; c0 += kChunk) {
  const int64_t c1 = c0 + kChunk < s1 ? c0 + kChunk : s1;
#pragma unroll
  for (int rs = 0; rs < 2; ++rs)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[rs][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int64_t st = c0; st < c1; ++st) {
    float xj[8][D];
    const float* xb = xp2 + (st * kJStep + g) * DP;
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) load_point<D>(xb + 4 * kk * DP, xj[kk]);
    float b[CT][8];
    const float* tb = vf + st * CT * 512 + (l16 * 4 + g) * 8;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const float4 lo4 = *reinterpret_cast<const float4*>(tb + ct * 512);
      const float4 hi4 = *reinterpret_cast<const float4*>(tb + ct * 512 + 4);
      b[ct][0] = lo4.x; b[ct][1] = lo4.y; b[ct][2] = lo4.z; b[ct][3] = lo4.w;
      b[ct][4] = hi4.x; b[ct][5] = hi4.y; b[ct][6] = hi4.z; b[ct][7] = hi4.w;
    }
#pragma unroll
    for (int rs = 0; rs < 2; ++rs)
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) {
        const float m = (FN == FN_MATERN) ? matern_r2(sqdist<D>(xi[rs], xj[kk]))
                                          : dlen_val<D>(xi[rs], xj[kk], fn_dim);
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
          acc[rs][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(m, b[ct][kk], acc[rs][ct], 0, 0, 0);
      }
  }
#pragma unroll
  for (int rs = 0; rs < 2; ++rs)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) tot[rs][ct] += acc[rs][ct];
  }
  epilogue<CT>(tot, row0, l16, g, n1, n1_pad, c, S, sp, out, ldo, part, scale, vn, ldv, noise);
}

template <int D, int CT>
hipError_t launch(const FwdArgs& a, hipStream_t st) {
  const dim3 grid((unsigned)(a.n1_pad / kFwdRowsPerWG * a.S));
  if (a.prec == P_BF16X3) {
    hipLaunchKernelGGL((kfwd_bf16<P_BF16X3, D, CT>), grid, dim3(256), 0, st, a.xp1, a.xp2,
                       (const uint16_t*)a.vhi, (const uint16_t*)a.vlo, a.n1, a.n1_pad, a.steps,
                       a.S, a.out, a.ldo, a.c, a.part, a.scale, a.vn, a.ldv, a.noise);
  } else if (a.prec == P_BF16) {
    hipLaunchKernelGGL((kfwd_bf16<P_BF16, D, CT>), grid, dim3(256), 0, st, a.xp1, a.xp2,
                       (const uint16_t*)a.vhi, (const uint16_t*)a.vlo, a.n1, a.n1_pad, a.steps,
                       a.S, a.out, a.ldo, a.c, a.part, a.scale, a.vn, a.ldv, a.noise);
  } else if (a.fn == FN_MATERN) {
    hipLaunchKernelGGL((kfwd_f32<D, CT, FN_MATERN>), grid, dim3(256), 0, st, a.xp1, a.xp2,
                       (const float*)a.vhi, a.n1, a.n1_pad, a.steps, a.S, a.out, a.ldo, a.c,
                       a.part, a.scale, a.vn, a.ldv, a.noise, a.fn_dim);
  } else {
    hipLaunchKernelGGL((kfwd_f32<D, CT, FN_DLEN>), grid, dim3(256), 0, st, a.xp1, a.xp2,
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
