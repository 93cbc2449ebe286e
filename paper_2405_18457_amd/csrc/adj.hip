// Fused one-pass adjoint of the kernel-matrix product.
//
// For column weights w the gradient estimators need, for every hyperparameter,
//   g_k = sum_c w_c u_c^T (dK/dtheta_k) w_c = sum_ij G_ij dK_ij/dtheta_k,
//   G = U diag(w) W^T
// (Sec. 2 eq. mll_grad with the trace estimators of Sec. 2 eq. trace and
// Sec. 3 eq. pathwise_estimator).  This kernel never stores K or G: each wave
// owns 2 x 16 rows of U diag(w) (packed once into MFMA A operands) and streams
// W in steps of 16 columns; per step it forms the 16x16 tile of G on the
// matrix cores (bf16x3 or FP32 MFMA), recomputes the matching kernel tile in
// registers from the inputs, and accumulates
//   S_k = sum_ij G_ij 2^-rho_ij dhat_ijk^2   (k < d)   and   S_a = sum_ij G_ij m_ij
// in FP32 per lane, flushed to FP64 every 32 steps; FP64 wave / workgroup
// reductions write one partial row per workgroup, summed on the host.
//
// With pre-scaled inputs dhat_k = sqrt(3) log2(e) (x_k - x'_k) / ell_k:
//   dK/dell_k = 3 a^2 exp(-sqrt3 r) (x_k - x'_k)^2 / ell_k^3 = a^2 / (ell_k log2(e)^2) * 2^-rho dhat_k^2
//   dK/da     = 2 a m
// (the constant factors are applied on the host).
#include "gpk.h"

namespace gpk {

namespace {

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

template <int GM, int D, int KT>
__global__ __launch_bounds__(256, 2) void kadj(const float* __restrict__ xp, int64_t steps16,
                                               int S, const void* __restrict__ uhi_,
                                               const void* __restrict__ ulo_,
                                               const void* __restrict__ whi_,
                                               const void* __restrict__ wlo_,
                                               double* __restrict__ partial) {
  constexpr int DP = (D + 3) & ~3;
  constexpr int CK = 32 * KT;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int l16 = lane & 15;
  const int g = lane >> 4;
  const int64_t rb = blockIdx.x / S;
  const int64_t sp = blockIdx.x % S;
  const int64_t row0 = rb * kAdjRowsPerWG + wave * 32;
  const int64_t s0 = steps16 * sp / S;
  const int64_t s1 = steps16 * (sp + 1) / S;

  // A operands: rows row0 + rs*16 + l16 of U diag(w).
  bf16x8 ah[2][KT], al[2][KT];
  float af[2][KT][8];
  if (GM == P_BF16X3) {
    const uint16_t* uh = (const uint16_t*)uhi_;
    const uint16_t* ul = (const uint16_t*)ulo_;
#pragma unroll
    for (int rs = 0; rs < 2; ++rs)
#pragma unroll
      for (int kt = 0; kt < KT; ++kt) {
        const int64_t off = (row0 + rs * 16 + l16) * CK + 32 * kt + 8 * g;
        ah[rs][kt] = *reinterpret_cast<const bf16x8*>(uh + off);
        al[rs][kt] = *reinterpret_cast<const bf16x8*>(ul + off);
      }
  } else {
    const float* uf = (const float*)uhi_;
#pragma unroll
    for (int rs = 0; rs < 2; ++rs)
#pragma unroll
      for (int kt = 0; kt < KT; ++kt)
#pragma unroll
        for (int kk = 0; kk < 8; ++kk)
          af[rs][kt][kk] = uf[(row0 + rs * 16 + l16) * CK + 32 * kt + 4 * kk + g];
  }
  // Inputs of the 4 G rows this lane holds per sub-tile: rows 4g + q.
  float xi[2][4][D];
#pragma unroll
  for (int rs = 0; rs < 2; ++rs)
#pragma unroll
    for (int q = 0; q < 4; ++q) load_point<D>(xp + (row0 + rs * 16 + 4 * g + q) * DP, xi[rs][q]);

  float acc[D + 1];
  double dacc[D + 1];
#pragma unroll
  for (int k = 0; k <= D; ++k) {
    acc[k] = 0.f;
    dacc[k] = 0.0;
  }
  int since_flush = 0;

  for (int64_t st = s0; st < s1; ++st) {
    const int64_t j = st * 16 + l16;
    float xj[D];
    load_point<D>(xp + j * DP, xj);
    bf16x8 bh[KT], bl[KT];
    float bf[KT][8];
    if (GM == P_BF16X3) {
      const uint16_t* wh = (const uint16_t*)whi_;
      const uint16_t* wl = (const uint16_t*)wlo_;
#pragma unroll
      for (int kt = 0; kt < KT; ++kt) {
        bh[kt] = *reinterpret_cast<const bf16x8*>(wh + j * CK + 32 * kt + 8 * g);
        bl[kt] = *reinterpret_cast<const bf16x8*>(wl + j * CK + 32 * kt + 8 * g);
      }
    } else {
      const float* wf = (const float*)whi_;
#pragma unroll
      for (int kt = 0; kt < KT; ++kt)
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) bf[kt][kk] = wf[j * CK + 32 * kt + 4 * kk + g];
    }
#pragma unroll
    for (int rs = 0; rs < 2; ++rs) {
      f32x4 G = {0.f, 0.f, 0.f, 0.f};
      if (GM == P_BF16X3) {
#pragma unroll
        for (int kt = 0; kt < KT; ++kt) {
          G = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[rs][kt], bh[kt], G, 0, 0, 0);
          G = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[rs][kt], bl[kt], G, 0, 0, 0);
          G = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[rs][kt], bh[kt], G, 0, 0, 0);
        }
      } else {
#pragma unroll
        for (int kt = 0; kt < KT; ++kt)
#pragma unroll
          for (int kk = 0; kk < 8; ++kk)
            G = __builtin_amdgcn_mfma_f32_16x16x4f32(af[rs][kt][kk], bf[kt][kk], G, 0, 0, 0);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float dl[D];
        float r2 = 0.f;
#pragma unroll
        for (int k = 0; k < D; ++k) {
          dl[k] = xi[rs][q][k] - xj[k];
          r2 = __builtin_fmaf(dl[k], dl[k], r2);
        }
        const float rho = __builtin_amdgcn_sqrtf(r2);
        const float e = __builtin_amdgcn_exp2f(-rho);
        const float m = __builtin_fmaf(rho, kLn2, 1.0f) * e;
        const float P = G[q] * e;
#pragma unroll
        for (int k = 0; k < D; ++k) acc[k] = __builtin_fmaf(P * dl[k], dl[k], acc[k]);
        acc[D] = __builtin_fmaf(G[q], m, acc[D]);
      }
    }
    if (++since_flush == 32) {
#pragma unroll
      for (int k = 0; k <= D; ++k) {
        dacc[k] += (double)acc[k];
        acc[k] = 0.f;
      }
      since_flush = 0;
    }
  }
#pragma unroll
  for (int k = 0; k <= D; ++k) dacc[k] += (double)acc[k];

  // Wave reduction (FP64), then across the 4 waves through LDS.
  __shared__ double red[4][D + 1];
#pragma unroll
  for (int k = 0; k <= D; ++k) {
    double v = dacc[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) red[wave][k] = v;
  }
  __syncthreads();
  if (threadIdx.x <= D) {
    const int k = threadIdx.x;
    partial[(rb * S + sp) * (D + 1) + k] = red[0][k] + red[1][k] + red[2][k] + red[3][k];
  }
}

template <int GM, int D>
hipError_t launch_kt(const AdjArgs& a, int64_t rowblocks, hipStream_t st) {
  const dim3 grid((unsigned)(rowblocks * a.S));
  const int64_t steps16 = a.n_pad / 16;
#define GPK_ADJ_CASE(KTV)                                                                    \
  case KTV:                                                                                  \
    hipLaunchKernelGGL((kadj<GM, D, KTV>), grid, dim3(256), 0, st, a.xp, steps16, a.S, a.uhi, \
                       a.ulo, a.whi, a.wlo, a.partial);                                      \
    break;
  switch (a.KT) {
    GPK_ADJ_CASE(1)
    GPK_ADJ_CASE(2)
    GPK_ADJ_CASE(3)
    GPK_ADJ_CASE(4)
    GPK_ADJ_CASE(8)
    default: return hipErrorInvalidValue;
  }
#undef GPK_ADJ_CASE
  return hipGetLastError();
}

}  // namespace

#ifndef GPK_D
#error "compile with -DGPK_D=<dimension>"
#endif
#define GPK_CAT2(a, b) a##b
#define GPK_CAT(a, b) GPK_CAT2(a, b)
hipError_t GPK_CAT(adj_d, GPK_D)(const AdjArgs& a, int64_t rowblocks, hipStream_t st) {
  if (a.prec == P_BF16X3) return launch_kt<P_BF16X3, GPK_D>(a, rowblocks, st);
  return launch_kt<P_FP32, GPK_D>(a, rowblocks, st);
}

}  // namespace gpk
