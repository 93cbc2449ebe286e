// Random-Fourier-feature prior samples (App. B, "Kernel Function and Random
// Features"): with omega_m = t_m / ell and M sin/cos pairs,
//   F[i, j] = (a / sqrt(M)) sum_m cos(x_i . omega_m) W[m, j] + sin(x_i . omega_m) W[M + m, j]
// optionally plus sigma * w_eps[i, j] (the pathwise right-hand side
// xi_j = f_j(x) + eps_j of Sec. 3 with eps = sigma w_eps under warm start).
//
// One thread per row and 64 output columns per workgroup column slice; the
// frequencies (FP64) and weights of 32 features at a time are staged in LDS
// and read as broadcasts.  The phase is accumulated and reduced modulo 2 pi in
// FP64 (so that large phases keep their accuracy), then sine and cosine are
// taken in FP32.
#include "gpk.h"

namespace gpk {

namespace {

constexpr int kFeatChunk = 32;
constexpr int kColChunk = 64;

template <int D>
__global__ __launch_bounds__(256) void krff(const float* __restrict__ x, int d, int64_t m,
                                            const double* __restrict__ omega, int M,
                                            const float* __restrict__ W, int64_t ldw, int s,
                                            float amp, float* __restrict__ F, int64_t ldf,
                                            int f_col0, const float* __restrict__ weps,
                                            int64_t ldeps, float sigma) {
  __shared__ double om[kFeatChunk][D];
  __shared__ float wc[kFeatChunk][kColChunk];
  __shared__ float ws[kFeatChunk][kColChunk];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int col0 = blockIdx.y * kColChunk;
  const int ncols = min(kColChunk, s - col0);
  const bool valid = i < m;
  double xi[D];
#pragma unroll
  for (int k = 0; k < D; ++k) xi[k] = (valid && k < d) ? (double)x[i * d + k] : 0.0;
  float acc[kColChunk];
#pragma unroll
  for (int cc = 0; cc < kColChunk; ++cc) acc[cc] = 0.f;
  constexpr double kTwoPi = 6.283185307179586477;
  constexpr double kInvTwoPi = 0.15915494309189533577;

  for (int m0 = 0; m0 < M; m0 += kFeatChunk) {
    const int cnt = min(kFeatChunk, M - m0);
    for (int t = threadIdx.x; t < kFeatChunk * D; t += 256) {
      const int mm = t / D, k = t % D;
      om[mm][k] = (mm < cnt && k < d) ? omega[(int64_t)(m0 + mm) * d + k] : 0.0;
    }
    for (int t = threadIdx.x; t < kFeatChunk * kColChunk; t += 256) {
      const int mm = t / kColChunk, cc = t % kColChunk;
      const bool ok = mm < cnt && cc < ncols;
      wc[mm][cc] = ok ? W[(int64_t)(m0 + mm) * ldw + col0 + cc] : 0.f;
      ws[mm][cc] = ok ? W[(int64_t)(M + m0 + mm) * ldw + col0 + cc] : 0.f;
    }
    __syncthreads();
    for (int mm = 0; mm < cnt; ++mm) {
      double ph = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) ph = __builtin_fma(xi[k], om[mm][k], ph);
      ph -= kTwoPi * __builtin_rint(ph * kInvTwoPi);
      float sn, cs;
      sincosf((float)ph, &sn, &cs);
#pragma unroll
      for (int cc = 0; cc < kColChunk; ++cc)
        acc[cc] = __builtin_fmaf(cs, wc[mm][cc], __builtin_fmaf(sn, ws[mm][cc], acc[cc]));
    }
    __syncthreads();
  }
  if (!valid) return;
  for (int cc = 0; cc < ncols; ++cc) {
    float v = amp * acc[cc];
    if (weps) v = __builtin_fmaf(sigma, weps[i * ldeps + col0 + cc], v);
    F[i * ldf + f_col0 + col0 + cc] = v;
  }
}

}  // namespace

#ifndef GPK_D
#error "compile with -DGPK_D=<dimension>"
#endif
#define GPK_CAT2(a, b) a##b
#define GPK_CAT(a, b) GPK_CAT2(a, b)
hipError_t GPK_CAT(rff_d, GPK_D)(const RffArgs& a, hipStream_t st) {
  if (a.m == 0 || a.s == 0) return hipSuccess;
  const dim3 grid((unsigned)((a.m + 255) / 256), (unsigned)((a.s + kColChunk - 1) / kColChunk));
  hipLaunchKernelGGL((krff<GPK_D>), grid, dim3(256), 0, st, a.x, a.d, a.m, a.omega, a.M, a.W,
                     a.ldw, a.s, a.amp, a.F, a.ldf, a.f_col0, a.weps, a.ldeps, a.sigma);
  return hipGetLastError();
}

}  // namespace gpk
