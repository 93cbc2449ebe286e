// Kernels specific to alternating projections and SGD (App. B, Algorithms 2-3).
//
// AP: the regularised diagonal blocks H[I, I] (contiguous row blocks of size b)
// are assembled in FP64, factorised once per solve by a tiled right-looking
// Cholesky (one workgroup per block, 32x32 tiles staged in LDS), and each
// iteration solves H[I, I] delta = r[I] for all c columns with a left-looking
// forward and a right-looking backward substitution (both read rows of L, so
// every access to the factor is contiguous).  Block scores
// ||sum_c r[I, c]|| are one workgroup per block.
// SGD: the gradient rows H[I, :] u - b~[I] reuse the forward product kernel on
// the gathered rows; the fix-up of the noise term and the targets is here.
#include <algorithm>

#include "gpk.h"

namespace gpk {

namespace {

constexpr int kT = 32;  // Cholesky tile

// H[I, I] for every block, lower triangle, padded to P x P with the identity.
__global__ __launch_bounds__(256) void kbuild_blocks(const float* __restrict__ xp, int DP, int d,
                                                     int64_t n, int b, int P, double a2,
                                                     double s2, double* __restrict__ M) {
  const int k = blockIdx.y;
  const int64_t base = (int64_t)k * b;
  const int bk = (int)(n - base < b ? n - base : b);
  double* Mk = M + (int64_t)k * P * P;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < (int64_t)P * P;
       t += (int64_t)gridDim.x * 256) {
    const int i = (int)(t / P), j = (int)(t % P);
    if (j > i) continue;
    double v;
    if (i < bk && j < bk) {
      double r2 = 0.0;
      for (int q = 0; q < d; ++q) {
        const double df = (double)xp[(base + i) * DP + q] - (double)xp[(base + j) * DP + q];
        r2 += df * df;
      }
      const double rho = sqrt(r2);
      v = a2 * (1.0 + 0.69314718055994530942 * rho) * exp2(-rho);
      if (i == j) v += s2;
    } else {
      v = (i == j) ? 1.0 : 0.0;
    }
    Mk[(int64_t)i * P + j] = v;
  }
}

// In-place lower Cholesky of each P x P block (P multiple of 32).  status bit 2
// is set if a pivot is not positive.
__global__ __launch_bounds__(256) void kchol(double* __restrict__ M, int P, int* status) {
  double* A = M + (int64_t)blockIdx.x * P * P;
  __shared__ double Dt[kT][kT + 1];
  __shared__ double Li[kT][kT + 1];
  __shared__ double Lj[kT][kT + 1];
  __shared__ int bad;
  const int tid = threadIdx.x;
  const int T = P / kT;
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int kt = 0; kt < T; ++kt) {
    const int k0 = kt * kT;
    // (a) diagonal tile
    for (int e = tid; e < kT * kT; e += 256) Dt[e / kT][e % kT] = A[(int64_t)(k0 + e / kT) * P + k0 + e % kT];
    __syncthreads();
    for (int k = 0; k < kT; ++k) {
      if (tid == 0) {
        const double p = Dt[k][k];
        if (!(p > 0.0)) bad = 1;
        Dt[k][k] = p > 0.0 ? sqrt(p) : 1.0;
      }
      __syncthreads();
      if (tid > k && tid < kT) Dt[tid][k] /= Dt[k][k];
      __syncthreads();
      for (int e = tid; e < kT * kT; e += 256) {
        const int i = e / kT, j = e % kT;
        if (j > k && i >= j) Dt[i][j] -= Dt[i][k] * Dt[j][k];
      }
      __syncthreads();
    }
    for (int e = tid; e < kT * kT; e += 256) {
      const int i = e / kT, j = e % kT;
      if (j <= i) A[(int64_t)(k0 + i) * P + k0 + j] = Dt[i][j];
    }
    // (b) panel: rows below the diagonal tile, X L_kk^T = A  (one row per thread)
    for (int r = k0 + kT + tid; r < P; r += 256) {
      double x[kT];
#pragma unroll
      for (int c = 0; c < kT; ++c) x[c] = A[(int64_t)r * P + k0 + c];
#pragma unroll
      for (int c = 0; c < kT; ++c) {
        double v = x[c];
#pragma unroll
        for (int q = 0; q < c; ++q) v -= x[q] * Dt[c][q];
        x[c] = v / Dt[c][c];
      }
#pragma unroll
      for (int c = 0; c < kT; ++c) A[(int64_t)r * P + k0 + c] = x[c];
    }
    __syncthreads();
    // (c) trailing update of tiles (it, jt), kt < jt <= it
    for (int it = kt + 1; it < T; ++it) {
      for (int e = tid; e < kT * kT; e += 256)
        Li[e / kT][e % kT] = A[(int64_t)(it * kT + e / kT) * P + k0 + e % kT];
      for (int jt = kt + 1; jt <= it; ++jt) {
        __syncthreads();
        for (int e = tid; e < kT * kT; e += 256)
          Lj[e / kT][e % kT] = A[(int64_t)(jt * kT + e / kT) * P + k0 + e % kT];
        __syncthreads();
        for (int e = tid; e < kT * kT; e += 256) {
          const int i = e / kT, j = e % kT;
          if (it == jt && j > i) continue;
          double s = 0.0;
#pragma unroll 8
          for (int q = 0; q < kT; ++q) s += Li[i][q] * Lj[j][q];
          A[(int64_t)(it * kT + i) * P + jt * kT + j] -= s;
        }
      }
      __syncthreads();
    }
    __syncthreads();
  }
  if (tid == 0 && bad) atomicOr(status, 2);
}

// Blocked right-looking Cholesky of one large P x P matrix (P multiple of 32)
// spread over many workgroups, one 32-column panel at a time: the diagonal tile
// (one workgroup), the panel below it (one row per thread) and the trailing
// lower tiles A[it][jt] -= L[it][kt] L[jt][kt]^T (one workgroup per tile).
__global__ __launch_bounds__(256) void kchol_diag(double* __restrict__ A, int P, int kt,
                                                  int* status) {
  __shared__ double Dt[kT][kT + 1];
  __shared__ int bad;
  const int tid = threadIdx.x;
  const int k0 = kt * kT;
  if (tid == 0) bad = 0;
  for (int e = tid; e < kT * kT; e += 256) Dt[e / kT][e % kT] = A[(int64_t)(k0 + e / kT) * P + k0 + e % kT];
  __syncthreads();
  for (int k = 0; k < kT; ++k) {
    if (tid == 0) {
      const double p = Dt[k][k];
      if (!(p > 0.0)) bad = 1;
      Dt[k][k] = p > 0.0 ? sqrt(p) : 1.0;
    }
    __syncthreads();
    if (tid > k && tid < kT) Dt[tid][k] /= Dt[k][k];
    __syncthreads();
    for (int e = tid; e < kT * kT; e += 256) {
      const int i = e / kT, j = e % kT;
      if (j > k && i >= j) Dt[i][j] -= Dt[i][k] * Dt[j][k];
    }
    __syncthreads();
  }
  for (int e = tid; e < kT * kT; e += 256) {
    const int i = e / kT, j = e % kT;
    if (j <= i) A[(int64_t)(k0 + i) * P + k0 + j] = Dt[i][j];
  }
  if (tid == 0 && bad) atomicOr(status, 2);
}

__global__ __launch_bounds__(256) void kchol_panel(double* __restrict__ A, int P, int kt) {
  __shared__ double Dt[kT][kT + 1];
  const int tid = threadIdx.x;
  const int k0 = kt * kT;
  for (int e = tid; e < kT * kT; e += 256) Dt[e / kT][e % kT] = A[(int64_t)(k0 + e / kT) * P + k0 + e % kT];
  __syncthreads();
  const int r = k0 + kT + blockIdx.x * 256 + tid;
  if (r >= P) return;
  double x[kT];
#pragma unroll
  for (int c = 0; c < kT; ++c) x[c] = A[(int64_t)r * P + k0 + c];
#pragma unroll
  for (int c = 0; c < kT; ++c) {
    double v = x[c];
#pragma unroll
    for (int q = 0; q < c; ++q) v -= x[q] * Dt[c][q];
    x[c] = v / Dt[c][c];
  }
#pragma unroll
  for (int c = 0; c < kT; ++c) A[(int64_t)r * P + k0 + c] = x[c];
}

// Workgroup b updates the b-th lower tile (it, jt), kt < jt <= it, in row order.
__global__ __launch_bounds__(256) void kchol_update(double* __restrict__ A, int P, int kt) {
  __shared__ double Li[kT][kT + 1];
  __shared__ double Lj[kT][kT + 1];
  const int tid = threadIdx.x;
  const int k0 = kt * kT;
  // tile index b -> (it, jt) with m = it - kt - 1 >= 0 and jt - kt - 1 in [0, m]
  const int64_t b = blockIdx.x;
  int m = (int)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
  while ((int64_t)(m + 1) * (m + 2) / 2 <= b) ++m;
  while ((int64_t)m * (m + 1) / 2 > b) --m;
  const int it = kt + 1 + m;
  const int jt = kt + 1 + (int)(b - (int64_t)m * (m + 1) / 2);
  for (int e = tid; e < kT * kT; e += 256) {
    Li[e / kT][e % kT] = A[(int64_t)(it * kT + e / kT) * P + k0 + e % kT];
    Lj[e / kT][e % kT] = A[(int64_t)(jt * kT + e / kT) * P + k0 + e % kT];
  }
  __syncthreads();
  for (int e = tid; e < kT * kT; e += 256) {
    const int i = e / kT, j = e % kT;
    if (it == jt && j > i) continue;
    double sacc = 0.0;
#pragma unroll 8
    for (int q = 0; q < kT; ++q) sacc += Li[i][q] * Lj[j][q];
    A[(int64_t)(it * kT + i) * P + jt * kT + j] -= sacc;
  }
}

// Solve L L^T delta = r for block `blk` (bk rows) and 4 columns per workgroup.
// r is read from R[base + i, c] (ld ldr), delta written to out[i, c] (ld ldo).
__global__ __launch_bounds__(256) void ktrisolve(const double* __restrict__ M, int P, int blk,
                                                 int b, int64_t n, const float* __restrict__ R,
                                                 int64_t ldr, int c, float* __restrict__ out,
                                                 int64_t ldo) {
  constexpr int CW = 4;                // columns per workgroup
  __shared__ double y[kMaxAPBlock][CW];  // 63 KiB: fits the 64 KiB workgroup LDS limit
  __shared__ double red[256 / 64][CW];
  const double* L = M + (int64_t)blk * P * P;
  const int64_t base = (int64_t)blk * b;
  const int bk = (int)(n - base < b ? n - base : b);
  const int c0 = blockIdx.x * CW;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int e = tid; e < bk * CW; e += 256) {
    const int i = e / CW, q = e % CW;
    y[i][q] = (c0 + q < c) ? (double)R[(base + i) * ldr + c0 + q] : 0.0;
  }
  __syncthreads();
  // forward: y_k = (r_k - sum_{j<k} L_kj y_j) / L_kk   (row k of L, dot products)
  for (int k = 0; k < bk; ++k) {
    double acc[CW];
#pragma unroll
    for (int q = 0; q < CW; ++q) acc[q] = 0.0;
    for (int j = tid; j < k; j += 256) {
      const double l = L[(int64_t)k * P + j];
#pragma unroll
      for (int q = 0; q < CW; ++q) acc[q] += l * y[j][q];
    }
#pragma unroll
    for (int q = 0; q < CW; ++q) {
      double v = acc[q];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      if (lane == 0) red[wave][q] = v;
    }
    __syncthreads();
    if (tid < CW) {
      const double s = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
      y[k][tid] = (y[k][tid] - s) / L[(int64_t)k * P + k];
    }
    __syncthreads();
  }
  // backward: delta_k = y_k / L_kk; y_j -= L_kj delta_k for j < k  (row k of L, axpy)
  for (int k = bk - 1; k >= 0; --k) {
    if (tid < CW) y[k][tid] /= L[(int64_t)k * P + k];
    __syncthreads();
    for (int j = tid; j < k; j += 256) {
      const double l = L[(int64_t)k * P + j];
#pragma unroll
      for (int q = 0; q < CW; ++q) y[j][q] -= l * y[k][q];
    }
    __syncthreads();
  }
  for (int e = tid; e < bk * CW; e += 256) {
    const int i = e / CW, q = e % CW;
    if (c0 + q < c) out[(int64_t)i * ldo + c0 + q] = (float)y[i][q];
  }
}

// score_k = || sum_c R[I_k, c] ||^2 (block of b contiguous rows).
__global__ __launch_bounds__(256) void kap_scores(const float* __restrict__ R, int64_t ld,
                                                  int64_t n, int b, int c,
                                                  double* __restrict__ scores) {
  const int64_t base = (int64_t)blockIdx.x * b;
  const int64_t end = base + b < n ? base + b : n;
  double acc = 0.0;
  for (int64_t i = base + threadIdx.x; i < end; i += 256) {
    double s = 0.0;
    for (int q = 0; q < c; ++q) s += (double)R[i * ld + q];
    acc += s * s;
  }
  __shared__ double sh[256];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) scores[blockIdx.x] = sh[0];
}

// G[i, :] += s2 * Ut[idx[i], :] - Bt[idx[i], :]
__global__ void ksgd_fix(float* __restrict__ G, int64_t ldg, const float* __restrict__ Ut,
                         const float* __restrict__ Bt, int64_t ld, const int32_t* __restrict__ idx,
                         int64_t b, int c, float s2) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= b * c) return;
  const int64_t i = t / c;
  const int q = (int)(t % c);
  const int64_t src = (int64_t)idx[i] * ld + q;
  G[i * ldg + q] += s2 * Ut[src] - Bt[src];
}

// rows [base, base + bk): Y[base + i, :] += alpha * X[i, :]
__global__ void kadd_block(float* __restrict__ Y, int64_t ldy, int64_t base, int bk,
                           const float* __restrict__ X, int64_t ldx, int c, float alpha) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)bk * c) return;
  const int64_t i = t / c;
  const int q = (int)(t % c);
  Y[(base + i) * ldy + q] = __builtin_fmaf(alpha, X[i * ldx + q], Y[(base + i) * ldy + q]);
}

}  // namespace

hipError_t ap_build_blocks(const float* xp, int DP, int d, int64_t n, int b, int P, double a2,
                           double s2, double* M, hipStream_t st) {
  const int nblk = (int)((n + b - 1) / b);
  const int64_t per = (int64_t)P * P;
  const unsigned gx = (unsigned)std::min<int64_t>((per + 255) / 256, 1024);
  hipLaunchKernelGGL(kbuild_blocks, dim3(gx, nblk), dim3(256), 0, st, xp, DP, d, n, b, P, a2, s2,
                     M);
  return hipGetLastError();
}

hipError_t chol_blocked(double* A, int P, int* status, hipStream_t st) {
  if (P % kT) return hipErrorInvalidValue;
  const int T = P / kT;
  for (int kt = 0; kt < T; ++kt) {
    hipLaunchKernelGGL(kchol_diag, dim3(1), dim3(256), 0, st, A, P, kt, status);
    const int rows = P - (kt + 1) * kT;
    if (rows <= 0) break;
    hipLaunchKernelGGL(kchol_panel, dim3((rows + 255) / 256), dim3(256), 0, st, A, P, kt);
    const int64_t m = T - kt - 1;
    hipLaunchKernelGGL(kchol_update, dim3((unsigned)(m * (m + 1) / 2)), dim3(256), 0, st, A, P,
                       kt);
  }
  return hipGetLastError();
}

hipError_t ap_cholesky(double* M, int nblk, int P, int* status, hipStream_t st) {
  hipLaunchKernelGGL(kchol, dim3(nblk), dim3(256), 0, st, M, P, status);
  return hipGetLastError();
}

hipError_t ap_solve_block(const double* M, int P, int blk, int b, int64_t n, const float* R,
                          int64_t ldr, int c, float* out, int64_t ldo, hipStream_t st) {
  if (P > kMaxAPBlock) return hipErrorInvalidValue;
  hipLaunchKernelGGL(ktrisolve, dim3((c + 3) / 4), dim3(256), 0, st, M, P, blk, b, n, R, ldr, c,
                     out, ldo);
  return hipGetLastError();
}

hipError_t ap_scores(const float* R, int64_t ld, int64_t n, int b, int c, double* scores,
                     hipStream_t st) {
  const int nblk = (int)((n + b - 1) / b);
  hipLaunchKernelGGL(kap_scores, dim3(nblk), dim3(256), 0, st, R, ld, n, b, c, scores);
  return hipGetLastError();
}

hipError_t add_block(float* Y, int64_t ldy, int64_t base, int bk, const float* X, int64_t ldx,
                     int c, float alpha, hipStream_t st) {
  const int64_t tot = (int64_t)bk * c;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(kadd_block, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, Y, ldy,
                     base, bk, X, ldx, c, alpha);
  return hipGetLastError();
}

hipError_t sgd_fix(float* G, int64_t ldg, const float* Ut, const float* Bt, int64_t ld,
                   const int32_t* idx, int64_t b, int c, float s2, hipStream_t st) {
  const int64_t tot = b * c;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(ksgd_fix, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, G, ldg, Ut,
                     Bt, ld, idx, b, c, s2);
  return hipGetLastError();
}

}  // namespace gpk
