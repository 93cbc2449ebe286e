// Kernels specific to alternating projections and SGD (App. B, Algorithms 2-3).
//
// AP: the regularised diagonal blocks H[I, I] (contiguous row blocks of size b)
// are assembled in FP64, factorised once per solve by a tiled right-looking
// Cholesky (one workgroup per block, 32x32 tiles staged in LDS), and the factors
// are inverted in place (X = L^-1), so that each iteration's solve
// H[I, I] delta = r[I] is the two triangular products X^T (X r[I]), parallel
// over rows and columns instead of two sequential substitutions.  The residual
// update after the column-block product is one pass over R per block that also
// yields the block scores ||sum_c r[I, c]||^2 and the column norms.
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

// In place, for every block: the lower Cholesky factor L becomes X = L^-1 (one
// workgroup per block).  First every 32x32 diagonal tile is inverted (one column
// of the tile per thread, forward substitution in LDS); then, from X L = I,
// X_ij = -(sum_{k=j+1..i} X_ik L_kj) X_jj for the tile columns j from right to
// left and, within a column, the tile rows i from bottom to top, so each X_ij
// replaces L_ij once nothing later reads it.  The upper triangle is never read.
__global__ __launch_bounds__(256) void kchol_inv(double* __restrict__ M, int P) {
  double* A = M + (int64_t)blockIdx.x * P * P;
  __shared__ double Ta[kT][kT + 1];
  __shared__ double Tb[kT][kT + 1];
  __shared__ double Tx[kT][kT + 1];
  const int tid = threadIdx.x;
  const int T = P / kT;
  // (a) diagonal tiles
  for (int dt = 0; dt < T; ++dt) {
    const int64_t o = (int64_t)dt * kT * P + dt * kT;
    for (int e = tid; e < kT * kT; e += 256) {
      const int i = e / kT, j = e % kT;
      Ta[i][j] = j <= i ? A[o + (int64_t)i * P + j] : 0.0;
    }
    __syncthreads();
    if (tid < kT) {
      const int c0 = tid;  // column c0 of the tile's inverse
      for (int r = 0; r < kT; ++r) {
        double v;
        if (r < c0) {
          v = 0.0;
        } else if (r == c0) {
          v = 1.0 / Ta[r][r];
        } else {
          double acc = 0.0;
          for (int k = c0; k < r; ++k) acc += Ta[r][k] * Tx[k][c0];
          v = -acc / Ta[r][r];
        }
        Tx[r][c0] = v;
      }
    }
    __syncthreads();
    for (int e = tid; e < kT * kT; e += 256) {
      const int i = e / kT, j = e % kT;
      if (j <= i) A[o + (int64_t)i * P + j] = Tx[i][j];
    }
    __syncthreads();
  }
  // (b) off-diagonal tiles; thread -> rows r, columns 4 q .. 4 q + 3 of a tile
  const int r = tid / 8, q4 = 4 * (tid % 8);
  for (int jt = T - 2; jt >= 0; --jt) {
    for (int it = T - 1; it > jt; --it) {
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      for (int kt = jt + 1; kt <= it; ++kt) {
        const int64_t oa = (int64_t)it * kT * P + kt * kT;  // X_ik
        const int64_t ob = (int64_t)kt * kT * P + jt * kT;  // L_kj
        for (int e = tid; e < kT * kT; e += 256) {
          const int i = e / kT, j = e % kT;
          Ta[i][j] = (kt < it || j <= i) ? A[oa + (int64_t)i * P + j] : 0.0;
          Tb[i][j] = A[ob + (int64_t)i * P + j];
        }
        __syncthreads();
#pragma unroll 8
        for (int k = 0; k < kT; ++k) {
          const double a = Ta[r][k];
#pragma unroll
          for (int u = 0; u < 4; ++u) acc[u] += a * Tb[k][q4 + u];
        }
        __syncthreads();
      }
      // X_ij = -S X_jj (X_jj lower triangular)
      const int64_t od = (int64_t)jt * kT * P + jt * kT;
      for (int e = tid; e < kT * kT; e += 256) {
        const int i = e / kT, j = e % kT;
        Tb[i][j] = j <= i ? A[od + (int64_t)i * P + j] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) Ta[r][q4 + u] = acc[u];
      __syncthreads();
      double x[4] = {0.0, 0.0, 0.0, 0.0};
      for (int k = 0; k < kT; ++k) {
        const double sv = Ta[r][k];
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u] += sv * Tb[k][q4 + u];
      }
      const int64_t ox = (int64_t)it * kT * P + jt * kT;
#pragma unroll
      for (int u = 0; u < 4; ++u) A[ox + (int64_t)r * P + q4 + u] = -x[u];
      __syncthreads();
    }
  }
}

// y = X r for one block (X = L^-1 lower triangular, r = R[base .. base + bk) in
// FP64, zero beyond bk): workgroup (row group of 16, column group of 64), each
// thread 4 outputs, X and r staged in LDS 64 indices at a time.
constexpr int kTvRows = 16, kTvCols = 64, kTvK = 64;

__global__ __launch_bounds__(256) void ktrmv_lower(const double* __restrict__ M, int P, int blk,
                                                   int b, int64_t n, const float* __restrict__ R,
                                                   int64_t ldr, int c, double* __restrict__ y) {
  __shared__ double Xs[kTvRows][kTvK + 1];
  __shared__ double Rs[kTvK][kTvCols + 1];
  const double* X = M + (int64_t)blk * P * P;
  const int64_t base = (int64_t)blk * b;
  const int bk = (int)(n - base < b ? n - base : b);
  const int i0 = blockIdx.x * kTvRows, c0 = blockIdx.y * kTvCols;
  const int tid = threadIdx.x, r = tid / 16, cq = tid % 16;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < i0 + kTvRows; k0 += kTvK) {
    for (int e = tid; e < kTvRows * kTvK; e += 256) {
      const int i = e / kTvK, k = e % kTvK;
      Xs[i][k] = (k0 + k <= i0 + i) ? X[(int64_t)(i0 + i) * P + k0 + k] : 0.0;
    }
    for (int e = tid; e < kTvK * kTvCols; e += 256) {
      const int k = e / kTvCols, cc = e % kTvCols;
      Rs[k][cc] = (k0 + k < bk && c0 + cc < c) ? (double)R[(base + k0 + k) * ldr + c0 + cc] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int k = 0; k < kTvK; ++k) {
      const double xv = Xs[r][k];
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] += xv * Rs[k][cq + 16 * u];
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int col = c0 + cq + 16 * u;
    if (col < c) y[(int64_t)(i0 + r) * c + col] = acc[u];
  }
}

// out[k, :] = (X^T y)[k, :] for k < bk (FP32 output): workgroup (row group of 16,
// column group of 64), X columns and y rows staged 64 rows at a time.
__global__ __launch_bounds__(256) void ktrmv_upper_t(const double* __restrict__ M, int P, int blk,
                                                     int b, int64_t n, const double* __restrict__ y,
                                                     int c, float* __restrict__ out,
                                                     int64_t ldo) {
  __shared__ double Xs[kTvK][kTvRows + 1];
  __shared__ double Ys[kTvK][kTvCols + 1];
  const double* X = M + (int64_t)blk * P * P;
  const int64_t base = (int64_t)blk * b;
  const int bk = (int)(n - base < b ? n - base : b);
  const int k0 = blockIdx.x * kTvRows, c0 = blockIdx.y * kTvCols;
  const int tid = threadIdx.x, r = tid / 16, cq = tid % 16;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i0 = (k0 / kTvK) * kTvK; i0 < P; i0 += kTvK) {
    for (int e = tid; e < kTvK * kTvRows; e += 256) {
      const int i = e / kTvRows, k = e % kTvRows;
      Xs[i][k] = (i0 + i >= k0 + k) ? X[(int64_t)(i0 + i) * P + k0 + k] : 0.0;
    }
    for (int e = tid; e < kTvK * kTvCols; e += 256) {
      const int i = e / kTvCols, cc = e % kTvCols;
      Ys[i][cc] = c0 + cc < c ? y[(int64_t)(i0 + i) * c + c0 + cc] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int i = 0; i < kTvK; ++i) {
      const double xv = Xs[i][r];
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] += xv * Ys[i][cq + 16 * u];
    }
    __syncthreads();
  }
  if (k0 + r < bk) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int col = c0 + cq + 16 * u;
      if (col < c) out[(int64_t)(k0 + r) * ldo + col] = (float)acc[u];
    }
  }
  (void)base;
}

// One workgroup per sub-block w (ap_subblocks(b) equal parts of AP block
// k = w / nsub): R -= G (if G is given) and, on the selected block's rows,
// R -= s2 delta; then the sub-block's share of its block's score
// ||sum_c R[I_k, c]||^2 into scores[w] and its column sums of squares into
// part[w * c ..] (rows staged 32 at a time in LDS; fixed summation order).
__global__ __launch_bounds__(256) void kap_update(float* __restrict__ R, int64_t ld,
                                                  const float* __restrict__ G, int64_t ldg,
                                                  int64_t n, int b, int nsub, int c,
                                                  int64_t sel_base, int sel_bk,
                                                  const float* __restrict__ delta, int64_t ldd,
                                                  float s2, double* __restrict__ scores,
                                                  double* __restrict__ part) {
  __shared__ float ch[32][kMaxSolveCP + 1];
  __shared__ double sc[32];
  const int tid = threadIdx.x;
  const int k = blockIdx.x / nsub, sub = blockIdx.x % nsub;
  const int64_t k0 = (int64_t)k * b;
  const int blk = (int)(n - k0 < b ? n - k0 : b);
  const int64_t kb = k0 + (int64_t)blk * sub / nsub;
  const int bk = (int)(k0 + (int64_t)blk * (sub + 1) / nsub - kb);
  double colsq = 0.0, rowsq = 0.0;
  for (int r0 = 0; r0 < bk; r0 += 32) {
    const int rows = bk - r0 < 32 ? bk - r0 : 32;
    for (int e = tid; e < rows * c; e += 256) {
      const int rr = e / c, col = e % c;
      const int64_t i = kb + r0 + rr;
      float v = R[i * ld + col];
      if (G) {
        v = v - G[i * ldg + col];
        const int64_t si = i - sel_base;
        if (si >= 0 && si < sel_bk) v = __builtin_fmaf(-s2, delta[si * ldd + col], v);
        R[i * ld + col] = v;
      }
      ch[rr][col] = v;
    }
    __syncthreads();
    // thread t sums column t (t < c) and row t of the chunk (t < rows)
    if (tid < c)
      for (int rr = 0; rr < rows; ++rr) {
        const double v = ch[rr][tid];
        colsq += v * v;
      }
    if (tid < rows) {
      double s = 0.0;
      for (int col = 0; col < c; ++col) s += (double)ch[tid][col];
      rowsq += s * s;
    }
    __syncthreads();
  }
  if (tid < c) part[(int64_t)blockIdx.x * c + tid] = colsq;
  if (tid < 32) sc[tid] = rowsq;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int q = 0; q < 32; ++q) s += sc[q];
    scores[blockIdx.x] = s;
  }
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

hipError_t ap_cholesky(double* M, int nblk, int P, int* status, hipStream_t st) {
  hipLaunchKernelGGL(kchol, dim3(nblk), dim3(256), 0, st, M, P, status);
  return hipGetLastError();
}

hipError_t ap_invert_factors(double* M, int nblk, int P, hipStream_t st) {
  if (P % kT) return hipErrorInvalidValue;
  if (nblk <= 0) return hipSuccess;
  hipLaunchKernelGGL(kchol_inv, dim3(nblk), dim3(256), 0, st, M, P);
  return hipGetLastError();
}

hipError_t ap_solve_block(const double* M, int P, int blk, int b, int64_t n, const float* R,
                          int64_t ldr, int c, double* y, float* out, int64_t ldo, hipStream_t st) {
  if (P % kTvK || c < 1) return hipErrorInvalidValue;
  const dim3 grid((unsigned)(P / kTvRows), (unsigned)((c + kTvCols - 1) / kTvCols));
  hipLaunchKernelGGL(ktrmv_lower, grid, dim3(256), 0, st, M, P, blk, b, n, R, ldr, c, y);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(ktrmv_upper_t, grid, dim3(256), 0, st, M, P, blk, b, n, y, c, out, ldo);
  return hipGetLastError();
}

hipError_t ap_update(float* R, int64_t ld, const float* G, int64_t ldg, int64_t n, int b, int c,
                     int64_t sel_base, int sel_bk, const float* delta, int64_t ldd, float s2,
                     double* scores, double* part, hipStream_t st) {
  if (c < 1 || c > kMaxSolveCP || b < 1) return hipErrorInvalidValue;
  const int64_t nblk = (n + b - 1) / b;
  if (nblk <= 0) return hipSuccess;
  const int nsub = ap_subblocks(b);
  hipLaunchKernelGGL(kap_update, dim3((unsigned)(nblk * nsub)), dim3(256), 0, st, R, ld, G, ldg,
                     n, b, nsub, c, sel_base, sel_bk, delta, ldd, s2, scores, part);
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
