// Exact log marginal likelihood and its gradient on a dense FP64 kernel matrix
// (Sec. 2, eqs. mll and mll_grad), the inner objective of the initial-
// hyperparameter heuristic of App. B ("Iterative Optimiser"), which maximises
// it on subsets of up to 10,000 points.
//
//   L    = -1/2 y^T alpha - sum_i log C_ii - m/2 log 2 pi,  H = C C^T,  alpha = H^-1 y
//   g_k  = 1/2 sum_ij (alpha_i alpha_j - (H^-1)_ij) (dH/dtheta_k)_ij
//
// The matrix work (about m^3 flops) runs on the FP64 matrix cores:
//   * H (m_p x m_p, m_p = m rounded up to 64, identity on the padding) is built
//     from the raw inputs in FP64, lower 64 x 64 tiles only;
//   * a recursive Cholesky that also returns the inverse factor W = C^-1: for a
//     split [A11 .; A21 A22] it factors A11 (-> W11), forms C21 = A21 W11^T,
//     updates A22 -= C21 C21^T, factors A22 (-> W22) and sets
//     W21 = -W22 (C21 W11).  Leaves are 64 x 64 blocks factored and inverted by
//     one workgroup in LDS; every other step is a GEMM whose K range is cut to
//     the non-zero part of its triangular operands;
//   * H^-1 = W^T W (lower tiles), alpha = W^T (W y);
//   * the gradient contraction recomputes distances per entry of the lower
//     triangle, with FP64 partial sums per tile and a fixed-order final sum.
// Only the diagonal of C is kept (for log det H): C21 lives in the W21 slot until
// W21 replaces it, and C21 W11 in the A21 slot, so two m_p x m_p buffers suffice.
#include "gpk.h"

namespace gpk {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr double kSqrt3 = 1.7320508075688772935;
constexpr int kET = kExactTile;  // 64

__device__ __forceinline__ double wsum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// xs[t, :] = X[r, :], ys[t] = y[r] with r = idx[t] (or t); rows t in [m, m_p) are
// zero.  An index outside [0, n) sets status bit 1 and reads nothing.
__global__ void kex_gather(const float* __restrict__ X, int64_t n, int d,
                           const int64_t* __restrict__ idx, int64_t m, int64_t mp,
                           const float* __restrict__ y, double* __restrict__ xs,
                           double* __restrict__ ys, int* __restrict__ status) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= mp) return;
  int64_t r = t;
  bool ok = t < m;
  if (ok && idx) {
    r = idx[t];
    if (r < 0 || r >= n) {
      atomicOr(status, 1);
      ok = false;
    }
  }
  for (int k = 0; k < d; ++k) xs[t * d + k] = ok ? (double)X[r * d + k] : 0.0;
  ys[t] = ok ? (double)y[r] : 0.0;
}

// Lower 64 x 64 tiles of H = a^2 (1 + sqrt3 r) exp(-sqrt3 r) + s2 I (identity on
// the padding), r^2 = sum_k ((x_ik - x_jk) / ell_k)^2.
__global__ __launch_bounds__(256) void kex_build(const double* __restrict__ xs, int d, int64_t m,
                                                 int64_t mp, const double* __restrict__ inv_ell,
                                                 double a2, double s2, double* __restrict__ H) {
  const int64_t it = blockIdx.y, jt = blockIdx.x;
  if (jt > it) return;
  for (int e = threadIdx.x; e < kET * kET; e += 256) {
    const int64_t i = it * kET + (e >> 6), j = jt * kET + (e & 63);
    double v;
    if (i < m && j < m) {
      double r2 = 0.0;
      for (int k = 0; k < d; ++k) {
        const double u = (xs[i * d + k] - xs[j * d + k]) * inv_ell[k];
        r2 += u * u;
      }
      const double sr = kSqrt3 * sqrt(r2);
      v = a2 * (1.0 + sr) * exp(-sr);
      if (i == j) v += s2;
    } else {
      v = (i == j) ? 1.0 : 0.0;
    }
    H[i * mp + j] = v;
  }
}

__device__ __forceinline__ double rdlane(double v, int k) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)bits, k);
  const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), k);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// 1/sqrt(p) for p > 0: hardware estimate and two Newton steps r <- r (3 - p r^2) / 2.
__device__ __forceinline__ double rsqrt_nr(double p) {
  double r = __builtin_amdgcn_rsq(p);
  r = r * (1.5 - 0.5 * p * r * r);
  return r * (1.5 - 0.5 * p * r * r);
}

// Leaf of the recursion: the 64 x 64 diagonal block at (off, off), one wave,
// lane r holding row r in registers (every loop below is unrolled, so all
// register indices are static).  No barriers: the wave's LDS accesses complete
// in order, and each column is broadcast through LDS.
// Cholesky, step k: pivot from lane k, lanes below scale their entry of column k,
// which every lane then reads to update its entries right of k
// (C_rc -= C_rk C_ck).  A non-positive pivot sets status bit 2 and is replaced
// by 1 so the kernel completes; the pivots go to diag.
// Inverse factor: lane c forms column c of W = C^-1 by forward substitution,
// x_s = (delta_sc - acc_s) / C_ss, then acc_r += C_rs x_s for r > s, with
// column s of C broadcast the same way; columns left of c stay exactly zero.
__global__ __launch_bounds__(64) void kex_leaf(const double* __restrict__ A, double* __restrict__ W,
                                               int64_t ld, int64_t off, double* __restrict__ diag,
                                               int* __restrict__ status) {
  __shared__ double colb[kET];
  const int r = threadIdx.x;
  double dr[kET];
#pragma unroll
  for (int c = 0; c < kET; ++c) dr[c] = (c <= r) ? A[(off + r) * ld + off + c] : 0.0;
  bool bad = false;
  double mydiag = 1.0, myinv = 1.0;
#pragma unroll
  for (int k = 0; k < kET; ++k) {
    double p = rdlane(dr[k], k);
    if (!(p > 0.0)) {
      bad = true;
      p = 1.0;
    }
    const double ri = rsqrt_nr(p);
    const double sk = p * ri;
    if (r == k) {
      mydiag = sk;
      myinv = ri;
    }
    dr[k] = r > k ? dr[k] * ri : (r == k ? sk : dr[k]);
    colb[r] = dr[k];
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int c = k + 1; c < kET; ++c) dr[c] = __builtin_fma(-dr[k], colb[c], dr[c]);
    __builtin_amdgcn_wave_barrier();
  }
  diag[off + r] = mydiag;
  // column r of W (lane r computes column c = r)
  double x[kET];
#pragma unroll
  for (int s2 = 0; s2 < kET; ++s2) x[s2] = 0.0;
#pragma unroll
  for (int s2 = 0; s2 < kET; ++s2) {
    x[s2] = ((r == s2 ? 1.0 : 0.0) - x[s2]) * rdlane(myinv, s2);
    colb[r] = dr[s2];
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int rr = s2 + 1; rr < kET; ++rr) x[rr] = __builtin_fma(colb[rr], x[s2], x[rr]);
    __builtin_amdgcn_wave_barrier();
  }
#pragma unroll
  for (int rr = 0; rr < kET; ++rr) W[(off + rr) * ld + off + r] = x[rr];
  if (r == 0 && bad) atomicOr(status, 2);
}

// C (M x N) = alpha op(A) op(B) (+ C when accumulate).  op(A)[i][k] = A[i*lda + k]
// (TA false) or A[k*lda + i]; op(B)[k][j] = B[k*ldb + j] (TB false) or B[j*ldb + k].
// M, N, K multiples of 64.  One workgroup per 64 x 64 tile of C; K in stages of
// 32 staged through LDS as FP64 [k][row] / [k][col], the next stage prefetched
// into registers during the MFMAs.  Wave w: rows 16w..16w+15 x 64 columns, four
// v_mfma_f64_16x16x4f64 accumulators (A lane: op(A)[16w + l%16][k + l/16]; B lane:
// op(B)[k + l/16][16u + l%16]; D lane q: (16w + 4q + l/16, 16u + l%16)).
// flags: kExLowerC computes only tiles with j0 <= i0; the four triangle flags
// restrict K to where the operand can be non-zero at this tile.
template <bool TA, bool TB>
__global__ __launch_bounds__(256) void kex_gemm(int K, const double* __restrict__ A, int64_t lda,
                                                const double* __restrict__ B, int64_t ldb,
                                                double* __restrict__ C, int64_t ldc, double alpha,
                                                int accumulate, int flags) {
  constexpr int KT = 32;
  constexpr int LS = kET + 4;
  __shared__ double As[KT][LS];
  __shared__ double Bs[KT][LS];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int la = lane & 15, lk = lane >> 4;
  const int64_t i0 = (int64_t)blockIdx.y * kET, j0 = (int64_t)blockIdx.x * kET;
  if ((flags & kExLowerC) && j0 > i0) return;
  int64_t kb = 0, ke = K;
  if (flags & kExALower) ke = ke < i0 + kET ? ke : i0 + kET;
  if (flags & kExAUpper) kb = kb > i0 ? kb : i0;
  if (flags & kExBLower) kb = kb > j0 ? kb : j0;
  if (flags & kExBUpper) ke = ke < j0 + kET ? ke : j0 + kET;
  f64x4 acc[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) acc[u] = f64x4{0.0, 0.0, 0.0, 0.0};
  // loader coordinates: "row" layout = 64 rows x 32 k (4 threads x 8 per row),
  // "k" layout = 32 k-rows x 64 (8 threads x 8 per k-row)
  const int rr = tid >> 2, rc = (tid & 3) * 8;
  const int kr = tid >> 3, kc = (tid & 7) * 8;
  double ra[8], rb[8];
  auto load = [&](int64_t k) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      ra[e] = TA ? A[(k + kr) * lda + i0 + kc + e] : A[(i0 + rr) * lda + k + rc + e];
      rb[e] = TB ? B[(j0 + rr) * ldb + k + rc + e] : B[(k + kr) * ldb + j0 + kc + e];
    }
  };
  if (kb < ke) load(kb);
  for (int64_t k = kb; k < ke; k += KT) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      if (TA) As[kr][kc + e] = ra[e];
      else As[rc + e][rr] = ra[e];
      if (TB) Bs[rc + e][rr] = rb[e];
      else Bs[kr][kc + e] = rb[e];
    }
    __syncthreads();
    if (k + KT < ke) load(k + KT);
#pragma unroll
    for (int s = 0; s < KT / 4; ++s) {
      const double av = As[4 * s + lk][16 * wave + la];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Bs[4 * s + lk][16 * u + la], acc[u], 0,
                                                      0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t r = i0 + 16 * wave + 4 * q + lk;
      const int64_t c = j0 + 16 * u + la;
      const double v = alpha * acc[u][q];
      C[r * ldc + c] = accumulate ? C[r * ldc + c] + v : v;
    }
}

// v_i = sum_{j <= i} W_ij y_j (one wave per row).
__global__ __launch_bounds__(256) void kex_wy(const double* __restrict__ W, int64_t mp,
                                              const double* __restrict__ y,
                                              double* __restrict__ v) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= mp) return;
  double s = 0.0;
  for (int64_t j = lane; j <= i; j += 64) s += W[i * mp + j] * y[j];
  s = wsum(s);
  if (lane == 0) v[i] = s;
}

// part[c][j] = sum over rows i of chunk c with i >= j of W_ij v_i.
__global__ __launch_bounds__(256) void kex_wtv(const double* __restrict__ W, int64_t mp,
                                               const double* __restrict__ v, int64_t chunk,
                                               double* __restrict__ part) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= mp) return;
  const int64_t c = blockIdx.y;
  int64_t i = c * chunk;
  const int64_t i1 = i + chunk < mp ? i + chunk : mp;
  if (i < j) i = j;
  double s = 0.0;
  for (; i < i1; ++i) s += W[i * mp + j] * v[i];
  part[c * mp + j] = s;
}

__global__ __launch_bounds__(256) void kex_sum_parts(const double* __restrict__ part, int nc,
                                                     int64_t mp, double* __restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= mp) return;
  double s = 0.0;
  for (int c = 0; c < nc; ++c) s += part[c * mp + j];
  out[j] = s;
}

__device__ double block_sum(double v, double* red) {
  const int tid = threadIdx.x;
  v = wsum(v);
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

// out[0] = y^T alpha, out[1] = log det H = 2 sum_i log C_ii (rows < m; one
// workgroup, fixed order).
__global__ __launch_bounds__(256) void kex_scalars(const double* __restrict__ y,
                                                   const double* __restrict__ alpha,
                                                   const double* __restrict__ diag, int64_t m,
                                                   double* __restrict__ out) {
  __shared__ double red[4];
  double q = 0.0, l = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += 256) {
    q += y[i] * alpha[i];
    l += log(diag[i]);
  }
  q = block_sum(q, red);
  l = block_sum(l, red);
  if (threadIdx.x == 0) {
    out[0] = q;
    out[1] = 2.0 * l;
  }
}

// One lower tile of the gradient contraction, weight w = 2 off the diagonal
// (the matrices are symmetric) and 1 on it, G = alpha alpha^T - H^-1:
//   part[tile][k]   = sum w G_ij exp(-sqrt3 r) (x_ik - x_jk)^2   (k < d)
//   part[tile][d]   = sum w G_ij (1 + sqrt3 r) exp(-sqrt3 r)
//   part[tile][d+1] = sum_i G_ii
__global__ __launch_bounds__(256) void kex_grad(const double* __restrict__ xs, int d, int64_t m,
                                                int64_t mp, const double* __restrict__ inv_ell,
                                                const double* __restrict__ Hinv,
                                                const double* __restrict__ alpha,
                                                double* __restrict__ part) {
  __shared__ double red[4][kMaxD + 2];
  const int64_t it = blockIdx.y, jt = blockIdx.x;
  if (jt > it) return;
  const int64_t tile = it * (it + 1) / 2 + jt;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int EPT = kET * kET / 256;
  double E[EPT];
  double sa = 0.0, ss = 0.0;
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int e = tid + 256 * q;
    const int64_t i = it * kET + (e >> 6), j = jt * kET + (e & 63);
    E[q] = 0.0;
    if (i < m && j <= i) {
      const double g = alpha[i] * alpha[j] - Hinv[i * mp + j];
      const double w = i == j ? 1.0 : 2.0;
      double r2 = 0.0;
      for (int k = 0; k < d; ++k) {
        const double u = (xs[i * d + k] - xs[j * d + k]) * inv_ell[k];
        r2 += u * u;
      }
      const double sr = kSqrt3 * sqrt(r2);
      const double ex = exp(-sr);
      E[q] = w * g * ex;
      sa += w * g * (1.0 + sr) * ex;
      if (i == j) ss += g;
    }
  }
  for (int k = 0; k < d; ++k) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int e = tid + 256 * q;
      const int64_t i = it * kET + (e >> 6), j = jt * kET + (e & 63);
      if (i < m && j <= i) {
        const double dx = xs[i * d + k] - xs[j * d + k];
        t += E[q] * dx * dx;
      }
    }
    t = wsum(t);
    if (lane == 0) red[wave][k] = t;
  }
  sa = wsum(sa);
  ss = wsum(ss);
  if (lane == 0) {
    red[wave][d] = sa;
    red[wave][d + 1] = ss;
  }
  __syncthreads();
  if (tid < d + 2) part[tile * (d + 2) + tid] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
}

// grad[k] from the tile partials: one workgroup per component k, thread t summing
// tiles t, t + 256, ... in order, then a fixed tree (deterministic).
__global__ __launch_bounds__(256) void kex_grad_final(const double* __restrict__ part,
                                                      int64_t ntiles, int d,
                                                      const double* __restrict__ inv_ell,
                                                      double a, double sigma,
                                                      double* __restrict__ grad) {
  __shared__ double red[4];
  const int k = blockIdx.x;
  double s = 0.0;
  for (int64_t t = threadIdx.x; t < ntiles; t += 256) s += part[t * (d + 2) + k];
  s = block_sum(s, red);
  if (threadIdx.x != 0) return;
  double g;
  if (k < d) {
    const double il = inv_ell[k];
    g = 0.5 * 3.0 * a * a * s * il * il * il;  // dk/dell_k = 3 a^2 e (x_k - x'_k)^2 / ell_k^3
  } else if (k == d) {
    g = a * s;  // dk/da = 2 a (1 + sqrt3 r) e
  } else {
    g = sigma * s;  // dH/dsigma = 2 sigma I
  }
  grad[k] = g;
}

hipError_t gemm(bool ta, bool tb, int64_t M, int64_t N, int64_t K, const double* A, int64_t lda,
                const double* B, int64_t ldb, double* C, int64_t ldc, double alpha, bool acc,
                int flags, hipStream_t st) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const dim3 grid((unsigned)(N / kET), (unsigned)(M / kET));
  if (!ta && !tb)
    hipLaunchKernelGGL((kex_gemm<false, false>), grid, dim3(256), 0, st, (int)K, A, lda, B, ldb, C,
                       ldc, alpha, (int)acc, flags);
  else if (!ta && tb)
    hipLaunchKernelGGL((kex_gemm<false, true>), grid, dim3(256), 0, st, (int)K, A, lda, B, ldb, C,
                       ldc, alpha, (int)acc, flags);
  else if (ta && !tb)
    hipLaunchKernelGGL((kex_gemm<true, false>), grid, dim3(256), 0, st, (int)K, A, lda, B, ldb, C,
                       ldc, alpha, (int)acc, flags);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// Factor the diagonal block [off, off + m) of A (its trailing updates done) and
// write its inverse factor into the same block of W (see the file comment).
// With a side stream, T = C21 W11 (which needs only C21 and W11) runs there,
// concurrently with the update of A22 and its factorisation on the main stream;
// W21 = -W22 T waits for it.  Two events per split, taken from ev in order.
struct ExStreams {
  hipStream_t main, side;
  hipEvent_t* ev;
  int nev, used;
};

hipError_t chol_inv(double* A, double* W, int64_t ld, int64_t off, int64_t m, double* diag,
                    int* status, ExStreams& xs) {
  hipStream_t st = xs.main;
  if (m == kET) {
    hipLaunchKernelGGL(kex_leaf, dim3(1), dim3(64), 0, st, A, W, ld, off, diag, status);
    return hipGetLastError();
  }
  const int64_t m1 = kET * ((m / kET + 1) / 2), m2 = m - m1;
  double* A21 = A + (off + m1) * ld + off;
  double* A22 = A + (off + m1) * ld + off + m1;
  double* W11 = W + off * ld + off;
  double* W21 = W + (off + m1) * ld + off;
  double* W22 = W + (off + m1) * ld + off + m1;
  hipError_t e;
  if ((e = chol_inv(A, W, ld, off, m1, diag, status, xs)) != hipSuccess) return e;
  // C21 = A21 W11^T (op(B) = W11^T is upper triangular) -> W21 slot
  if ((e = gemm(false, true, m2, m1, m1, A21, ld, W11, ld, W21, ld, 1.0, false, kExBUpper, st)) !=
      hipSuccess)
    return e;
  const bool overlap = xs.side && xs.used + 2 <= xs.nev;
  hipEvent_t e_c21 = nullptr, e_t = nullptr;
  if (overlap) {
    e_c21 = xs.ev[xs.used++];
    e_t = xs.ev[xs.used++];
    if ((e = hipEventRecord(e_c21, st)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(xs.side, e_c21, 0)) != hipSuccess) return e;
    // T = C21 W11 (W11 lower) -> A21 slot, on the side stream
    if ((e = gemm(false, false, m2, m1, m1, W21, ld, W11, ld, A21, ld, 1.0, false, kExBLower,
                  xs.side)) != hipSuccess)
      return e;
    if ((e = hipEventRecord(e_t, xs.side)) != hipSuccess) return e;
  }
  // A22 -= C21 C21^T, lower tiles
  if ((e = gemm(false, true, m2, m2, m1, W21, ld, W21, ld, A22, ld, -1.0, true, kExLowerC, st)) !=
      hipSuccess)
    return e;
  if ((e = chol_inv(A, W, ld, off + m1, m2, diag, status, xs)) != hipSuccess) return e;
  if (overlap) {
    if ((e = hipStreamWaitEvent(st, e_t, 0)) != hipSuccess) return e;
  } else if ((e = gemm(false, false, m2, m1, m1, W21, ld, W11, ld, A21, ld, 1.0, false, kExBLower,
                       st)) != hipSuccess) {
    return e;
  }
  // W21 = -W22 T (W22 lower)
  return gemm(false, false, m2, m1, m2, W22, ld, A21, ld, W21, ld, -1.0, false, kExALower, st);
}

}  // namespace

hipError_t spd_inverse(double* A, double* W, int64_t mp, double* diag, int* status,
                       hipStream_t st) {
  if (mp <= 0 || mp % kET) return hipErrorInvalidValue;
  ExStreams xst{st, nullptr, nullptr, 0, 0};
  hipError_t e = chol_inv(A, W, mp, 0, mp, diag, status, xst);
  if (e != hipSuccess) return e;
  // A^-1 = W^T W into A (lower tiles; op(A) = W^T upper, op(B) = W lower)
  return gemm(true, false, mp, mp, mp, W, mp, W, mp, A, mp, 1.0, false,
              kExLowerC | kExAUpper | kExBLower, st);
}

hipError_t exact_gather(const float* X, int64_t n, int d, const int64_t* idx, int64_t m,
                        int64_t mp, const float* y, double* xs, double* ys, int* status,
                        hipStream_t st) {
  hipLaunchKernelGGL(kex_gather, dim3((unsigned)((mp + 255) / 256)), dim3(256), 0, st, X, n, d, idx,
                     m, mp, y, xs, ys, status);
  return hipGetLastError();
}

hipError_t exact_factor(const double* xs, int d, int64_t m, int64_t mp, const double* inv_ell,
                        double a, double sigma, double* A, double* W, double* diag, int* status,
                        hipStream_t st, hipStream_t side, hipEvent_t* ev, int nev) {
  if (mp % kET || mp < m) return hipErrorInvalidValue;
  const unsigned T = (unsigned)(mp / kET);
  hipLaunchKernelGGL(kex_build, dim3(T, T), dim3(256), 0, st, xs, d, m, mp, inv_ell, a * a,
                     sigma * sigma, A);
  ExStreams xst{st, side, ev, nev, 0};
  hipError_t e = chol_inv(A, W, mp, 0, mp, diag, status, xst);
  if (e != hipSuccess) return e;
  // H^-1 = W^T W into A (lower tiles; op(A) = W^T upper, op(B) = W lower)
  return gemm(true, false, mp, mp, mp, W, mp, W, mp, A, mp, 1.0, false,
              kExLowerC | kExAUpper | kExBLower, st);
}

hipError_t exact_finish(const double* xs, const double* ys, int d, int64_t m, int64_t mp,
                        const double* inv_ell, double a, double sigma, const double* Hinv,
                        const double* W, const double* diag, double* v, double* alpha,
                        double* part, double* gpart, double* out, hipStream_t st) {
  if (mp % kET || mp < m) return hipErrorInvalidValue;
  const unsigned T = (unsigned)(mp / kET);
  // alpha = W^T (W y)
  hipLaunchKernelGGL(kex_wy, dim3((unsigned)((mp + 3) / 4)), dim3(256), 0, st, W, mp, ys, v);
  const int nc = (int)((mp + kExactChunk - 1) / kExactChunk);
  hipLaunchKernelGGL(kex_wtv, dim3((unsigned)((mp + 255) / 256), (unsigned)nc), dim3(256), 0, st, W,
                     mp, v, (int64_t)kExactChunk, part);
  hipLaunchKernelGGL(kex_sum_parts, dim3((unsigned)((mp + 255) / 256)), dim3(256), 0, st, part, nc,
                     mp, alpha);
  hipLaunchKernelGGL(kex_scalars, dim3(1), dim3(256), 0, st, ys, alpha, diag, m, out);
  hipLaunchKernelGGL(kex_grad, dim3(T, T), dim3(256), 0, st, xs, d, m, mp, inv_ell, Hinv, alpha,
                     gpart);
  hipLaunchKernelGGL(kex_grad_final, dim3((unsigned)(d + 2)), dim3(256), 0, st, gpart,
                     (int64_t)T * (T + 1) / 2, d, inv_ell, a, sigma, out + 2);
  return hipGetLastError();
}

int64_t exact_part_doubles(int64_t mp) {
  return ((mp + kExactChunk - 1) / kExactChunk) * mp;
}

int64_t exact_gpart_doubles(int64_t mp, int d) {
  const int64_t T = mp / kET;
  return T * (T + 1) / 2 * (d + 2);
}

}  // namespace gpk
