// Packing (pre-scaling of the inputs, bf16 hi/lo splitting of V), FP64-
// accumulating column reductions and the vector updates of the solvers
// (App. B, Algorithms 1-3).  All of these are HBM-bound passes over
// [n, c] blocks; reductions are two-stage (per-block FP64 partials, then a
// fixed-order sum) so results are deterministic.
#include "gpk.h"

namespace gpk {

namespace {

constexpr int kThreads = 256;

inline unsigned blocks_for(int64_t total) { return (unsigned)((total + kThreads - 1) / kThreads); }

__device__ __forceinline__ uint16_t bf16_bits(float v) {
  return __builtin_bit_cast(uint16_t, (__bf16)v);
}
__device__ __forceinline__ float bf16_val(uint16_t b) {
  return __builtin_bit_cast(float, (uint32_t)b << 16);
}

__global__ void kpack_x(const float* __restrict__ X, const int32_t* __restrict__ idx, int64_t n,
                        int d, int DP, DimScale sc, float* __restrict__ Xp, int64_t n_pad) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t >= n_pad * DP) return;
  const int64_t i = t / DP;
  const int k = (int)(t % DP);
  float v = 0.f;
  if (i < n && k < d) {
    const int64_t src = idx ? (int64_t)idx[i] : i;
    v = X[src * d + k] * sc.s[k];
  }
  Xp[t] = v;
}

// Points with d <= 3 packed as [x^_0, x^_1, x^_2, |x^|^2] (unused coordinates 0);
// the largest |x^|^2 is recorded (float bits, non-negative) for the caller.
// Cross-term layout, chunk-major: Xp[(q * n_pad + i) * 4 + g] holds slot 4q + g of
// point i: scaled coordinates in slots 0..d-1, |x^|^2 in the last slot 4nk-1,
// zeros elsewhere and on padding rows.  The maximum |x^|^2 goes to maxbits.
__global__ void kpack_x_aug(const float* __restrict__ X, const int32_t* __restrict__ idx,
                            int64_t n, int d, DimScale sc, int nk, float* __restrict__ Xp,
                            int64_t n_pad, unsigned* __restrict__ stats) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n_pad) return;
  const int64_t src = i < n ? (idx ? (int64_t)idx[i] : i) : 0;
  float nn = 0.f;
  if (i < n)
    for (int k = 0; k < d; ++k) {
      const float v = X[src * d + k] * sc.s[k];
      nn = __builtin_fmaf(v, v, nn);
    }
  for (int q = 0; q < nk; ++q) {
    float v[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int slot = 4 * q + g;
      v[g] = (i < n && slot < d) ? X[src * d + slot] * sc.s[slot] : 0.f;
      if (slot == 4 * nk - 1) v[g] = nn;
    }
    reinterpret_cast<float4*>(Xp)[q * n_pad + i] = make_float4(v[0], v[1], v[2], v[3]);
  }
  if (stats && i < n) {
    atomicMax(stats, __builtin_bit_cast(unsigned, nn));
    if (!(nn <= kXTMaxNorm2)) atomicAdd(stats + 1, 1u);
    if (!(nn <= kXTMaxNorm2F32)) atomicAdd(stats + 2, 1u);
  }
}

// When the kernel tile comes from two 16x16x4 cross-term products, rows 4g..4g+3
// and 16+4g..16+4g+3 of a 32-row tile (lane group g) feed positions k = 8g..8g+7
// of the MFMA contraction index: row j = 16 h + 4 g + r sits at k = 8 g + 4 h + r.
// This returns the row at position jk.
__device__ __forceinline__ int xt_j_of_k(int jk) {
  return 16 * ((jk & 7) >> 2) + 4 * (jk >> 3) + (jk & 3);
}

constexpr int kPackMaxCP = 128;  // columns of one forward pass (16 * CT, CT <= 8)

// One workgroup per 32-row tile of V: the tile's rows (contiguous for ld == c)
// are read coalesced into LDS, then its CT blocks of 512 outputs, which are
// contiguous in the forward layout, are written 16 bytes per thread.
__device__ void load_v_tile(const float* __restrict__ V, int64_t n, int64_t ldv, int c,
                            const float* __restrict__ colscale, int CP,
                            float (*tile)[kPackMaxCP + 1]) {
  const int64_t j0 = (int64_t)blockIdx.x * 32;
  for (int e = threadIdx.x; e < 32 * CP; e += kThreads) {
    const int r = e / CP, col = e % CP;
    const int64_t j = j0 + r;
    float v = 0.f;
    if (j < n && col < c) v = V[j * ldv + col] * (colscale ? colscale[col] : 1.f);
    tile[r][col] = v;
  }
  __syncthreads();
}

// bf16 layout: element (row j, column col) at ((j / 32) CT + col / 16) 512 +
// (col % 16) 32 + jk, jk = j % 32 or its cross-term position.
__device__ void store_tile_bf16(const float (*tile)[kPackMaxCP + 1], int CT, int perm,
                                uint16_t* __restrict__ hi, uint16_t* __restrict__ lo) {
  const int64_t base = (int64_t)blockIdx.x * CT * 512;
  for (int p8 = threadIdx.x; p8 < CT * 64; p8 += kThreads) {
    const int p = 8 * p8;
    const int col = 16 * (p >> 9) + ((p & 511) >> 5);
    const int jk0 = p & 31;
    uint32_t h2[4], l2[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      uint32_t hw = 0, lw = 0;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int jk = jk0 + 2 * u + q;
        const float v = tile[perm ? xt_j_of_k(jk) : jk][col];
        const uint16_t h = bf16_bits(v);
        const uint16_t l = bf16_bits(v - bf16_val(h));
        hw |= (uint32_t)h << (16 * q);
        lw |= (uint32_t)l << (16 * q);
      }
      h2[u] = hw;
      l2[u] = lw;
    }
    *reinterpret_cast<uint4*>(hi + base + p) = make_uint4(h2[0], h2[1], h2[2], h2[3]);
    if (lo) *reinterpret_cast<uint4*>(lo + base + p) = make_uint4(l2[0], l2[1], l2[2], l2[3]);
  }
}

// FP32 layout: element (row j, column col) at ((j / 32) CT + col / 16) 512 +
// ((col % 16) 4 + g) 8 + kk, where lane group g and MFMA step kk consume row
// jj = j % 32: jj = 4 kk + g (direct kernel) or 16 (kk / 4) + 4 g + kk % 4 (the
// cross-term output order, see fwd.hip).
__device__ void store_tile_f32(const float (*tile)[kPackMaxCP + 1], int CT, int perm,
                               float* __restrict__ out) {
  const int64_t base = (int64_t)blockIdx.x * CT * 512;
  for (int p4 = threadIdx.x; p4 < CT * 128; p4 += kThreads) {
    const int p = 4 * p4;
    const int col = 16 * (p >> 9) + ((p & 511) >> 5);
    const int g = (p >> 3) & 3;
    const int kk0 = p & 7;
    float v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int kk = kk0 + u;
      v[u] = tile[perm ? 16 * (kk >> 2) + 4 * g + (kk & 3) : 4 * kk + g][col];
    }
    *reinterpret_cast<float4*>(out + base + p) = make_float4(v[0], v[1], v[2], v[3]);
  }
}

__global__ __launch_bounds__(kThreads) void kpack_v_bf16(const float* __restrict__ V, int64_t n,
                                                          int64_t ldv, int c,
                                                          const float* __restrict__ colscale,
                                                          int CT, uint16_t* __restrict__ hi,
                                                          uint16_t* __restrict__ lo, int perm) {
  __shared__ float tile[32][kPackMaxCP + 1];
  load_v_tile(V, n, ldv, c, colscale, 16 * CT, tile);
  store_tile_bf16(tile, CT, perm, hi, lo);
}

__global__ __launch_bounds__(kThreads) void kpack_v_f32(const float* __restrict__ V, int64_t n,
                                                         int64_t ldv, int c,
                                                         const float* __restrict__ colscale,
                                                         int CT, float* __restrict__ out,
                                                         int perm) {
  __shared__ float tile[32][kPackMaxCP + 1];
  load_v_tile(V, n, ldv, c, colscale, 16 * CT, tile);
  store_tile_f32(tile, CT, perm, out);
}

// SGD (App. B, Algorithm 3), the dense half of an iteration, one workgroup per
// 32-row tile: rows outside this iteration's batch (stamp != t) decay their
// momentum, Mom = rho Mom (the batch rows were updated by ksgd_sparse); every row
// moves, U += Mom; the tile of the new U is packed into the forward layout
// (bf16 hi/lo, or FP32 when f32 is given) for the next iteration's product.
__global__ __launch_bounds__(kThreads) void ksgd_update_pack(
    float* __restrict__ U, float* __restrict__ Mom, int64_t ld, const int32_t* __restrict__ stamp,
    int t, float rho, int64_t n, int c, int CT, int perm, uint16_t* __restrict__ hi,
    uint16_t* __restrict__ lo, float* __restrict__ f32) {
  __shared__ float tile[32][kPackMaxCP + 1];
  const int CP = 16 * CT;
  const int64_t j0 = (int64_t)blockIdx.x * 32;
  if (ld == c && j0 + 32 <= n) {
    // a full tile of contiguous rows: 32 c floats from j0 c (16-byte aligned)
    for (int e = threadIdx.x; e < 32 * CP; e += kThreads) {
      const int r = e / CP, col = e % CP;
      if (col >= c) tile[r][col] = 0.f;
    }
    float4* U4 = reinterpret_cast<float4*>(U + j0 * c);
    float4* M4 = reinterpret_cast<float4*>(Mom + j0 * c);
    for (int e4 = threadIdx.x; e4 < 8 * c; e4 += kThreads) {
      float4 m = M4[e4];
      float4 u = U4[e4];
      float* mv = reinterpret_cast<float*>(&m);
      float* uv = reinterpret_cast<float*>(&u);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = 4 * e4 + q;
        const int r = e / c, col = e % c;
        if (stamp[j0 + r] != t) mv[q] = rho * mv[q];
        uv[q] = uv[q] + mv[q];
        tile[r][col] = uv[q];
      }
      M4[e4] = m;
      U4[e4] = u;
    }
  } else {
    for (int e = threadIdx.x; e < 32 * CP; e += kThreads) {
      const int r = e / CP, col = e % CP;
      const int64_t j = j0 + r;
      float v = 0.f;
      if (j < n && col < c) {
        const int64_t o = j * ld + col;
        float m = Mom[o];
        if (stamp[j] != t) {
          m = rho * m;
          Mom[o] = m;
        }
        v = U[o] + m;
        U[o] = v;
      }
      tile[r][col] = v;
    }
  }
  __syncthreads();
  if (f32)
    store_tile_f32(tile, CT, perm, f32);
  else
    store_tile_bf16(tile, CT, perm, hi, lo);
}

// SGD, the sparse half (one workgroup of 1024 threads): for the batch rows
// i = idx[q], Mom[i] = rho Mom[i] - (lr / b) G[q] and stamp[i] = t; the residual
// estimate takes R[i] = G[q], and its running column sums of squares move by
// G[q]^2 - R_old[i]^2 (lanes in a fixed order, so deterministic); then
// rnorm = sqrt(sums).  Batch indices are distinct.
__global__ __launch_bounds__(1024) void ksgd_sparse(
    const float* __restrict__ G, int64_t ldg, const int32_t* __restrict__ idx, int b,
    float* __restrict__ Mom, float* __restrict__ R, int64_t ld, int c, float rho, float lrb,
    int32_t* __restrict__ stamp, int t, double* __restrict__ sumsq, double* __restrict__ rnorm,
    int* __restrict__ status) {
  __shared__ double sh[1024];
  const int lanes = 1024 / c;
  const int col = threadIdx.x % c, lane = threadIdx.x / c;
  double acc = 0.0;
  if (lane < lanes)
    for (int q = lane; q < b; q += lanes) {
      const int64_t i = idx[q];
      const float g = G[(int64_t)q * ldg + col];
      const int64_t o = i * ld + col;
      Mom[o] = __builtin_fmaf(-lrb, g, rho * Mom[o]);
      const float r = R[o];
      acc += (double)g * g - (double)r * r;
      R[o] = g;
      if (col == 0) stamp[i] = t;
    }
  sh[threadIdx.x] = lane < lanes ? acc : 0.0;
  __syncthreads();
  if (threadIdx.x < c) {
    double s = 0.0;
    for (int l = 0; l < lanes; ++l) s += sh[l * c + threadIdx.x];
    const double v = sumsq[threadIdx.x] + s;
    sumsq[threadIdx.x] = v;
    if (!isfinite(v)) atomicOr(status, 1);
    rnorm[threadIdx.x] = sqrt(v > 0.0 ? v : 0.0);
  }
}

__global__ void kfill_i32(int32_t* __restrict__ dst, int64_t count, int32_t v) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t < count) dst[t] = v;
}

__global__ void kpack_rows(const float* __restrict__ U, int64_t n, int64_t ldu, int c,
                           const float* __restrict__ colw, int CK, uint16_t* __restrict__ hi,
                           uint16_t* __restrict__ lo, float* __restrict__ f32out,
                           int64_t n_pad) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t >= n_pad * CK) return;
  const int64_t j = t / CK;
  const int col = (int)(t % CK);
  float v = 0.f;
  if (j < n && col < c) v = U[j * ldu + col] * (colw ? colw[col] : 1.f);
  if (f32out) {
    f32out[t] = v;
  } else {
    const uint16_t h = bf16_bits(v);
    hi[t] = h;
    lo[t] = bf16_bits(v - bf16_val(h));
  }
}

// Column-parallel block reduction layout: thread t handles column t % c of
// row lane t / c (c <= 256); rows of the block range are strided by the
// number of row lanes.
struct ColLanes {
  int col, lane, lanes;
  __device__ ColLanes(int c) {
    lanes = kThreads / c;
    col = threadIdx.x % c;
    lane = threadIdx.x / c;
  }
  __device__ bool active() const { return lane < lanes; }
};

__device__ void block_rows(int64_t n, int nb, int64_t& r0, int64_t& r1) {
  r0 = n * blockIdx.x / nb;
  r1 = n * (blockIdx.x + 1) / nb;
}

__device__ void finish_partial(double v, int c, const ColLanes& cl, double* __restrict__ partial) {
  __shared__ double sh[kThreads];
  sh[threadIdx.x] = cl.active() ? v : 0.0;
  __syncthreads();
  if (threadIdx.x < c) {
    double s = 0.0;
    for (int l = 0; l < cl.lanes; ++l) s += sh[l * c + threadIdx.x];
    partial[(int64_t)blockIdx.x * c + threadIdx.x] = s;
  }
}

// The row loops below take kUnroll rows of a lane per step, loads first, then
// the FP64 sums in row order (so many loads are in flight per wave; the order
// of the additions is that of the plain loop).
constexpr int kUnroll = 8;

__global__ void kcol_dot(const float* __restrict__ A, const float* __restrict__ B, int64_t n,
                         int64_t lda, int64_t ldb, int c, double* __restrict__ partial, int nb) {
  const ColLanes cl(c);
  int64_t r0, r1;
  block_rows(n, nb, r0, r1);
  double acc = 0.0;
  if (cl.active()) {
    const int64_t step = cl.lanes;
    int64_t r = r0 + cl.lane;
    for (; r + (kUnroll - 1) * step < r1; r += kUnroll * step) {
      float a[kUnroll], b[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        a[u] = A[(r + u * step) * lda + cl.col];
        b[u] = B ? B[(r + u * step) * ldb + cl.col] : a[u];
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) acc += (double)a[u] * (double)b[u];
    }
    for (; r < r1; r += step) {
      const double a = A[r * lda + cl.col];
      acc += a * (B ? (double)B[r * ldb + cl.col] : a);
    }
  }
  finish_partial(acc, c, cl, partial);
}

// Sum of partial[b * c + col] over b < nb for column col = blockIdx.x, one
// workgroup per column: thread t adds b = t, t + 256, ... in order, then a fixed
// tree over the threads (deterministic).  The result is valid in thread 0.
__device__ double col_total(const double* __restrict__ partial, int nb, int c) {
  __shared__ double sh[kThreads];
  const int col = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += kThreads) s += partial[(int64_t)b * c + col];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  return sh[0];
}

__global__ void kcol_reduce(const double* __restrict__ partial, int nb, int c,
                            double* __restrict__ out) {
  const double s = col_total(partial, nb, c);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

__global__ void knorm_to_scale(const double* __restrict__ sumsq, int c, double eps,
                               double* __restrict__ scale_d, float* __restrict__ scale_f) {
  const int col = threadIdx.x;
  if (col >= c) return;
  const double s = 1.0 / (sqrt(sumsq[col]) + eps);
  scale_d[col] = s;
  scale_f[col] = (float)s;
}

__global__ void kscale_cols(const float* __restrict__ src, int64_t lds, int64_t n, int c,
                            const float* __restrict__ scale, float* __restrict__ dst,
                            int64_t ldd, int cpad) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t >= n * cpad) return;
  const int64_t i = t / cpad;
  const int col = (int)(t % cpad);
  dst[i * ldd + col] = col < c ? src[i * lds + col] * (scale ? scale[col] : 1.f) : 0.f;
}

__global__ void kunscale_cols(const float* __restrict__ src, int64_t lds, int64_t n, int c,
                              const double* __restrict__ scale_d, float* __restrict__ dst,
                              int64_t ldd) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t >= n * c) return;
  const int64_t i = t / c;
  const int col = (int)(t % c);
  dst[i * ldd + col] = (float)((double)src[i * lds + col] / scale_d[col]);
}

__global__ void kresidual_init(const float* __restrict__ Bt, const float* __restrict__ HU,
                               float* __restrict__ R, float* __restrict__ Dv, int64_t n,
                               int64_t ld, int c, double* __restrict__ partial, int nb,
                               int set_d) {
  const ColLanes cl(c);
  int64_t r0, r1;
  block_rows(n, nb, r0, r1);
  double acc = 0.0;
  if (cl.active()) {
    const int64_t step = cl.lanes;
    int64_t r = r0 + cl.lane;
    for (; r + (kUnroll - 1) * step < r1; r += kUnroll * step) {
      float v[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int64_t o = (r + u * step) * ld + cl.col;
        v[u] = Bt[o] - HU[o];
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int64_t o = (r + u * step) * ld + cl.col;
        R[o] = v[u];
        if (set_d) Dv[o] = v[u];
        acc += (double)v[u] * v[u];
      }
    }
    for (; r < r1; r += step) {
      const int64_t o = r * ld + cl.col;
      const float v = Bt[o] - HU[o];
      R[o] = v;
      if (set_d) Dv[o] = v;
      acc += (double)v * v;
    }
  }
  finish_partial(acc, c, cl, partial);
}

__global__ void kcg_alpha(const double* __restrict__ partial, int nb, int c,
                          const double* __restrict__ gamma, double* __restrict__ alpha,
                          int* __restrict__ status) {
  const double dhd = col_total(partial, nb, c);
  const int col = blockIdx.x;
  if (threadIdx.x != 0) return;
  const bool live = gamma[col] != 0.0;
  double a = 0.0;
  if (live) {
    if (!isfinite(dhd)) atomicOr(status, 1);
    else if (!(dhd > 0.0)) atomicOr(status, 2);
    else a = gamma[col] / dhd;
  }
  alpha[col] = a;
}

__global__ void kcg_update_ur(float* __restrict__ U, float* __restrict__ R,
                              const float* __restrict__ Dv, const float* __restrict__ HD,
                              const double* __restrict__ alpha, int64_t n, int64_t ld, int c,
                              double* __restrict__ partial, int nb) {
  const ColLanes cl(c);
  int64_t r0, r1;
  block_rows(n, nb, r0, r1);
  double acc = 0.0;
  if (cl.active()) {
    const float a = (float)alpha[cl.col];
    const int64_t step = cl.lanes;
    int64_t r = r0 + cl.lane;
    for (; r + (kUnroll - 1) * step < r1; r += kUnroll * step) {
      float u[kUnroll], rv[kUnroll];
#pragma unroll
      for (int q = 0; q < kUnroll; ++q) {
        const int64_t o = (r + q * step) * ld + cl.col;
        u[q] = __builtin_fmaf(a, Dv[o], U[o]);
        rv[q] = __builtin_fmaf(-a, HD[o], R[o]);
      }
#pragma unroll
      for (int q = 0; q < kUnroll; ++q) {
        const int64_t o = (r + q * step) * ld + cl.col;
        U[o] = u[q];
        R[o] = rv[q];
        acc += (double)rv[q] * rv[q];
      }
    }
    for (; r < r1; r += step) {
      const int64_t o = r * ld + cl.col;
      U[o] = __builtin_fmaf(a, Dv[o], U[o]);
      const float rv = __builtin_fmaf(-a, HD[o], R[o]);
      R[o] = rv;
      acc += (double)rv * rv;
    }
  }
  finish_partial(acc, c, cl, partial);
}

__global__ void kcg_beta(const double* __restrict__ partial, int nb, int c,
                         double* __restrict__ gamma, double* __restrict__ beta,
                         double* __restrict__ rnorm, int* __restrict__ status) {
  const double g = col_total(partial, nb, c);
  const int col = blockIdx.x;
  if (threadIdx.x != 0) return;
  if (!isfinite(g)) atomicOr(status, 1);
  const double old = gamma[col];
  beta[col] = old != 0.0 ? g / old : 0.0;
  gamma[col] = old != 0.0 ? g : 0.0;
  if (rnorm) rnorm[col] = sqrt(g);
}

__global__ void kgamma(const double* __restrict__ partial, int nb, int c,
                       double* __restrict__ gamma, double* __restrict__ rnorm,
                       int* __restrict__ status) {
  const double g = col_total(partial, nb, c);
  const int col = blockIdx.x;
  if (threadIdx.x != 0) return;
  if (!isfinite(g)) atomicOr(status, 1);
  if (gamma) gamma[col] = g;
  rnorm[col] = sqrt(g);
}

__global__ void kcg_update_d(float* __restrict__ Dv, const float* __restrict__ R,
                             const double* __restrict__ beta, int64_t n, int64_t ld, int c) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t >= n * c) return;
  const int64_t i = t / c;
  const int col = (int)(t % c);
  const int64_t o = i * ld + col;
  Dv[o] = __builtin_fmaf((float)beta[col], Dv[o], R[o]);
}

__global__ void kset_col(const float* __restrict__ y, int64_t n, float* __restrict__ B,
                         int64_t ld, int col) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) B[i * ld + col] = y[i];
}

__global__ void krff_omega(const float* __restrict__ t, int M, int d,
                           const double* __restrict__ inv_ell, double* __restrict__ omega) {
  const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (k >= (int64_t)M * d) return;
  omega[k] = (double)t[k] * inv_ell[k % d];
}

__global__ void kgather_rows(const float* __restrict__ A, int64_t lda,
                             const int32_t* __restrict__ idx, int64_t nidx, int c,
                             float* __restrict__ out, int64_t ldo) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t >= nidx * c) return;
  const int64_t i = t / c;
  const int col = (int)(t % c);
  out[i * ldo + col] = A[(int64_t)idx[i] * lda + col];
}

__global__ void ksub_rows(float* __restrict__ G, int64_t ldg, const float* __restrict__ Bt,
                          int64_t ldb, const int32_t* __restrict__ idx, int64_t b, int c) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t >= b * c) return;
  const int64_t i = t / c;
  const int col = (int)(t % c);
  G[i * ldg + col] -= Bt[(int64_t)idx[i] * ldb + col];
}

__global__ void kadd_rows_scaled(float* __restrict__ dst, int64_t ldd,
                                 const int32_t* __restrict__ idx, const float* __restrict__ src,
                                 int64_t lds, int64_t b, int c, float alpha) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t >= b * c) return;
  const int64_t i = t / c;
  const int col = (int)(t % c);
  const int64_t o = (int64_t)idx[i] * ldd + col;
  dst[o] = __builtin_fmaf(alpha, src[i * lds + col], dst[o]);
}

__global__ void kscatter_rows(float* __restrict__ dst, int64_t ldd,
                              const int32_t* __restrict__ idx, const float* __restrict__ src,
                              int64_t lds, int64_t b, int c) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t >= b * c) return;
  const int64_t i = t / c;
  const int col = (int)(t % c);
  dst[(int64_t)idx[i] * ldd + col] = src[i * lds + col];
}

__global__ void kaxpy_cols(float* __restrict__ Y, const float* __restrict__ X, int64_t n,
                           int64_t ld, int c, float alpha) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t >= n * c) return;
  const int64_t o = (t / c) * ld + (t % c);
  Y[o] = __builtin_fmaf(alpha, X[o], Y[o]);
}

__global__ void kcopy_cols(const float* __restrict__ src, int64_t lds, int64_t n, int c,
                           float* __restrict__ dst, int64_t ldd) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t >= n * c) return;
  const int64_t i = t / c;
  const int col = (int)(t % c);
  dst[i * ldd + col] = src[i * lds + col];
}

// D[i][j] = U[i][0] - U[i][1 + j] for j < s (pathwise posterior weights v_y - zhat_j).
__global__ void kpost_diff(const float* __restrict__ U, int64_t ldu, int64_t n, int s,
                           float* __restrict__ D) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t >= n * s) return;
  const int64_t i = t / s;
  const int j = (int)(t % s);
  D[t] = U[i * ldu] - U[i * ldu + 1 + j];
}

__global__ void kfill(float* __restrict__ dst, int64_t count, float v) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t < count) dst[t] = v;
}

__global__ void kcheck_finite(const float* __restrict__ A, int64_t n, int64_t ld, int c,
                              int* __restrict__ status) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t >= n * c) return;
  if (!isfinite(A[(t / c) * ld + (t % c)])) atomicOr(status, 1);
}

__global__ void ksgd_momentum(float* __restrict__ Mom, const float* __restrict__ G,
                              const int32_t* __restrict__ idx, int64_t b, int64_t n, int64_t ld,
                              int c, float rho, float lrb) {
  // Mom = rho Mom everywhere, then Mom[idx] -= lr/b G (indices are distinct).
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t < n * c) {
    const int64_t o = (t / c) * ld + (t % c);
    Mom[o] *= rho;
  }
}

// Fingerprint of a float array: sum over t of (bits(x_t) + 1) (2t + 1) K mod 2^64,
// position-dependent and independent of the summation order.
__global__ void kchecksum(const float* __restrict__ x, int64_t count,
                          unsigned long long* __restrict__ out) {
  unsigned long long h = 0;
  for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < count;
       t += (int64_t)gridDim.x * kThreads) {
    const unsigned long long b = __builtin_bit_cast(unsigned, x[t]);
    h += (b + 1ull) * (2ull * (unsigned long long)t + 1ull) * 0x9E3779B97F4A7C15ull;
  }
  atomicAdd(out, h);
}

}  // namespace

hipError_t pack_x(const float* X, int64_t n, int d, int DP, const DimScale& sc, float* Xp,
                  int64_t n_pad, hipStream_t st) {
  hipLaunchKernelGGL(kpack_x, dim3(blocks_for(n_pad * DP)), dim3(kThreads), 0, st, X,
                     (const int32_t*)nullptr, n, d, DP, sc, Xp, n_pad);
  return hipGetLastError();
}

hipError_t pack_x_rows(const float* X, const int32_t* idx, int64_t nidx, int d, int DP,
                       const DimScale& sc, float* Xp, int64_t n_pad, hipStream_t st) {
  hipLaunchKernelGGL(kpack_x, dim3(blocks_for(n_pad * DP)), dim3(kThreads), 0, st, X, idx, nidx,
                     d, DP, sc, Xp, n_pad);
  return hipGetLastError();
}

hipError_t pack_x_aug(const float* X, const int32_t* idx, int64_t n, int d, const DimScale& sc,
                      int nk, float* Xp, int64_t n_pad, unsigned* stats, hipStream_t st) {
  hipLaunchKernelGGL(kpack_x_aug, dim3(blocks_for(n_pad)), dim3(kThreads), 0, st, X, idx, n, d, sc,
                     nk, Xp, n_pad, stats);
  return hipGetLastError();
}

hipError_t pack_v_bf16(const float* V, int64_t n, int64_t ldv, int c, const float* colscale,
                       int CT, uint16_t* hi, uint16_t* lo, int64_t n_pad, bool perm,
                       hipStream_t st) {
  if (CT < 1 || 16 * CT > kPackMaxCP || c > 16 * CT || n_pad % 32 != 0 || n > n_pad)
    return hipErrorInvalidValue;
  if (n_pad == 0) return hipSuccess;
  hipLaunchKernelGGL(kpack_v_bf16, dim3((unsigned)(n_pad / 32)), dim3(kThreads), 0, st, V, n, ldv,
                     c, colscale, CT, hi, lo, (int)perm);
  return hipGetLastError();
}

hipError_t pack_v_f32(const float* V, int64_t n, int64_t ldv, int c, const float* colscale,
                      int CT, float* out, int64_t n_pad, bool perm, hipStream_t st) {
  if (CT < 1 || 16 * CT > kPackMaxCP || c > 16 * CT || n_pad % 32 != 0 || n > n_pad)
    return hipErrorInvalidValue;
  if (n_pad == 0) return hipSuccess;
  hipLaunchKernelGGL(kpack_v_f32, dim3((unsigned)(n_pad / 32)), dim3(kThreads), 0, st, V, n, ldv,
                     c, colscale, CT, out, (int)perm);
  return hipGetLastError();
}

hipError_t pack_rows_bf16(const float* U, int64_t n, int64_t ldu, int c, const float* colw,
                          int KT, uint16_t* hi, uint16_t* lo, int64_t n_pad, hipStream_t st) {
  hipLaunchKernelGGL(kpack_rows, dim3(blocks_for(n_pad * 32 * KT)), dim3(kThreads), 0, st, U, n,
                     ldu, c, colw, 32 * KT, hi, lo, (float*)nullptr, n_pad);
  return hipGetLastError();
}

hipError_t pack_rows_f32(const float* U, int64_t n, int64_t ldu, int c, const float* colw,
                         int KT, float* out, int64_t n_pad, hipStream_t st) {
  hipLaunchKernelGGL(kpack_rows, dim3(blocks_for(n_pad * 32 * KT)), dim3(kThreads), 0, st, U, n,
                     ldu, c, colw, 32 * KT, (uint16_t*)nullptr, (uint16_t*)nullptr, out, n_pad);
  return hipGetLastError();
}

int reduce_blocks(int64_t n) {
  int64_t nb = (n + 255) / 256;
  if (nb > 1024) nb = 1024;
  if (nb < 1) nb = 1;
  return (int)nb;
}

hipError_t col_dot_partial(const float* A, const float* B, int64_t n, int64_t lda, int64_t ldb,
                           int c, double* partial, int nb, hipStream_t st) {
  hipLaunchKernelGGL(kcol_dot, dim3(nb), dim3(kThreads), 0, st, A, B, n, lda, ldb, c, partial,
                     nb);
  return hipGetLastError();
}

hipError_t col_reduce(const double* partial, int nb, int c, double* out, hipStream_t st) {
  if (c <= 0) return hipSuccess;
  hipLaunchKernelGGL(kcol_reduce, dim3(c), dim3(kThreads), 0, st, partial, nb, c, out);
  return hipGetLastError();
}

hipError_t norm_to_scale(const double* sumsq, int c, double eps, double* scale_d, float* scale_f,
                         hipStream_t st) {
  hipLaunchKernelGGL(knorm_to_scale, dim3(1), dim3(kThreads), 0, st, sumsq, c, eps, scale_d,
                     scale_f);
  return hipGetLastError();
}

hipError_t scale_cols(const float* src, int64_t lds, int64_t n, int c, const float* scale,
                      float* dst, int64_t ldd, int cpad, hipStream_t st) {
  if (n * cpad == 0) return hipSuccess;
  hipLaunchKernelGGL(kscale_cols, dim3(blocks_for(n * cpad)), dim3(kThreads), 0, st, src, lds, n,
                     c, scale, dst, ldd, cpad);
  return hipGetLastError();
}

hipError_t unscale_cols(const float* src, int64_t lds, int64_t n, int c, const double* scale_d,
                        float* dst, int64_t ldd, hipStream_t st) {
  if (n * c == 0) return hipSuccess;
  hipLaunchKernelGGL(kunscale_cols, dim3(blocks_for(n * c)), dim3(kThreads), 0, st, src, lds, n,
                     c, scale_d, dst, ldd);
  return hipGetLastError();
}

hipError_t residual_init(const float* Bt, const float* HU, float* R, float* Dv, int64_t n,
                         int64_t ld, int c, double* partial, int nb, bool set_d, hipStream_t st) {
  hipLaunchKernelGGL(kresidual_init, dim3(nb), dim3(kThreads), 0, st, Bt, HU, R, Dv, n, ld, c,
                     partial, nb, (int)set_d);
  return hipGetLastError();
}

hipError_t cg_alpha(const double* partial, int nb, int c, const double* gamma, double* alpha,
                    int* status, hipStream_t st) {
  if (c <= 0) return hipSuccess;
  hipLaunchKernelGGL(kcg_alpha, dim3(c), dim3(kThreads), 0, st, partial, nb, c, gamma, alpha,
                     status);
  return hipGetLastError();
}

hipError_t cg_update_ur(float* U, float* R, const float* Dv, const float* HD,
                        const double* alpha, int64_t n, int64_t ld, int c, double* partial,
                        int nb, hipStream_t st) {
  hipLaunchKernelGGL(kcg_update_ur, dim3(nb), dim3(kThreads), 0, st, U, R, Dv, HD, alpha, n, ld,
                     c, partial, nb);
  return hipGetLastError();
}

hipError_t cg_beta(const double* partial, int nb, int c, double* gamma, double* beta,
                   double* rnorm, int* status, hipStream_t st) {
  if (c <= 0) return hipSuccess;
  hipLaunchKernelGGL(kcg_beta, dim3(c), dim3(kThreads), 0, st, partial, nb, c, gamma, beta, rnorm,
                     status);
  return hipGetLastError();
}

hipError_t gamma_from_partial(const double* partial, int nb, int c, double* gamma,
                              double* rnorm, int* status, hipStream_t st) {
  if (c <= 0) return hipSuccess;
  hipLaunchKernelGGL(kgamma, dim3(c), dim3(kThreads), 0, st, partial, nb, c, gamma, rnorm, status);
  return hipGetLastError();
}

hipError_t cg_update_d(float* Dv, const float* R, const double* beta, int64_t n, int64_t ld,
                       int c, hipStream_t st) {
  if (n * c == 0) return hipSuccess;
  hipLaunchKernelGGL(kcg_update_d, dim3(blocks_for(n * c)), dim3(kThreads), 0, st, Dv, R, beta, n,
                     ld, c);
  return hipGetLastError();
}

hipError_t weighted_dot_partial(const float* U, int64_t ldu, const float* W, int64_t ldw,
                                int64_t n, int c, double* partial, int nb, hipStream_t st) {
  return col_dot_partial(U, W, n, ldu, ldw, c, partial, nb, st);
}

hipError_t rff_omega(const float* t, int M, int d, const double* inv_ell_dev, double* omega,
                     hipStream_t st) {
  hipLaunchKernelGGL(krff_omega, dim3(blocks_for((int64_t)M * d)), dim3(kThreads), 0, st, t, M,
                     d, inv_ell_dev, omega);
  return hipGetLastError();
}

hipError_t set_col(const float* y, int64_t n, float* B, int64_t ld, int col, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(kset_col, dim3(blocks_for(n)), dim3(kThreads), 0, st, y, n, B, ld, col);
  return hipGetLastError();
}

hipError_t gather_rows(const float* A, int64_t lda, const int32_t* idx, int64_t nidx, int c,
                       float* out, int64_t ldo, hipStream_t st) {
  if (nidx * c == 0) return hipSuccess;
  hipLaunchKernelGGL(kgather_rows, dim3(blocks_for(nidx * c)), dim3(kThreads), 0, st, A, lda, idx,
                     nidx, c, out, ldo);
  return hipGetLastError();
}

hipError_t sub_rows(float* G, int64_t ldg, const float* Bt, int64_t ldb, const int32_t* idx,
                    int64_t b, int c, hipStream_t st) {
  if (b * c == 0) return hipSuccess;
  hipLaunchKernelGGL(ksub_rows, dim3(blocks_for(b * c)), dim3(kThreads), 0, st, G, ldg, Bt, ldb,
                     idx, b, c);
  return hipGetLastError();
}

hipError_t add_rows_scaled(float* dst, int64_t ldd, const int32_t* idx, const float* src,
                           int64_t lds, int64_t b, int c, float alpha, hipStream_t st) {
  if (b * c == 0) return hipSuccess;
  hipLaunchKernelGGL(kadd_rows_scaled, dim3(blocks_for(b * c)), dim3(kThreads), 0, st, dst, ldd,
                     idx, src, lds, b, c, alpha);
  return hipGetLastError();
}

hipError_t sgd_momentum(float* Mom, const float* G, const int32_t* idx, int64_t b, int64_t n,
                        int64_t ld, int c, float rho, float lrb, hipStream_t st) {
  if (n * c > 0)
    hipLaunchKernelGGL(ksgd_momentum, dim3(blocks_for(n * c)), dim3(kThreads), 0, st, Mom, G, idx,
                       b, n, ld, c, rho, lrb);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return add_rows_scaled(Mom, ld, idx, G, ld, b, c, -lrb, st);
}

hipError_t sgd_sparse(const float* G, int64_t ldg, const int32_t* idx, int b, float* Mom,
                      float* R, int64_t ld, int c, float rho, float lrb, int32_t* stamp, int t,
                      double* sumsq, double* rnorm, int* status, hipStream_t st) {
  if (c < 1 || c > 256) return hipErrorInvalidValue;
  if (b <= 0) return hipSuccess;
  hipLaunchKernelGGL(ksgd_sparse, dim3(1), dim3(1024), 0, st, G, ldg, idx, b, Mom, R, ld, c, rho,
                     lrb, stamp, t, sumsq, rnorm, status);
  return hipGetLastError();
}

hipError_t sgd_update_pack(float* U, float* Mom, int64_t ld, const int32_t* stamp, int t,
                           float rho, int64_t n, int c, int CT, bool perm, int64_t n_pad,
                           uint16_t* hi, uint16_t* lo, float* f32, hipStream_t st) {
  if (CT < 1 || 16 * CT > kPackMaxCP || c > 16 * CT || n_pad % 32 != 0 || n > n_pad)
    return hipErrorInvalidValue;
  if (n_pad == 0) return hipSuccess;
  hipLaunchKernelGGL(ksgd_update_pack, dim3((unsigned)(n_pad / 32)), dim3(kThreads), 0, st, U, Mom,
                     ld, stamp, t, rho, n, c, CT, (int)perm, hi, lo, f32);
  return hipGetLastError();
}

hipError_t fill_i32(int32_t* dst, int64_t count, int32_t v, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(kfill_i32, dim3(blocks_for(count)), dim3(kThreads), 0, st, dst, count, v);
  return hipGetLastError();
}

hipError_t sgd_finish(float* U, float* R, const float* Mom, const float* G, const int32_t* idx,
                      int64_t b, int64_t n, int64_t ld, int c, hipStream_t st) {
  hipError_t e = axpy_cols(U, Mom, n, ld, c, 1.f, st);
  if (e != hipSuccess) return e;
  // R[idx] = G  (scatter of the batch residual estimate)
  if (b * c == 0) return hipSuccess;
  hipLaunchKernelGGL(kscatter_rows, dim3(blocks_for(b * c)), dim3(kThreads), 0, st, R, ld, idx,
                     G, ld, b, c);
  return hipGetLastError();
}

hipError_t axpy_cols(float* Y, const float* X, int64_t n, int64_t ld, int c, float alpha,
                     hipStream_t st) {
  if (n * c == 0) return hipSuccess;
  hipLaunchKernelGGL(kaxpy_cols, dim3(blocks_for(n * c)), dim3(kThreads), 0, st, Y, X, n, ld, c,
                     alpha);
  return hipGetLastError();
}

hipError_t copy_cols(const float* src, int64_t lds, int64_t n, int c, float* dst, int64_t ldd,
                     hipStream_t st) {
  if (n * c == 0) return hipSuccess;
  hipLaunchKernelGGL(kcopy_cols, dim3(blocks_for(n * c)), dim3(kThreads), 0, st, src, lds, n, c,
                     dst, ldd);
  return hipGetLastError();
}

hipError_t post_diff(const float* U, int64_t ldu, int64_t n, int s, float* D, hipStream_t st) {
  hipLaunchKernelGGL(kpost_diff, dim3(blocks_for(n * s)), dim3(kThreads), 0, st, U, ldu, n, s, D);
  return hipGetLastError();
}

hipError_t fill(float* dst, int64_t count, float v, hipStream_t st) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(kfill, dim3(blocks_for(count)), dim3(kThreads), 0, st, dst, count, v);
  return hipGetLastError();
}

hipError_t check_finite(const float* A, int64_t n, int64_t ld, int c, int* status,
                        hipStream_t st) {
  if (n * c == 0) return hipSuccess;
  hipLaunchKernelGGL(kcheck_finite, dim3(blocks_for(n * c)), dim3(kThreads), 0, st, A, n, ld, c,
                     status);
  return hipGetLastError();
}

hipError_t checksum_f32(const float* x, int64_t count, unsigned long long* out, hipStream_t st) {
  const int64_t blocks = (count + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(kchecksum, dim3((unsigned)(blocks < 1024 ? (blocks > 0 ? blocks : 1) : 1024)),
                     dim3(kThreads), 0, st, x, count, out);
  return hipGetLastError();
}

}  // namespace gpk
