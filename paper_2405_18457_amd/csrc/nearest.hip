// The k training rows nearest to a centroid row, step 2 of the initial-
// hyperparameter heuristic (App. B, "Iterative Optimiser").
//
// Distances are squared Euclidean distances in the raw inputs, summed in FP64 in
// dimension order with every product and sum rounded on its own (no fused
// multiply-add), so any FP64 implementation of the same order selects the same
// rows.  A non-negative double orders like its 64-bit pattern, so the k-th
// smallest key T is found by an 8-pass radix select on the bit patterns (256-bin
// histograms of the rows still matching the selected prefix; the digit choice
// stays on the device).  Rows with key < T, and the lowest-index rows with
// key == T up to k, are then written in ascending row order by a two-level
// exclusive scan over blocks of 1024 rows.
#include "gpk.h"

namespace gpk {

namespace {

constexpr int kSelThreads = 256;
constexpr int kSelPer = 4;  // rows per thread in the compaction
constexpr int kSelBlock = kSelThreads * kSelPer;

__global__ __launch_bounds__(256) void knr_dist(const float* __restrict__ X, int64_t n, int d,
                                                int64_t centre, uint64_t* __restrict__ key) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int k = 0; k < d; ++k) {
    const double diff = (double)X[i * d + k] - (double)X[centre * d + k];
    const double sq = diff * diff;
    acc = acc + sq;
  }
  key[i] = (uint64_t)__double_as_longlong(acc);
}

__global__ void knr_init(SelState* __restrict__ st, int64_t k) {
  const int t = threadIdx.x;
  st->hist[t] = 0u;
  if (t == 0) {
    st->prefix = 0ull;
    st->mask = 0ull;
    st->want = k;
  }
}

__global__ __launch_bounds__(256) void knr_hist(const uint64_t* __restrict__ key, int64_t n,
                                                SelState* __restrict__ st, int shift) {
  __shared__ unsigned h[256];
  const int tid = threadIdx.x;
  h[tid] = 0u;
  __syncthreads();
  const uint64_t prefix = st->prefix, mask = st->mask;
  for (int64_t i = (int64_t)blockIdx.x * 256 + tid; i < n; i += (int64_t)gridDim.x * 256) {
    const uint64_t k = key[i];
    if ((k & mask) == prefix) atomicAdd(&h[(unsigned)(k >> shift) & 255u], 1u);
  }
  __syncthreads();
  if (h[tid]) atomicAdd(&st->hist[tid], h[tid]);
}

// Pick the digit holding the want-th smallest remaining key; clear the histogram.
__global__ void knr_pick(SelState* __restrict__ st, int shift) {
  const int tid = threadIdx.x;
  if (tid == 0) {
    const int64_t want = st->want;
    int64_t below = 0;
    int digit = 255;
    for (int b = 0; b < 256; ++b) {
      const int64_t c = st->hist[b];
      if (below + c >= want) {
        digit = b;
        break;
      }
      below += c;
    }
    st->want = want - below;
    st->prefix |= (uint64_t)digit << shift;
    st->mask |= (uint64_t)255 << shift;
  }
  __syncthreads();
  st->hist[tid] = 0u;
}

// Inclusive scan of (lt, eq) pairs over the workgroup; returns the exclusive value.
__device__ void scan_pair(int64_t& lt, int64_t& eq, int64_t* s_lt, int64_t* s_eq) {
  const int tid = threadIdx.x;
  s_lt[tid] = lt;
  s_eq[tid] = eq;
  __syncthreads();
  for (int off = 1; off < kSelThreads; off <<= 1) {
    int64_t a = 0, b = 0;
    if (tid >= off) {
      a = s_lt[tid - off];
      b = s_eq[tid - off];
    }
    __syncthreads();
    s_lt[tid] += a;
    s_eq[tid] += b;
    __syncthreads();
  }
  lt = s_lt[tid] - lt;
  eq = s_eq[tid] - eq;
}

__global__ __launch_bounds__(256) void knr_count(const uint64_t* __restrict__ key, int64_t n,
                                                 const SelState* __restrict__ st,
                                                 int64_t* __restrict__ cnt) {
  __shared__ int64_t s_lt[kSelThreads], s_eq[kSelThreads];
  const uint64_t T = st->prefix;
  const int64_t base = (int64_t)blockIdx.x * kSelBlock + threadIdx.x * kSelPer;
  int64_t lt = 0, eq = 0;
  for (int e = 0; e < kSelPer; ++e) {
    const int64_t i = base + e;
    if (i < n) {
      const uint64_t k = key[i];
      lt += k < T;
      eq += k == T;
    }
  }
  const int64_t l0 = lt, e0 = eq;
  scan_pair(lt, eq, s_lt, s_eq);
  if (threadIdx.x == kSelThreads - 1) {
    cnt[2 * blockIdx.x] = lt + l0;
    cnt[2 * blockIdx.x + 1] = eq + e0;
  }
}

// In-place exclusive scan of the per-block (lt, eq) counts, one workgroup.
__global__ __launch_bounds__(256) void knr_scan(int64_t* __restrict__ cnt, int64_t nb) {
  __shared__ int64_t s_lt[kSelThreads], s_eq[kSelThreads];
  __shared__ int64_t carry[2];
  if (threadIdx.x == 0) carry[0] = carry[1] = 0;
  __syncthreads();
  for (int64_t b0 = 0; b0 < nb; b0 += kSelThreads) {
    const int64_t b = b0 + threadIdx.x;
    int64_t lt = b < nb ? cnt[2 * b] : 0, eq = b < nb ? cnt[2 * b + 1] : 0;
    const int64_t l0 = lt, e0 = eq;
    scan_pair(lt, eq, s_lt, s_eq);
    const int64_t c0 = carry[0], c1 = carry[1];
    if (b < nb) {
      cnt[2 * b] = c0 + lt;
      cnt[2 * b + 1] = c1 + eq;
    }
    __syncthreads();
    if (threadIdx.x == kSelThreads - 1) {
      carry[0] = c0 + lt + l0;
      carry[1] = c1 + eq + e0;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void knr_write(const uint64_t* __restrict__ key, int64_t n,
                                                 const SelState* __restrict__ st,
                                                 const int64_t* __restrict__ off,
                                                 int64_t* __restrict__ idx) {
  __shared__ int64_t s_lt[kSelThreads], s_eq[kSelThreads];
  const uint64_t T = st->prefix;
  const int64_t want = st->want;
  const int64_t base = (int64_t)blockIdx.x * kSelBlock + threadIdx.x * kSelPer;
  uint64_t k[kSelPer];
  int64_t lt = 0, eq = 0;
  for (int e = 0; e < kSelPer; ++e) {
    const int64_t i = base + e;
    k[e] = i < n ? key[i] : ~0ull;
    lt += i < n && k[e] < T;
    eq += i < n && k[e] == T;
  }
  scan_pair(lt, eq, s_lt, s_eq);
  lt += off[2 * blockIdx.x];
  eq += off[2 * blockIdx.x + 1];
  for (int e = 0; e < kSelPer; ++e) {
    const int64_t i = base + e;
    if (i >= n) break;
    if (k[e] < T) {
      idx[lt + (eq < want ? eq : want)] = i;
      ++lt;
    } else if (k[e] == T) {
      if (eq < want) idx[lt + eq] = i;
      ++eq;
    }
  }
}

__global__ void knr_iota(int64_t* __restrict__ idx, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) idx[i] = i;
}

}  // namespace

int64_t nearest_blocks(int64_t n) { return (n + kSelBlock - 1) / kSelBlock; }

hipError_t nearest(const float* X, int64_t n, int d, int64_t centre, int64_t k, uint64_t* key,
                   SelState* st, int64_t* cnt, int64_t* idx, hipStream_t s) {
  if (k <= 0 || n <= 0) return hipSuccess;
  if (k >= n) {
    hipLaunchKernelGGL(knr_iota, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, idx, n);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(knr_dist, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, X, n, d, centre,
                     key);
  hipLaunchKernelGGL(knr_init, dim3(1), dim3(256), 0, s, st, k);
  const int64_t hblocks = (n + 255) / 256;
  const unsigned hb = (unsigned)(hblocks < 2048 ? hblocks : 2048);
  for (int shift = 56; shift >= 0; shift -= 8) {
    hipLaunchKernelGGL(knr_hist, dim3(hb), dim3(256), 0, s, key, n, st, shift);
    hipLaunchKernelGGL(knr_pick, dim3(1), dim3(256), 0, s, st, shift);
  }
  const int64_t nb = nearest_blocks(n);
  hipLaunchKernelGGL(knr_count, dim3((unsigned)nb), dim3(256), 0, s, key, n, st, cnt);
  hipLaunchKernelGGL(knr_scan, dim3(1), dim3(256), 0, s, cnt, nb);
  hipLaunchKernelGGL(knr_write, dim3((unsigned)nb), dim3(256), 0, s, key, n, st, cnt, idx);
  return hipGetLastError();
}

}  // namespace gpk
