// Host-side selection of kernel instantiations and the split-column reduction
// of the forward product (the per-dimension instantiations live in fwd.hip).
#include "gpk.h"

namespace gpk {

hipError_t fwd_d1(const FwdArgs&, hipStream_t);
hipError_t fwd_d2(const FwdArgs&, hipStream_t);
hipError_t fwd_d3(const FwdArgs&, hipStream_t);
hipError_t fwd_d4(const FwdArgs&, hipStream_t);
hipError_t fwd_d8(const FwdArgs&, hipStream_t);
hipError_t fwd_d12(const FwdArgs&, hipStream_t);
hipError_t fwd_d16(const FwdArgs&, hipStream_t);
hipError_t fwd_d24(const FwdArgs&, hipStream_t);
hipError_t fwd_d32(const FwdArgs&, hipStream_t);
hipError_t fwd_d64(const FwdArgs&, hipStream_t);

hipError_t adj_d1(const AdjArgs&, int64_t, hipStream_t);
hipError_t rff_d1(const RffArgs&, hipStream_t);
hipError_t adj_d2(const AdjArgs&, int64_t, hipStream_t);
hipError_t rff_d2(const RffArgs&, hipStream_t);
hipError_t adj_d3(const AdjArgs&, int64_t, hipStream_t);
hipError_t rff_d3(const RffArgs&, hipStream_t);
hipError_t adj_d4(const AdjArgs&, int64_t, hipStream_t);
hipError_t rff_d4(const RffArgs&, hipStream_t);
hipError_t adj_d8(const AdjArgs&, int64_t, hipStream_t);
hipError_t rff_d8(const RffArgs&, hipStream_t);
hipError_t adj_d12(const AdjArgs&, int64_t, hipStream_t);
hipError_t rff_d12(const RffArgs&, hipStream_t);
hipError_t adj_d16(const AdjArgs&, int64_t, hipStream_t);
hipError_t rff_d16(const RffArgs&, hipStream_t);
hipError_t adj_d24(const AdjArgs&, int64_t, hipStream_t);
hipError_t rff_d24(const RffArgs&, hipStream_t);
hipError_t adj_d32(const AdjArgs&, int64_t, hipStream_t);
hipError_t rff_d32(const RffArgs&, hipStream_t);
hipError_t adj_d64(const AdjArgs&, int64_t, hipStream_t);
hipError_t rff_d64(const RffArgs&, hipStream_t);

int select_D(int d) {
  static const int list[] = {1, 2, 3, 4, 8, 12, 16, 24, 32, 64};
  for (int v : list)
    if (d <= v) return v;
  return 0;
}

int select_CT(int c) {
  if (c <= 16) return 1;
  if (c <= 32) return 2;
  if (c <= 48) return 3;
  if (c <= 80) return 5;
  if (c <= 128) return 8;
  return 0;
}

int select_KT(int c) {
  if (c <= 32) return 1;
  if (c <= 64) return 2;
  if (c <= 96) return 3;
  if (c <= 128) return 4;
  if (c <= 256) return 8;
  return 0;
}

int choose_splits(int64_t rowblocks, int64_t steps) {
  // Power-of-two splits: with blockIdx -> (row block = b / S, split = b % S)
  // and round-robin dispatch over the 8 XCDs, each XCD then sees a fixed
  // subset of column splits, so its L2 holds only those slices of V.
  int S = 1;
  while (rowblocks * S < 2048 && steps / (2 * S) >= 16) S *= 2;
  return S;
}

hipError_t fwd(const FwdArgs& a, hipStream_t st) {
  switch (a.D) {
    case 1: return fwd_d1(a, st);
    case 2: return fwd_d2(a, st);
    case 3: return fwd_d3(a, st);
    case 4: return fwd_d4(a, st);
    case 8: return fwd_d8(a, st);
    case 12: return fwd_d12(a, st);
    case 16: return fwd_d16(a, st);
    case 24: return fwd_d24(a, st);
    case 32: return fwd_d32(a, st);
    case 64: return fwd_d64(a, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t adj(const AdjArgs& a, int64_t* rows, hipStream_t st) {
  if (a.n_pad % kAdjRowsPerWG) return hipErrorInvalidValue;
  const int64_t rowblocks = a.n_pad / kAdjRowsPerWG;
  *rows = rowblocks * a.S;
  switch (a.D) {
    case 1: return adj_d1(a, rowblocks, st);
    case 2: return adj_d2(a, rowblocks, st);
    case 3: return adj_d3(a, rowblocks, st);
    case 4: return adj_d4(a, rowblocks, st);
    case 8: return adj_d8(a, rowblocks, st);
    case 12: return adj_d12(a, rowblocks, st);
    case 16: return adj_d16(a, rowblocks, st);
    case 24: return adj_d24(a, rowblocks, st);
    case 32: return adj_d32(a, rowblocks, st);
    case 64: return adj_d64(a, rowblocks, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t rff(const RffArgs& a, hipStream_t st) {
  switch (a.D) {
    case 1: return rff_d1(a, st);
    case 2: return rff_d2(a, st);
    case 3: return rff_d3(a, st);
    case 4: return rff_d4(a, st);
    case 8: return rff_d8(a, st);
    case 12: return rff_d12(a, st);
    case 16: return rff_d16(a, st);
    case 24: return rff_d24(a, st);
    case 32: return rff_d32(a, st);
    case 64: return rff_d64(a, st);
    default: return hipErrorInvalidValue;
  }
}

namespace {
__global__ __launch_bounds__(256) void kfwd_reduce(const float* __restrict__ part, int S,
                                                   int64_t n1, int64_t n1_pad, int CP, int c,
                                                   float scale, const float* __restrict__ vn,
                                                   int64_t ldv, float noise,
                                                   float* __restrict__ out, int64_t ldo) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= n1 * c) return;
  const int64_t row = idx / c;
  const int col = (int)(idx % c);
  // the split sums in split order; loads 16 at a time so that many are in flight
  float sum = 0.f;
  const int64_t stride = n1_pad * CP;
  const float* p = part + row * CP + col;
  int sp = 0;
  for (; sp + 16 <= S; sp += 16) {
    float v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = p[(sp + u) * stride];
#pragma unroll
    for (int u = 0; u < 16; ++u) sum += v[u];
  }
  for (; sp < S; ++sp) sum += p[sp * stride];
  float v = scale * sum;
  if (vn) v = __builtin_fmaf(noise, vn[row * ldv + col], v);
  out[row * ldo + col] = v;
}
}  // namespace

hipError_t fwd_reduce(const float* part, int S, int64_t n1, int64_t n1_pad, int CP, int c,
                      float scale, const float* vn, int64_t ldv, float noise, float* out,
                      int64_t ldo, hipStream_t st) {
  const int64_t total = n1 * c;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(kfwd_reduce, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, part,
                     S, n1, n1_pad, CP, c, scale, vn, ldv, noise, out, ldo);
  return hipGetLastError();
}

}  // namespace gpk
