// Rank-k pivoted Cholesky preconditioner of conjugate gradients (App. B: CG
// with its preconditioner P(.), a rank-100 pivoted Cholesky factor in the
// paper's experiments).
//
//   construction   greedy partial Cholesky of K, one pivot per step: the row
//                  with the largest remaining diagonal (lowest index on ties),
//                  l_j = (K[:, p] - L[:, :j] L[p, :j]^T) / sqrt(d_p),
//                  d <- d - l_j^2.  Two launches per step (column + pivot);
//                  the pivot stays in device memory, so the k steps run without
//                  host round trips.  Kernel columns are evaluated in FP64 from
//                  the raw inputs.  The solver's preconditioner keeps the factor
//                  in FP32 (the dot products with earlier columns read half the
//                  bytes; sums stay FP64); gp_pivoted_cholesky keeps it in FP64.
//   inverse        M = (sigma^2 I + L^T L)^-1 (k x k, FP64): the Gram matrix on
//                  FP64 MFMA once per factor; per sigma the shifted matrix,
//                  padded with the identity to a multiple of 64, goes through
//                  the recursive matrix-core Cholesky with inverse factor of the
//                  exact-likelihood code (spd_inverse), and kpc_mirror fills in
//                  the upper triangle.
//   apply          P^-1 R = (R - L (M (L^T R))) / sigma^2 (Woodbury), the skinny
//                  products and M (L^T R) LDS-tiled on FP64 MFMA with FP64
//                  accumulation (with 65 columns the last one runs on the vector
//                  ALU beside the 64 matrix-core columns); the subtraction
//                  cancels most of R, which is why the arithmetic is FP64.  The
//                  products read an FP32 copy of the factor (the
//                  preconditioner is P = L~ L~^T + sigma^2 I for that copy L~,
//                  Gram matrix included, so P stays exactly SPD).
//
// L is stored transposed, L[t * ldl + i] (row t = factor column t), so that both
// the construction's per-row dot products and the MFMA operand loads are
// coalesced along i.
#include "gpk.h"

namespace gpk {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kPcThreads = 256;

__global__ void kpc_init(double* __restrict__ diag, int64_t n, double a2, PcState* __restrict__ s,
                         int32_t* __restrict__ piv) {
  const int64_t i = (int64_t)blockIdx.x * kPcThreads + threadIdx.x;
  if (i < n) diag[i] = a2;
  if (i == 0) {
    s->p = 0;  // every diagonal entry equals a^2: the tie goes to index 0
    s->stop = 0;
    s->rank = 0;
    s->dp = a2;
    piv[0] = 0;
  }
}

// (value, index) maximum with the lowest index on ties; idx < 0 marks "none".
__device__ __forceinline__ bool better(double v, int64_t i, double bv, int64_t bi) {
  if (i < 0) return false;
  if (bi < 0) return true;
  return v > bv || (v == bv && i < bi);
}

__device__ void block_argmax(double v, int64_t i, double* sv, int64_t* si, double* out_v,
                             int64_t* out_i) {
  const int tid = threadIdx.x;
  sv[tid] = v;
  si[tid] = i;
  __syncthreads();
  for (int off = kPcThreads / 2; off > 0; off >>= 1) {
    if (tid < off && better(sv[tid + off], si[tid + off], sv[tid], si[tid])) {
      sv[tid] = sv[tid + off];
      si[tid] = si[tid + off];
    }
    __syncthreads();
  }
  if (tid == 0) {
    *out_v = sv[0];
    *out_i = si[0];
  }
}

// Step j: factor column j for pivot s->p, diagonal update, per-block argmax.
// Each thread owns kPcRows consecutive rows, so the dot products with the
// previous factor columns run as kPcRows independent FP64 chains fed by one
// vector load per column.  F32: the factor is kept only as FP32 (L32), which
// halves the bytes these dot products read (products and sums stay FP64);
// otherwise the factor is FP64 (L) throughout.
constexpr int kPcRows = 4;

template <bool F32>
__global__ __launch_bounds__(kPcThreads) void kpc_column(
    const float* __restrict__ X, int64_t n, int d, const double* __restrict__ ell, double a2,
    double* __restrict__ L, float* __restrict__ L32, int64_t ldl, int j,
    double* __restrict__ diag, const PcState* __restrict__ s, const double* __restrict__ lp,
    double* __restrict__ pval, int64_t* __restrict__ pidx) {
  __shared__ double sv[kPcThreads];
  __shared__ int64_t si[kPcThreads];
  const int64_t i0 = ((int64_t)blockIdx.x * kPcThreads + threadIdx.x) * kPcRows;
  const int64_t p = s->p;
  const double dp = s->dp;
  const bool stop = s->stop != 0;
  double nd = 0.0;
  int64_t ni = -1;
  if (!stop && i0 < n) {
    double kv[kPcRows];
#pragma unroll
    for (int q = 0; q < kPcRows; ++q) {
      const int64_t i = i0 + q < n ? i0 + q : n - 1;
      double r2 = 0.0;
      for (int k = 0; k < d; ++k) {
        const double t = (double)X[i * d + k] / ell[k] - (double)X[p * d + k] / ell[k];
        r2 += t * t;
      }
      const double r = sqrt(3.0 * r2);
      kv[q] = a2 * (1.0 + r) * exp(-r);
    }
    // F32: ldl is a multiple of kPcRows, so the vector loads stay inside each
    // factor column (rows >= n load unused values that are never stored)
    if (F32) {
#pragma unroll 8
      for (int t = 0; t < j; ++t) {
        const float4 v = *reinterpret_cast<const float4*>(L32 + (int64_t)t * ldl + i0);
        const double w = lp[t];
        kv[0] -= (double)v.x * w;
        kv[1] -= (double)v.y * w;
        kv[2] -= (double)v.z * w;
        kv[3] -= (double)v.w * w;
      }
    } else {
      for (int t = 0; t < j; ++t) {
        const double w = lp[t];
#pragma unroll
        for (int q = 0; q < kPcRows; ++q)
          if (i0 + q < n) kv[q] -= L[(int64_t)t * ldl + i0 + q] * w;
      }
    }
    const double inv = 1.0 / sqrt(dp);
#pragma unroll
    for (int q = 0; q < kPcRows; ++q) {
      const int64_t i = i0 + q;
      if (i >= n) break;
      const double l = kv[q] * inv;
      if (F32)
        L32[(int64_t)j * ldl + i] = (float)l;
      else
        L[(int64_t)j * ldl + i] = l;
      double di = diag[i] - l * l;
      if (i == p) di = 0.0;
      diag[i] = di;
      if (better(di, i, nd, ni)) {
        nd = di;
        ni = i;
      }
    }
  }
  block_argmax(nd, ni, sv, si, pval + blockIdx.x, pidx + blockIdx.x);
}

// After step j: the next pivot from the block maxima, its remaining diagonal and
// its factor row L[p, :j+1] (gathered for the next step's dot products).
template <bool F32>
__global__ __launch_bounds__(kPcThreads) void kpc_pivot(const double* __restrict__ pval,
                                                        const int64_t* __restrict__ pidx,
                                                        int nparts, const double* __restrict__ L,
                                                        const float* __restrict__ L32,
                                                        int64_t ldl, int j, int k,
                                                        PcState* __restrict__ s,
                                                        double* __restrict__ lp,
                                                        int32_t* __restrict__ piv) {
  __shared__ double sv[kPcThreads];
  __shared__ int64_t si[kPcThreads];
  __shared__ double bv;
  __shared__ int64_t bi;
  const bool stop = s->stop != 0;
  __syncthreads();
  if (stop) return;  // uniform across the block
  double v = 0.0;
  int64_t idx = -1;
  for (int b = threadIdx.x; b < nparts; b += kPcThreads)
    if (better(pval[b], pidx[b], v, idx)) {
      v = pval[b];
      idx = pidx[b];
    }
  block_argmax(v, idx, sv, si, &bv, &bi);
  __syncthreads();
  if (j + 1 >= k) {
    if (threadIdx.x == 0) s->rank = j + 1;
    return;
  }
  if (bi >= 0 && bv > 0.0) {
    for (int t = threadIdx.x; t <= j; t += kPcThreads)
      lp[t] = F32 ? (double)L32[(int64_t)t * ldl + bi] : L[(int64_t)t * ldl + bi];
    if (threadIdx.x == 0) {
      s->rank = j + 1;
      s->p = bi;
      s->dp = bv;
      piv[j + 1] = (int32_t)bi;
    }
  } else if (threadIdx.x == 0) {
    s->rank = j + 1;
    s->stop = 1;
  }
}

// part[z][a][b] = sum over rows i of chunk z of L[a][i] * Bop(i, b) for a < ka,
// b < nb, with L the FP32 copy of the factor ([ka][ldl]) and
//   BMODE 0: Bop(i, b) = R[i * ldr + b]   (FP32 row-major solver vectors)
//   BMODE 1: Bop(i, b) = L[b * ldl + i]   (the factor itself: the Gram matrix).
// One workgroup: a 64 (a) x 16*NBT (b) tile; tiles of 32 rows i are staged in
// LDS as FP64 and every wave runs v_mfma_f64_16x16x4f64 on 16 a-rows x NBT
// column tiles (A lane: L[a0 + 16w + l%16][i + 4s + l/16]; B lane:
// Bop(i + 4s + l/16, b0 + 16u + l%16); D lane q: (a0 + 16w + 4q + l/16,
// b0 + 16u + l%16)).  Products of two FP32 values are exact in FP64.  X1 adds
// the column b0 + 16*NBT on the vector ALU: each lane accumulates its A value
// times that column's entry in FP64, and the four lane groups (l/16) are summed
// at the end.  WPE is the occupancy the register allocation aims for (4 waves
// per SIMD is also the LDS limit; the all-FP64 instantiation needs 3 to stay
// clear of spills).
constexpr int kTI = 32;  // rows i per LDS stage
static_assert(kTI * 8 == 256, "the factor-tile loaders cover kTI with 4 or 8 threads of 8 values");

// Eight consecutive entries [i, i + 8) of row a of a [rows][ldl] operand, zero
// past iend or the row count; two 16-byte loads when the segment is whole (FP32
// rows start at multiples of 64 values and every segment at a multiple of 8).
template <typename T>
__device__ __forceinline__ void load_seg(const T* __restrict__ L, int rows, int64_t ldl, int a,
                                         int64_t i, int64_t iend, T (&v)[8]) {
  if constexpr (sizeof(T) == 4) {
    if (a < rows && i + 8 <= iend) {
      const float4* q = reinterpret_cast<const float4*>(L + (int64_t)a * ldl + i);
      const float4 u0 = q[0], u1 = q[1];
      v[0] = u0.x; v[1] = u0.y; v[2] = u0.z; v[3] = u0.w;
      v[4] = u1.x; v[5] = u1.y; v[6] = u1.z; v[7] = u1.w;
      return;
    }
  }
#pragma unroll
  for (int e = 0; e < 8; ++e)
    v[e] = (a < rows && i + e < iend) ? L[(int64_t)a * ldl + i + e] : T(0);
}

template <int NBT, int BMODE, typename TL, typename TR = float, int WPE = 4, bool X1 = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) void kpc_tn(const TL* __restrict__ L, int64_t ldl, int ka,
                                              int64_t n, const TR* __restrict__ R,
                                              int64_t ldr, int nb, int64_t csize,
                                              double* __restrict__ part) {
  constexpr int NB = 16 * NBT;            // columns on the matrix cores
  constexpr int NBX = NB + (X1 ? 1 : 0);  // columns of the B tile
  static_assert(BMODE == 0 || NB == 64, "the factor-operand loader covers 64 columns");
  static_assert(!X1 || BMODE == 0, "the extra column is a column of R");
  __shared__ double As[64][kTI + 1];
  __shared__ double Bs[kTI][NBX + 1];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int la = lane & 15, lk = lane >> 4;
  const int a0 = blockIdx.x * 64;
  const int b0 = blockIdx.y * NB;
  const int64_t i0 = (int64_t)blockIdx.z * csize;
  const int64_t i1 = i0 + csize < n ? i0 + csize : n;
  f64x4 acc[NBT];
#pragma unroll
  for (int u = 0; u < NBT; ++u) acc[u] = f64x4{0.0, 0.0, 0.0, 0.0};
  double xacc = 0.0;  // X1: the extra column b0 + NB on the vector ALU
  // loaders: the factor tile with 4 threads per 32-value row segment (8 values
  // each); BMODE 0 reads the kTI x NBX B tile as consecutive entries, BPT per
  // thread (entry f = 256 e + tid: row f / NBX, column f % NBX), so that the
  // lanes of a wave load consecutive addresses of a row; BMODE 1 like the
  // factor tile.  The next stage is fetched into registers while the MFMAs of
  // the current one run.
  const int lr = tid >> 2, lc = (tid & 3) * 8;
  constexpr int BT = kTI * NBX;
  constexpr int BPT = (BT + 255) / 256;
  TL ra[8];
  TR rb[BMODE == 0 ? BPT : 1];
  TL rl[8];
  auto fetch = [&](int64_t i) {
    load_seg(L, ka, ldl, a0 + lr, i + lc, i1, ra);
    if constexpr (BMODE == 0) {
#pragma unroll
      for (int e = 0; e < BPT; ++e) {
        const int f = 256 * e + tid;
        const int64_t ii = i + f / NBX;
        const int bcol = b0 + f % NBX;
        rb[e] = (f < BT && ii < i1 && bcol < nb) ? R[ii * ldr + bcol] : TR(0);
      }
    } else {
      load_seg(L, nb, ldl, b0 + lr, i + lc, i1, rl);
    }
  };
  if (i0 < i1) fetch(i0);
  for (int64_t i = i0; i < i1; i += kTI) {
#pragma unroll
    for (int e = 0; e < 8; ++e) As[lr][lc + e] = (double)ra[e];
    if constexpr (BMODE == 0) {
#pragma unroll
      for (int e = 0; e < BPT; ++e) {
        const int f = 256 * e + tid;
        if (f < BT) Bs[f / NBX][f % NBX] = (double)rb[e];
      }
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) Bs[lc + e][lr] = (double)rl[e];
    }
    __syncthreads();
    if (i + kTI < i1) fetch(i + kTI);
#pragma unroll
    for (int s4 = 0; s4 < kTI / 4; ++s4) {
      const double av = As[16 * wave + la][4 * s4 + lk];
#pragma unroll
      for (int u = 0; u < NBT; ++u)
        acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Bs[4 * s4 + lk][16 * u + la], acc[u], 0,
                                                      0, 0);
      if constexpr (X1) xacc = fma(av, Bs[4 * s4 + lk][NB], xacc);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < NBT; ++u)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ar = a0 + 16 * wave + 4 * q + lk;
      const int bc = b0 + 16 * u + la;
      if (ar < ka && bc < nb) part[((int64_t)blockIdx.z * ka + ar) * nb + bc] = acc[u][q];
    }
  if constexpr (X1) {
    // the four lane groups hold the sums over i = 4s + 0..3: add them pairwise
    xacc += __shfl_xor(xacc, 16);
    xacc += __shfl_xor(xacc, 32);
    const int ar = a0 + 16 * wave + la;
    if (lk == 0 && ar < ka && b0 + NB < nb)
      part[((int64_t)blockIdx.z * ka + ar) * nb + b0 + NB] = xacc;
  }
}

// out[a][b] = sum_z part[z][a][b] (fixed order).  With diag_add: out is the
// kp x kp Cholesky input sigma^2 I + G, identity on the padding.
__global__ void kpc_sum(const double* __restrict__ part, int nz, int ka, int nb,
                        double* __restrict__ out, int ldo, int kp, double diag_add, int square) {
  const int64_t t = (int64_t)blockIdx.x * kPcThreads + threadIdx.x;
  if (square) {
    if (t >= (int64_t)kp * kp) return;
    const int a = (int)(t / kp), b = (int)(t % kp);
    double v;
    if (a < ka && b < ka) {
      v = 0.0;
      for (int z = 0; z < nz; ++z) v += part[((int64_t)z * ka + a) * nb + b];
      if (a == b) v += diag_add;
    } else {
      v = a == b ? 1.0 : 0.0;
    }
    out[(int64_t)a * ldo + b] = v;
  } else {
    if (t >= (int64_t)ka * nb) return;
    const int a = (int)(t / nb), b = (int)(t % nb);
    double v = 0.0;
    for (int z = 0; z < nz; ++z) v += part[((int64_t)z * ka + a) * nb + b];
    out[(int64_t)a * ldo + b] = v;
  }
}

// M[a][b] = A[max(a, b)][min(a, b)]: the full symmetric matrix from its lower
// 64 x 64 tiles (the lower tiles hold whole 64 x 64 blocks, both triangles of a
// diagonal tile included).
__global__ void kpc_mirror(const double* __restrict__ A, int kp, double* __restrict__ M) {
  const int64_t t = (int64_t)blockIdx.x * kPcThreads + threadIdx.x;
  if (t >= (int64_t)kp * kp) return;
  const int a = (int)(t / kp), b = (int)(t % kp);
  const bool lower_tile = (a >> 6) >= (b >> 6);
  M[t] = lower_tile ? A[t] : A[(int64_t)b * kp + a];
}

// Z[i][c] = (R[i][c] - sum_t L[t][i] S[t][c]) / sigma^2 with L the FP32 factor
// copy.  One workgroup: 64 rows i x 16*NBT columns (plus column c0 + 16*NBT on
// the vector ALU with X1, as in kpc_tn); tiles of 32 factor columns t are staged
// in LDS as FP64 (A lane: L[t + 4s + l/16][i0 + 16w + l%16]; B lane:
// S[t + 4s + l/16][c0 + 16u + l%16]; D lane q: (i0 + 16w + 4q + l/16,
// c0 + 16u + l%16)).
template <int NBT, bool X1 = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void kpc_apply(const float* __restrict__ L, int64_t ldl, int k,
                                                 int64_t n, const double* __restrict__ S, int nb,
                                                 const float* __restrict__ R, int64_t ldr,
                                                 float* __restrict__ Z, int64_t ldz, double s2) {
  constexpr int NB = 16 * NBT;            // columns on the matrix cores
  constexpr int NBX = NB + (X1 ? 1 : 0);  // columns of the S tile
  __shared__ double As[kTI][64 + 1];
  __shared__ double Bs[kTI][NBX + 1];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int la = lane & 15, lk = lane >> 4;
  const int64_t i0 = (int64_t)blockIdx.x * 64;
  const int c0 = blockIdx.y * NB;
  f64x4 acc[NBT];
#pragma unroll
  for (int u = 0; u < NBT; ++u) acc[u] = f64x4{0.0, 0.0, 0.0, 0.0};
  double xacc = 0.0;  // X1: the extra column c0 + NB on the vector ALU
  // loaders: 8 threads per 64-value row segment of the factor (8 values each);
  // the kTI x NBX tile of S as consecutive entries, BPT per thread (entry
  // f = 256 e + tid: row f / NBX, column f % NBX); the next stage is fetched
  // into registers while the MFMAs of the current one run.
  const int lr = tid >> 3, lc = (tid & 7) * 8;
  constexpr int BT = kTI * NBX;
  constexpr int BPT = (BT + 255) / 256;
  float ra[8];
  double rb[BPT];
  auto fetch = [&](int t0) {
    load_seg(L, k, ldl, t0 + lr, i0 + lc, n, ra);
#pragma unroll
    for (int e = 0; e < BPT; ++e) {
      const int f = 256 * e + tid;
      const int t = t0 + f / NBX;
      const int col = c0 + f % NBX;
      rb[e] = (f < BT && t < k && col < nb) ? S[(int64_t)t * nb + col] : 0.0;
    }
  };
  if (k > 0) fetch(0);
  for (int t0 = 0; t0 < k; t0 += kTI) {
#pragma unroll
    for (int e = 0; e < 8; ++e) As[lr][lc + e] = (double)ra[e];
#pragma unroll
    for (int e = 0; e < BPT; ++e) {
      const int f = 256 * e + tid;
      if (f < BT) Bs[f / NBX][f % NBX] = rb[e];
    }
    __syncthreads();
    if (t0 + kTI < k) fetch(t0 + kTI);
#pragma unroll
    for (int s4 = 0; s4 < kTI / 4; ++s4) {
      const double av = As[4 * s4 + lk][16 * wave + la];
#pragma unroll
      for (int u = 0; u < NBT; ++u)
        acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Bs[4 * s4 + lk][16 * u + la], acc[u], 0,
                                                      0, 0);
      if constexpr (X1) xacc = fma(av, Bs[4 * s4 + lk][NB], xacc);
    }
    __syncthreads();
  }
  const double inv = 1.0 / s2;
#pragma unroll
  for (int u = 0; u < NBT; ++u)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t i = i0 + 16 * wave + 4 * q + lk;
      const int c = c0 + 16 * u + la;
      if (i < n && c < nb) Z[i * ldz + c] = (float)(((double)R[i * ldr + c] - acc[u][q]) * inv);
    }
  if constexpr (X1) {
    // the four lane groups hold the sums over t = 4s + 0..3: add them pairwise
    xacc += __shfl_xor(xacc, 16);
    xacc += __shfl_xor(xacc, 32);
    const int64_t i = i0 + 16 * wave + la;
    const int c = c0 + NB;
    if (lk == 0 && i < n && c < nb) Z[i * ldz + c] = (float)(((double)R[i * ldr + c] - xacc) * inv);
  }
}

// FP32 copy of the factor (rows >= n of each factor column set to zero).
__global__ void kpc_to_f32(const double* __restrict__ L, int64_t ldl, int k, int64_t n,
                           float* __restrict__ L32) {
  const int64_t e = (int64_t)blockIdx.x * kPcThreads + threadIdx.x;
  if (e >= (int64_t)k * ldl) return;
  const int64_t i = e % ldl;
  L32[e] = i < n ? (float)L[e] : 0.f;
}

int blocks_of(int64_t count) { return (int)((count + kPcThreads - 1) / kPcThreads); }

}  // namespace

int pc_parts(int64_t n) { return blocks_of((n + kPcRows - 1) / kPcRows); }

hipError_t pc_init(double* diag, int64_t n, double a2, PcState* s, int32_t* piv, hipStream_t st) {
  hipLaunchKernelGGL(kpc_init, dim3(blocks_of(n > 0 ? n : 1)), dim3(kPcThreads), 0, st, diag, n,
                     a2, s, piv);
  return hipGetLastError();
}

hipError_t pc_step(const float* X, int64_t n, int d, const double* ell, double a2, double* L,
                   float* L32, int64_t ldl, int j, int k, double* diag, PcState* s, double* lp,
                   double* pval, int64_t* pidx, int32_t* piv, hipStream_t st) {
  if (L32 && ldl % kPcRows) return hipErrorInvalidValue;
  const int nparts = pc_parts(n);
  if (L32) {
    hipLaunchKernelGGL(kpc_column<true>, dim3(nparts), dim3(kPcThreads), 0, st, X, n, d, ell, a2,
                       L, L32, ldl, j, diag, s, lp, pval, pidx);
    hipLaunchKernelGGL(kpc_pivot<true>, dim3(1), dim3(kPcThreads), 0, st, pval, pidx, nparts, L,
                       L32, ldl, j, k, s, lp, piv);
  } else {
    hipLaunchKernelGGL(kpc_column<false>, dim3(nparts), dim3(kPcThreads), 0, st, X, n, d, ell,
                       a2, L, L32, ldl, j, diag, s, lp, pval, pidx);
    hipLaunchKernelGGL(kpc_pivot<false>, dim3(1), dim3(kPcThreads), 0, st, pval, pidx, nparts, L,
                       L32, ldl, j, k, s, lp, piv);
  }
  return hipGetLastError();
}

// Row-chunk length so that the split products launch about `target` workgroups.
static int64_t chunk_rows(int64_t n, int64_t tiles, int64_t target) {
  int64_t nz = target / (tiles > 0 ? tiles : 1);
  if (nz < 1) nz = 1;
  int64_t cs = (n + nz - 1) / nz;
  cs = (cs + 15) / 16 * 16;
  return cs < 64 ? 64 : cs;
}

hipError_t pc_to_f32(const double* L, int64_t ldl, int k, int64_t n, float* L32,
                     hipStream_t st) {
  if (k <= 0) return hipSuccess;
  hipLaunchKernelGGL(kpc_to_f32, dim3(blocks_of((int64_t)k * ldl)), dim3(kPcThreads), 0, st, L,
                     ldl, k, n, L32);
  return hipGetLastError();
}

hipError_t pc_gram(const float* L, int64_t ldl, int k, int64_t n, double* part,
                   int64_t part_cap, double* G, hipStream_t st) {
  const int64_t xt = (k + 63) / 64, yt = (k + 63) / 64;
  int64_t cs = chunk_rows(n, xt * yt, 2048);
  int64_t nz = (n + cs - 1) / cs;
  while (nz * k * k > part_cap) {
    cs *= 2;
    nz = (n + cs - 1) / cs;
  }
  if (k > 0 && n > 0)
    hipLaunchKernelGGL((kpc_tn<4, 1, float>), dim3(xt, yt, nz), dim3(256), 0, st, L, ldl, k, n,
                       (const float*)nullptr, (int64_t)0, k, cs, part);
  hipLaunchKernelGGL(kpc_sum, dim3(blocks_of((int64_t)k * k)), dim3(kPcThreads), 0, st, part,
                     (int)((k > 0 && n > 0) ? nz : 0), k, k, G, k, 0, 0.0, 0);
  return hipGetLastError();
}

hipError_t pc_shift(const double* G, int k, double* A, int kp, double s2, hipStream_t st) {
  hipLaunchKernelGGL(kpc_sum, dim3(blocks_of((int64_t)kp * kp)), dim3(kPcThreads), 0, st, G, 1, k,
                     k, A, kp, kp, s2, 1);
  return hipGetLastError();
}

int64_t pc_gram_parts(int64_t n, int k) {
  const int64_t xt = (k + 63) / 64;
  const int64_t cs = chunk_rows(n, xt * xt, 2048);
  return ((n + cs - 1) / cs) * (int64_t)k * k;
}

hipError_t pc_mirror(const double* A, int kp, double* M, hipStream_t st) {
  if (kp <= 0 || kp % 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(kpc_mirror, dim3(blocks_of((int64_t)kp * kp)), dim3(kPcThreads), 0, st, A, kp,
                     M);
  return hipGetLastError();
}

// Chunk count for the skinny products of the apply.  Every workgroup does the
// same work, so among nz0 .. 2 nz0 chunks (nz0 = max(1, 2048 / tiles)) the
// count whose workgroups fill the last round of the CUs' concurrent slots
// (CUs x workgroups per CU) best is taken; ties go to the smaller count.
static int64_t apply_nz0(int64_t tiles) {
  const int64_t nz0 = 2048 / (tiles > 0 ? tiles : 1);
  return nz0 < 1 ? 1 : nz0;
}

static int64_t balanced_nz(int64_t tiles, int per_cu) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    cus = 256;
  const int64_t slots = (int64_t)cus * per_cu, nz0 = apply_nz0(tiles);
  int64_t best = nz0;
  double best_fill = 0.0;
  for (int64_t nz = nz0; nz <= 2 * nz0; ++nz) {
    const int64_t wg = tiles * nz;
    const double fill = (double)wg / (double)(((wg + slots - 1) / slots) * slots);
    if (fill > best_fill) {
      best_fill = fill;
      best = nz;
    }
  }
  return best;
}

// Rows per chunk for nz chunks of n rows (a multiple of 16, at least 64).
static int64_t rows_per_chunk(int64_t n, int64_t nz) {
  int64_t cs = (n + nz - 1) / nz;
  cs = (cs + 15) / 16 * 16;
  return cs < 64 ? 64 : cs;
}

// 65 columns (64 probe vectors and the mean column): 64 on the matrix cores and
// one on the vector ALU in the same pass over the factor, instead of 80 padded
// matrix-core columns.
constexpr int kApplyX1Cols = 65;

int64_t pc_apply_parts(int64_t n, int k, int c) {
  // the chunk count grows with the requested count, which is at most 2 nz0
  const int64_t tiles = (k + 63) / 64 * ((c + 79) / 80), nzmax = 2 * apply_nz0(tiles);
  const int64_t cs = rows_per_chunk(n, nzmax), cs2 = rows_per_chunk(k, nzmax);
  const int64_t nz1 = (n + cs - 1) / cs, nz2 = (k + cs2 - 1) / cs2;
  return (nz1 > nz2 ? nz1 : nz2) * (int64_t)k * c;
}

hipError_t pc_apply(const float* L, int64_t ldl, int k, int64_t n, const double* M, int kp,
                    const float* R, int64_t ldr, int c, double* part, double* T, double* S,
                    float* Z, int64_t ldz, double s2, hipStream_t st) {
  if (k > 0 && n > 0) {
    // workgroups per CU: 4 for the FP32-factor product (LDS and its register
    // target), 3 for the all-FP64 one (registers)
    const int64_t xt = (k + 63) / 64, yt = (c + 79) / 80;
    const int64_t cs = rows_per_chunk(n, balanced_nz(xt * yt, 4));
    const int64_t nz = (n + cs - 1) / cs;
    if (c == kApplyX1Cols)
      hipLaunchKernelGGL((kpc_tn<4, 0, float, float, 4, true>), dim3(xt, 1, nz), dim3(256), 0, st, L,
                         ldl, k, n, R, ldr, c, cs, part);
    else
      hipLaunchKernelGGL((kpc_tn<5, 0, float>), dim3(xt, yt, nz), dim3(256), 0, st, L, ldl, k, n, R,
                         ldr, c, cs, part);
    hipLaunchKernelGGL(kpc_sum, dim3(blocks_of((int64_t)k * c)), dim3(kPcThreads), 0, st, part,
                       (int)nz, k, c, T, c, 0, 0.0, 0);
    // S = M T (k x c, reduction over the k factor columns) on the same tiled product
    const int64_t cs2 = rows_per_chunk(k, balanced_nz(xt * yt, 3));
    const int64_t nz2 = (k + cs2 - 1) / cs2;
    hipLaunchKernelGGL((kpc_tn<5, 0, double, double, 3>), dim3(xt, yt, nz2), dim3(256), 0, st, M,
                       (int64_t)kp, k, (int64_t)k, T, (int64_t)c, c, cs2, part);
    hipLaunchKernelGGL(kpc_sum, dim3(blocks_of((int64_t)k * c)), dim3(kPcThreads), 0, st, part,
                       (int)nz2, k, c, S, c, 0, 0.0, 0);
  }
  if (n > 0 && c == kApplyX1Cols)
    hipLaunchKernelGGL((kpc_apply<4, true>), dim3((n + 63) / 64, 1), dim3(256), 0, st, L, ldl, k, n,
                       S, c, R, ldr, Z, ldz, s2);
  else if (n > 0)
    hipLaunchKernelGGL((kpc_apply<5>), dim3((n + 63) / 64, (c + 79) / 80), dim3(256), 0, st, L,
                       ldl, k, n, S, c, R, ldr, Z, ldz, s2);
  return hipGetLastError();
}

}  // namespace gpk
