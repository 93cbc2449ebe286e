// Internal interface between the HIP kernels (fwd.hip, adj.hip, vec.hip) and
// the host runtime (runtime.hip).  Not part of the public C ABI (include/gp.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace gpk {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Inputs are pre-scaled by sqrt(3) log2(e) / ell_k, so that with
// rho = |x^_i - x^_j| the Matern-3/2 value is m = (1 + ln2 rho) 2^-rho
// (exp(-sqrt3 r) = 2^-rho, 1 + sqrt3 r = 1 + ln2 rho).
constexpr double kSqrt3Log2e = 1.7320508075688772935 * 1.4426950408889634074;
constexpr float kLn2 = 0.693147180559945309f;

// Every packed row array is padded with zero rows to a multiple of this, so
// that kernels need no bounds checks on the j (column) stream and every
// workgroup's rows are addressable.
constexpr int kRowAlign = 256;
constexpr int kJStep = 32;          // forward kernel: kernel columns per MFMA K-chunk
constexpr int kAdjRowsPerWG = 128;
constexpr int kAdjMaxCols = 256;  // columns of one fused-adjoint pass (8 K-tiles of 32)
// Row sub-tiles of 16 rows per wave in the forward kernel (4 waves per
// workgroup): 4 for up to 5 column tiles (80 columns), 2 for wider products.
constexpr int fwd_row_subtiles(int CT) { return CT <= 5 ? 4 : 2; }
// Cross-term path: K chunks of 4 (d coordinates + the squared norm) and row
// sub-tiles per wave (fewer when many chunk operands occupy registers).
constexpr int xt_chunks(int d) { return (d + 1 + 3) / 4; }
constexpr int fwd_xt_row_subtiles(int CT, int NK) { return (CT <= 5 && NK <= 3) ? 4 : 2; }
inline int fwd_rows_per_wg(int CT) { return 64 * fwd_row_subtiles(CT); }
constexpr int kMaxD = 64;
constexpr int kMaxC = 1024;      // columns of a product, adjoint or random-feature sample
constexpr int kMaxSolveC = 256;  // columns of a solve: the column reductions run one
                                 // thread per column in a 256-thread block

enum Prec { P_FP32 = 0, P_BF16X3 = 1, P_BF16 = 2 };
enum Fn { FN_MATERN = 0, FN_DLEN = 1 };

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Compile-time dimensions the kernels are instantiated for; inputs with
// d < D are zero-padded (zero coordinates add nothing to distances).
int select_D(int d);
inline int dp_of(int D) { return (D + 3) & ~3; }
// 16-column tiles of the forward product (c <= 16 * CT); 0 if c > 128.
int select_CT(int c);
// 32-column K-tiles of the adjoint tile product (c <= 32 * KT).
int select_KT(int c);

struct DimScale {
  float s[kMaxD];
};

// ---------------------------------------------------------------- packing (vec.hip)
hipError_t pack_x(const float* X, int64_t n, int d, int DP, const DimScale& sc, float* Xp,
                  int64_t n_pad, hipStream_t st);
hipError_t pack_x_rows(const float* X, const int32_t* idx, int64_t nidx, int d, int DP,
                       const DimScale& sc, float* Xp, int64_t n_pad, hipStream_t st);
// d <= 3: rows [x^_0, x^_1, x^_2, |x^|^2].  Cross-term layout with nk chunks
// (nk >= xt_chunks(d)).  stats[0]: max |x^|^2 (float bits, atomic max);
// stats[1], stats[2]: number of points with |x^|^2 > kXTMaxNorm2 and
// > kXTMaxNorm2F32 (atomic counts).
hipError_t pack_x_aug(const float* X, const int32_t* idx, int64_t n, int d, const DimScale& sc,
                      int nk, float* Xp, int64_t n_pad, unsigned* stats, hipStream_t st);
// When the cross-term path is used.  Its FP32 cancellation error in r^2 is about
// 6e-8 (|x^_i|^2 + |x^_j|^2) and matters only for pairs close enough to carry
// weight, so the product error follows the bulk of the norms, not the outliers
// (points far from the origin are far from most others): with |x^|^2 <= 1024 for
// all but one point in kXTOutlierShare and <= kXTHardNorm2 for every point, an
// FP32 emulation on the workloads' inputs gives column errors near 1e-5 (the
// bf16x3 budget is 2e-5).  FP32 products (budget 1e-5) use the bounds 640 and
// 2048 (column error 3.4e-6 on the d = 3 precision workload, max |x^|^2 595).
constexpr float kXTMaxNorm2 = 1024.f;     // bf16 modes: bulk bound
constexpr float kXTHardNorm2 = 4096.f;    // bf16 modes: every point
constexpr int64_t kXTOutlierShare = 1024;
constexpr float kXTMaxNorm2F32 = 640.f;   // FP32 mode (tighter budget): bulk bound
constexpr float kXTHardNorm2F32 = 2048.f; // FP32 mode: every point
// V [n, ldv] (first c columns, optional per-column scale) into forward tiles;
// perm = the row order of the cross-term path (see fwd.hip).
hipError_t pack_v_bf16(const float* V, int64_t n, int64_t ldv, int c, const float* colscale,
                       int CT, uint16_t* hi, uint16_t* lo, int64_t n_pad, bool perm,
                       hipStream_t st);
hipError_t pack_v_f32(const float* V, int64_t n, int64_t ldv, int c, const float* colscale,
                      int CT, float* out, int64_t n_pad, bool perm, hipStream_t st);
// Order-independent 64-bit fingerprint of x[0..count) added to *out (caller zeroes it).
hipError_t checksum_f32(const float* x, int64_t count, unsigned long long* out, hipStream_t st);
// Row-major [n_pad, 32*KT] packs for the adjoint (optional per-column weights).
hipError_t pack_rows_bf16(const float* U, int64_t n, int64_t ldu, int c, const float* colw,
                          int KT, uint16_t* hi, uint16_t* lo, int64_t n_pad, hipStream_t st);
hipError_t pack_rows_f32(const float* U, int64_t n, int64_t ldu, int c, const float* colw,
                         int KT, float* out, int64_t n_pad, hipStream_t st);

// ---------------------------------------------------------------- forward product (fwd.hip)
struct FwdArgs {
  int prec = P_FP32;
  int fn = FN_MATERN;
  int fn_dim = 0;
  int D = 1;                       // template dimension (>= d), X packs have dp_of(D) columns
  const float* xp1 = nullptr;      // [n1_pad, DP] row points
  const float* xp2 = nullptr;      // [n2_pad, DP] column points
  int64_t n1 = 0, n1_pad = 0;
  int64_t steps = 0;               // n2_pad / 32
  const void* vhi = nullptr;       // forward tiles: bf16 hi (or fp32)
  const void* vlo = nullptr;       // bf16 lo (BF16X3 only)
  int CT = 1;
  int c = 0;
  float* out = nullptr;            // [n1, ldo]
  int64_t ldo = 0;
  float* part = nullptr;           // [S, n1_pad, 16*CT] when S > 1
  int S = 1;
  float scale = 1.f;               // out = scale * (M V) + noise * vn
  const float* vn = nullptr;       // [n1, ldv] or null
  int64_t ldv = 0;
  float noise = 0.f;
  int xt = 0;                      // cross-term path (bf16 modes)
  const float* xt1 = nullptr;      // [xt_chunks(d)][n1_pad][4] row points (cross-term layout)
  const float* xt2 = nullptr;      // [xt_chunks(d)][n2_pad][4] column points
  int64_t n2_pad = 0;              // rows of xt2 per chunk
};
hipError_t fwd(const FwdArgs& a, hipStream_t st);
// Sum of the S partial products plus the epilogue (used when S > 1).
hipError_t fwd_reduce(const float* part, int S, int64_t n1, int64_t n1_pad, int CP, int c,
                      float scale, const float* vn, int64_t ldv, float noise, float* out,
                      int64_t ldo, hipStream_t st);
// Number of j-splits for a forward launch with `rowblocks` workgroup rows.
int choose_splits(int64_t rowblocks, int64_t steps);

// ---------------------------------------------------------------- fused adjoint (adj.hip)
struct AdjArgs {
  int prec = P_BF16X3;  // tile product U diag(w) W^T: P_FP32 or P_BF16X3
  int D = 1;
  const float* xp = nullptr;       // [n_pad, DP]
  int64_t n_pad = 0;
  const void* uhi = nullptr;       // [n_pad, 32 KT] (bf16 hi or fp32)
  const void* ulo = nullptr;
  const void* whi = nullptr;
  const void* wlo = nullptr;
  int KT = 1;
  int S = 1;                       // j-splits
  double* partial = nullptr;       // [rowblocks * S, D + 1]
};
// Writes per-workgroup FP64 sums: for k < D, sum_ij G_ij 2^-rho_ij dhat_ijk^2;
// slot D: sum_ij G_ij m_ij.  Returns the number of partial rows in *rows.
hipError_t adj(const AdjArgs& a, int64_t* rows, hipStream_t st);

// ---------------------------------------------------------------- vector kernels (vec.hip)
// Column sums of squares / dot products into FP64 partials [nb, ld].
int reduce_blocks(int64_t n);
hipError_t col_dot_partial(const float* A, const float* B, int64_t n, int64_t lda, int64_t ldb,
                           int c, double* partial, int nb, hipStream_t st);
hipError_t col_reduce(const double* partial, int nb, int c, double* out, hipStream_t st);
// ||B_c|| -> scale_c = 1 / (||B_c|| + eps) (double and float copies).
hipError_t norm_to_scale(const double* sumsq, int c, double eps, double* scale_d, float* scale_f,
                         hipStream_t st);
// dst[i, col] = src[i, col] * scale[col] for col < c, 0 for c <= col < ld_dst.
hipError_t scale_cols(const float* src, int64_t lds, int64_t n, int c, const float* scale,
                      float* dst, int64_t ldd, int cpad, hipStream_t st);
// dst[i, col] = src[i, col] * mul[col] (col < c) into a user array.
hipError_t unscale_cols(const float* src, int64_t lds, int64_t n, int c, const double* scale_d,
                        float* dst, int64_t ldd, hipStream_t st);
// R = Bt - HU; D = R; partial sums of R^2.
hipError_t residual_init(const float* Bt, const float* HU, float* R, float* Dv, int64_t n,
                         int64_t ld, int c, double* partial, int nb, bool set_d, hipStream_t st);
// CG scalars: alpha = gamma / sum(partial) with freeze / breakdown detection.
hipError_t cg_alpha(const double* partial, int nb, int c, const double* gamma, double* alpha,
                    int* status, hipStream_t st);
// U += alpha D; R -= alpha HD; partial sums of R^2.
hipError_t cg_update_ur(float* U, float* R, const float* Dv, const float* HD,
                        const double* alpha, int64_t n, int64_t ld, int c, double* partial,
                        int nb, hipStream_t st);
// gamma' = sum(partial); beta = gamma'/gamma (0 for frozen); gamma = gamma'; rnorm = sqrt.
hipError_t cg_beta(const double* partial, int nb, int c, double* gamma, double* beta,
                   double* rnorm, int* status, hipStream_t st);
// gamma = sum(partial); rnorm = sqrt(gamma).
hipError_t gamma_from_partial(const double* partial, int nb, int c, double* gamma,
                              double* rnorm, int* status, hipStream_t st);
// D = R + beta D.
hipError_t cg_update_d(float* Dv, const float* R, const double* beta, int64_t n, int64_t ld,
                       int c, hipStream_t st);
// sum_c w_c sum_i U_ic W_ic in FP64 partials -> used for the sigma derivative.
hipError_t weighted_dot_partial(const float* U, int64_t ldu, const float* W, int64_t ldw,
                                int64_t n, int c, double* partial, int nb, hipStream_t st);

// ---------------------------------------------------------------- random features (vec.hip)
struct RffArgs {
  int D = 1;
  const float* x = nullptr;        // [m, d] user layout
  int d = 1;
  int64_t m = 0;
  const double* omega = nullptr;   // [M, d] device, t / ell in FP64
  int M = 0;
  const float* W = nullptr;        // [2M, ldw]
  int64_t ldw = 0;
  int s = 0;
  float amp = 1.f;                 // a / sqrt(M)
  float* F = nullptr;              // [m, ldf] output, column offset f_col0
  int64_t ldf = 0;
  int f_col0 = 0;
  const float* weps = nullptr;     // optional: F += sigma * weps[:, j]
  int64_t ldeps = 0;
  float sigma = 0.f;
};
hipError_t rff(const RffArgs& a, hipStream_t st);
hipError_t rff_omega(const float* t, int M, int d, const double* inv_ell_dev, double* omega,
                     hipStream_t st);
// B[:, 0] = y (first column of an [n, ld] buffer).
hipError_t set_col(const float* y, int64_t n, float* B, int64_t ld, int col, hipStream_t st);

// ---------------------------------------------------------------- SGD / AP helpers (vec.hip)
hipError_t gather_rows(const float* A, int64_t lda, const int32_t* idx, int64_t nidx, int c,
                       float* out, int64_t ldo, hipStream_t st);
// G = HI - Bt[idx] (in place in HI); Mom = rho Mom; Mom[idx] -= lr/b G; U += Mom;
// R[idx] = G (residual estimate).
// SGD iteration halves (App. B, Algorithm 3): the batch rows' momentum, residual
// estimate and running column sums of squares (rnorm = their square roots), and
// the dense momentum decay, U update and packing of U for the next product.
hipError_t sgd_sparse(const float* G, int64_t ldg, const int32_t* idx, int b, float* Mom,
                      float* R, int64_t ld, int c, float rho, float lrb, int32_t* stamp, int t,
                      double* sumsq, double* rnorm, int* status, hipStream_t st);
hipError_t sgd_update_pack(float* U, float* Mom, int64_t ld, const int32_t* stamp, int t,
                           float rho, int64_t n, int c, int CT, bool perm, int64_t n_pad,
                           uint16_t* hi, uint16_t* lo, float* f32, hipStream_t st);
hipError_t fill_i32(int32_t* dst, int64_t count, int32_t v, hipStream_t st);
hipError_t sgd_momentum(float* Mom, const float* G, const int32_t* idx, int64_t b, int64_t n,
                        int64_t ld, int c, float rho, float lrb, hipStream_t st);
hipError_t sgd_finish(float* U, float* R, const float* Mom, const float* G, const int32_t* idx,
                      int64_t b, int64_t n, int64_t ld, int c, hipStream_t st);
hipError_t sub_rows(float* G, int64_t ldg, const float* Bt, int64_t ldb, const int32_t* idx,
                    int64_t b, int c, hipStream_t st);
hipError_t add_rows_scaled(float* dst, int64_t ldd, const int32_t* idx, const float* src,
                           int64_t lds, int64_t b, int c, float alpha, hipStream_t st);
hipError_t axpy_cols(float* Y, const float* X, int64_t n, int64_t ld, int c, float alpha,
                     hipStream_t st);
hipError_t copy_cols(const float* src, int64_t lds, int64_t n, int c, float* dst, int64_t ldd,
                     hipStream_t st);
hipError_t fill(float* dst, int64_t count, float v, hipStream_t st);
// D[i][j] = U[i][0] - U[i][1 + j], j < s (D row-major [n, s]).
hipError_t post_diff(const float* U, int64_t ldu, int64_t n, int s, float* D, hipStream_t st);
hipError_t check_finite(const float* A, int64_t n, int64_t ld, int c, int* status,
                        hipStream_t st);

// ---------------------------------------------------------------- AP / SGD (solve.hip)
constexpr int kMaxAPBlock = 2048;  // padded AP block size limit (multiple of 64)
constexpr int kMaxSolveCP = 256;  // columns of the AP residual update (kMaxSolveC)

// ---------------------------------------------------------------- preconditioner
// Pivoted-Cholesky construction state (device memory): current pivot, its
// remaining diagonal, the rank reached and a stop flag (rank deficiency).
struct PcState {
  int64_t p;
  int stop;
  int rank;
  double dp;
};
constexpr int kMaxPrecondRank = 32768;  // rank limit
int pc_parts(int64_t n);
hipError_t pc_init(double* diag, int64_t n, double a2, PcState* s, int32_t* piv, hipStream_t st);
// One pivoted-Cholesky step j of k (column j for the current pivot, then the next
// pivot); the factor is FP32 in L32 when L32 is non-null, else FP64 in L.
hipError_t pc_step(const float* X, int64_t n, int d, const double* ell, double a2, double* L,
                   float* L32, int64_t ldl, int j, int k, double* diag, PcState* s, double* lp,
                   double* pval, int64_t* pidx, int32_t* piv, hipStream_t st);
// FP32 copy of the factor, used by the products below.
hipError_t pc_to_f32(const double* L, int64_t ldl, int k, int64_t n, float* L32, hipStream_t st);
// G (k x k) = L^T L; A (kp x kp) = sigma^2 I + G on the leading k x k block,
// identity elsewhere.
hipError_t pc_gram(const float* L, int64_t ldl, int k, int64_t n, double* part,
                   int64_t part_cap, double* G, hipStream_t st);
hipError_t pc_shift(const double* G, int k, double* A, int kp, double s2, hipStream_t st);
int64_t pc_gram_parts(int64_t n, int k);
// M (kp x kp, full) from the lower 64 x 64 tiles of the symmetric A (kp a
// multiple of 64): M = A^-1 after spd_inverse.
hipError_t pc_mirror(const double* A, int kp, double* M, hipStream_t st);
int64_t pc_apply_parts(int64_t n, int k, int c);
// Z = (R - L M L^T R) / sigma^2 for c columns (T, S: k x c scratch).
hipError_t pc_apply(const float* L, int64_t ldl, int k, int64_t n, const double* M, int kp,
                    const float* R, int64_t ldr, int c, double* part, double* T, double* S,
                    float* Z, int64_t ldz, double s2, hipStream_t st);
// FP64 H[I, I] for every contiguous block of b rows, lower triangle, padded to P x P.
hipError_t ap_build_blocks(const float* xp, int DP, int d, int64_t n, int b, int P, double a2,
                           double s2, double* M, hipStream_t st);
// In-place lower Cholesky of nblk P x P blocks; status bit 2 on a non-positive pivot.
hipError_t ap_cholesky(double* M, int nblk, int P, int* status, hipStream_t st);
// In place: every block's lower Cholesky factor L becomes L^-1 (lower triangle).
hipError_t ap_invert_factors(double* M, int nblk, int P, hipStream_t st);
// out[i, :c] = H[I_blk, I_blk]^-1 R[I_blk, :c] = X^T (X R[I_blk]) with X = L^-1
// from ap_invert_factors (P a multiple of 64); y: P x c FP64 scratch.
hipError_t ap_solve_block(const double* M, int P, int blk, int b, int64_t n, const float* R,
                          int64_t ldr, int c, double* y, float* out, int64_t ldo, hipStream_t st);
// Per block k of b rows, split into ap_subblocks(b) equal parts w = k nsub + sub:
// R[I_k] -= G[I_k] (when G is given; on the rows sel_base .. sel_base + sel_bk
// also R -= s2 delta), then scores[w] = the part's sum over its rows i of
// (sum_c R[i, c])^2 (a block's score is the sum over its parts, in order) and
// part[w * c + col] = the part's sum of R^2.  c <= kMaxSolveCP.
inline int ap_subblocks(int b) { return (b + 255) / 256; }
hipError_t ap_update(float* R, int64_t ld, const float* G, int64_t ldg, int64_t n, int b, int c,
                     int64_t sel_base, int sel_bk, const float* delta, int64_t ldd, float s2,
                     double* scores, double* part, hipStream_t st);
// Y[base + i, :] += alpha X[i, :] for i < bk
hipError_t add_block(float* Y, int64_t ldy, int64_t base, int bk, const float* X, int64_t ldx,
                     int c, float alpha, hipStream_t st);
// G[i, :] += s2 Ut[idx[i], :] - Bt[idx[i], :]
hipError_t sgd_fix(float* G, int64_t ldg, const float* Ut, const float* Bt, int64_t ld,
                   const int32_t* idx, int64_t b, int c, float s2, hipStream_t st);

// ---------------------------------------------- initial-hyperparameter heuristic
// nearest.hip: the k rows of X nearest to row `centre` (squared Euclidean
// distance in FP64, dimension order, no fused multiply-add; ties to the lower
// row), written to idx in ascending row order.  key [n], cnt [2 nearest_blocks(n)]
// and st are scratch.
struct SelState {
  uint64_t prefix;
  uint64_t mask;
  int64_t want;
  unsigned hist[256];
};
int64_t nearest_blocks(int64_t n);
hipError_t nearest(const float* X, int64_t n, int d, int64_t centre, int64_t k, uint64_t* key,
                   SelState* st, int64_t* cnt, int64_t* idx, hipStream_t s);

// exact.hip: dense FP64 exact marginal likelihood on m gathered rows, padded to
// m_p (a multiple of kExactTile).  A, W: m_p x m_p scratch; xs [m_p, d], ys, diag,
// v, alpha [m_p]; part [exact_part_doubles]; gpart [exact_gpart_doubles];
// out [d + 4] = (y^T alpha, log det H, gradient (ell_1..ell_d, a, sigma)).
// status bit 1: an index outside [0, n); bit 2: a non-positive pivot.
constexpr int kExactTile = 64;
constexpr int kExactChunk = 256;
constexpr int64_t kExactMaxM = 32768;
enum ExFlags { kExLowerC = 1, kExALower = 2, kExAUpper = 4, kExBLower = 8, kExBUpper = 16 };
hipError_t exact_gather(const float* X, int64_t n, int d, const int64_t* idx, int64_t m,
                        int64_t mp, const float* y, double* xs, double* ys, int* status,
                        hipStream_t st);
// exact_factor: H (lower tiles), the recursive Cholesky with inverse factor W, and
// H^-1 = W^T W into A, on stream st; with a side stream (may be null) and
// exact_events(m_p) events, part of each split runs concurrently on it, joined
// back into st before return.  exact_finish: alpha = W^T W y, the scalars and
// the gradient.
hipError_t exact_factor(const double* xs, int d, int64_t m, int64_t mp, const double* inv_ell,
                        double a, double sigma, double* A, double* W, double* diag, int* status,
                        hipStream_t st, hipStream_t side, hipEvent_t* ev, int nev);
inline int exact_events(int64_t mp) { return 2 * (int)(mp / kExactTile); }
hipError_t exact_finish(const double* xs, const double* ys, int d, int64_t m, int64_t mp,
                        const double* inv_ell, double a, double sigma, const double* Hinv,
                        const double* W, const double* diag, double* v, double* alpha,
                        double* part, double* gpart, double* out, hipStream_t st);
int64_t exact_part_doubles(int64_t mp);
// In place inverse of an SPD matrix A (mp x mp row-major, mp a multiple of
// kExactTile, only the lower 64 x 64 tiles read) by the same recursive Cholesky
// with inverse factor: A^-1 = W^T W is left in the lower tiles of A, W = C^-1 in
// W, diag[i] = C_ii; status bit 2 on a non-positive pivot.
hipError_t spd_inverse(double* A, double* W, int64_t mp, double* diag, int* status,
                       hipStream_t st);
int64_t exact_gpart_doubles(int64_t mp, int d);

}  // namespace gpk
