// Host runtime behind the C ABI (include/gp.h): context, workspace, the
// kernel-product operator, the linear solvers of App. B (Algorithms 1-3),
// the gradient estimators of Secs. 2-3 and the outer-loop Adam update.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <random>
#include <string>
#include <vector>

#include "gp.h"
#include "gpk.h"

using namespace gpk;

namespace {

enum BufId {
  B_XP1, B_XP2, B_VHI, B_VLO, B_PART, B_BT, B_UT, B_R, B_DV, B_HD, B_AUX, B_MOM, B_SCALD,
  B_SCALF, B_PARTIAL, B_STATUS, B_UHI, B_ULO, B_WHI, B_WLO, B_ADJP, B_OMEGA, B_INVELL, B_RHS,
  B_WB, B_IDX, B_GX, B_G, B_APF, B_XTMAX, B_Z, B_PCL, B_PCDIAG, B_PCST, B_PCLP, B_PCPV,
  B_PCPI, B_PCPIV, B_PCPART, B_PCA, B_PCM, B_PCT, B_PCS, B_PCELL, B_PCSTAT, B_PCL32, B_PCW, B_POSTD, B_XT1, B_XT2,
  B_EXA, B_EXW, B_EXXS, B_EXYS, B_EXDG, B_EXV, B_EXAL, B_EXPART, B_EXGP, B_EXOUT, B_EXIE, B_EXST,
  B_NRKEY, B_NRST, B_NRCNT, B_NRIDX, B_PCG, B_PCSUM, B_STAMP, B_APY, B_PCID, B_COUNT
};

constexpr double kNormEps = 1e-10;
constexpr int64_t kSafetyCap = 100000;
constexpr int kProfClasses = 9;

struct Packed {
  float* xp = nullptr;  // [n_pad, DP] scaled points
  float* xt = nullptr;  // cross-term layout [xt_chunks(d)][n_pad][4] (== xp for d <= 3)
  int64_t n = 0, n_pad = 0;
  int D = 0, DP = 0;
  bool xt_ok = false;  // norms small enough for the cross-term path (bf16 modes)
  bool xt_ok32 = false;  // ... and for the FP32 mode
};

}  // namespace

struct gp_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t gstream = nullptr;  // library-owned stream for captured solver iterations
  hipEvent_t gev[2] = {nullptr, nullptr};
  hipStream_t xstream = nullptr;  // library-owned side stream of the exact factorisation
  // the last pivoted-Cholesky factor (B_PCL32) and its Gram matrix (B_PCG), for reuse
  struct {
    const float* X = nullptr;
    unsigned long long sum = 0;  // fingerprint of X's contents
    int64_t n = 0;
    int d = 0, k_req = 0, k = 0, uses = 0;
    bool valid = false;
  } pcc;
  std::vector<hipEvent_t> xev;    // its dependency events
  uint64_t alloc_epoch = 0;       // bumped on every workspace (re)allocation
  std::string err;
  void* buf[B_COUNT] = {};
  size_t cap[B_COUNT] = {};
  double* hpin = nullptr;  // pinned host scratch
  size_t hpin_cap = 0;
  // Allocation-free calls (gp_kmatvec_static): while `arena.on`, workspace
  // buffers are carved from the device's static scratch array and host staging
  // uses `arena_host`; nothing is allocated.
  struct {
    bool on = false;
    unsigned char* base = nullptr;
    size_t cap = 0, used = 0;
    unsigned char* ptr[B_COUNT] = {};
    size_t size[B_COUNT] = {};
  } arena;
  double arena_host[64] = {};
  bool prof = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[kProfClasses];
  std::vector<hipEvent_t> pool;
  double prof_ms[kProfClasses] = {};
  int64_t prof_n[kProfClasses] = {};
};

// Scratch of the allocation-free product (gp_kmatvec_static): a file-scope device
// array, one copy per device, held until the process ends.  Host code reaches it
// only through the address hipGetSymbolAddress returns for the current device.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

// Address of this device's scratch, looked up once per device with it current.
int scratch_address(int device, unsigned char** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return GP_ERR_HIP;
    }
    g_scratch_ptr[device] = static_cast<unsigned char*>(p);
  }
  *out = g_scratch_ptr[device];
  return GP_OK;
}

int fail(gp_ctx* c, int code, const char* fmt, ...) {
  char b[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(b, sizeof b, fmt, ap);
  va_end(ap);
  if (c) c->err = b;
  return code;
}

#define HIPCHK(expr)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(ctx, GP_ERR_HIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                  __FILE__, __LINE__);                                                   \
  } while (0)

#define CHK(expr)                 \
  do {                            \
    int r_ = (expr);              \
    if (r_ != GP_OK) return r_;   \
  } while (0)

template <typename T>
int ensure(gp_ctx* ctx, BufId id, size_t count, T** out) {
  size_t bytes = std::max<size_t>(count * sizeof(T), 256);
  if (ctx->arena.on) {
    auto& a = ctx->arena;
    if (a.size[id] < bytes) {
      const size_t off = (a.used + 255) & ~(size_t)255;
      if (off > a.cap || bytes > a.cap - off)
        return fail(ctx, GP_ERR_INVALID_ARG,
                    "the call needs more than the %zu bytes of static scratch of the "
                    "allocation-free entry point", a.cap);
      a.ptr[id] = a.base + off;
      a.size[id] = bytes;
      a.used = off + bytes;
    }
    *out = reinterpret_cast<T*>(a.ptr[id]);
    return GP_OK;
  }
  if (ctx->cap[id] < bytes) {
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (ctx->buf[id]) HIPCHK(hipFree(ctx->buf[id]));
    ctx->buf[id] = nullptr;
    ctx->cap[id] = 0;
    size_t want = bytes + bytes / 8;
    ++ctx->alloc_epoch;
    if (hipMalloc(&ctx->buf[id], want) != hipSuccess) {
      (void)hipGetLastError();
      ctx->buf[id] = nullptr;
      return fail(ctx, GP_ERR_NO_WORKSPACE, "hipMalloc of %zu bytes for workspace %d failed",
                  want, (int)id);
    }
    ctx->cap[id] = want;
  }
  *out = reinterpret_cast<T*>(ctx->buf[id]);
  return GP_OK;
}

int ensure_pinned(gp_ctx* ctx, size_t doubles) {
  if (ctx->hpin_cap >= doubles) return GP_OK;
  if (ctx->arena.on)
    return fail(ctx, GP_ERR_INVALID_ARG, "host staging of %zu values exceeds the %zu of the "
                "allocation-free entry point", doubles, ctx->hpin_cap);
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (ctx->hpin) HIPCHK(hipHostFree(ctx->hpin));
  ctx->hpin = nullptr;
  ctx->hpin_cap = 0;
  size_t want = std::max<size_t>(doubles, 4096);
  HIPCHK(hipHostMalloc((void**)&ctx->hpin, want * sizeof(double), hipHostMallocDefault));
  ctx->hpin_cap = want;
  return GP_OK;
}

// ------------------------------------------------------------------ profiling
hipEvent_t take_event(gp_ctx* ctx) {
  if (!ctx->pool.empty()) {
    hipEvent_t e = ctx->pool.back();
    ctx->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

struct ProfScope {
  gp_ctx* ctx;
  int cls;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(gp_ctx* c, int k) : ctx(c), cls(k) {
    if (!ctx->prof) return;
    a = take_event(ctx);
    b = take_event(ctx);
    if (a) (void)hipEventRecord(a, ctx->stream);
  }
  ~ProfScope() {
    if (!ctx->prof || !a || !b) return;
    (void)hipEventRecord(b, ctx->stream);
    ctx->ev[cls].push_back({a, b});
  }
};

int harvest(gp_ctx* ctx) {
  for (int k = 0; k < kProfClasses; ++k) {
    for (auto& p : ctx->ev[k]) {
      float ms = 0.f;
      HIPCHK(hipEventSynchronize(p.second));
      HIPCHK(hipEventElapsedTime(&ms, p.first, p.second));
      ctx->prof_ms[k] += ms;
      ctx->prof_n[k] += 1;
      ctx->pool.push_back(p.first);
      ctx->pool.push_back(p.second);
    }
    ctx->ev[k].clear();
  }
  return GP_OK;
}

// ------------------------------------------------------------------ validation
int check_theta(gp_ctx* ctx, const double* theta, int d) {
  if (!theta) return fail(ctx, GP_ERR_INVALID_ARG, "theta is NULL");
  for (int k = 0; k < d + 2; ++k)
    if (!(theta[k] > 0.0) || !std::isfinite(theta[k]))
      return fail(ctx, GP_ERR_INVALID_ARG, "theta[%d] = %g must be finite and > 0", k, theta[k]);
  return GP_OK;
}

int check_dims(gp_ctx* ctx, int d, int c, int cmax = kMaxC) {
  if (d < 1 || d > kMaxD) return fail(ctx, GP_ERR_INVALID_ARG, "d = %d outside [1, %d]", d, kMaxD);
  if (c < 0 || c > cmax) return fail(ctx, GP_ERR_INVALID_ARG, "c = %d outside [0, %d]", c, cmax);
  return GP_OK;
}

int check_mat(gp_ctx* ctx, const char* name, const void* p, int64_t rows, int64_t ld, int cols) {
  if (rows < 0) return fail(ctx, GP_ERR_INVALID_ARG, "%s: negative row count", name);
  if (rows > 0 && cols > 0 && !p) return fail(ctx, GP_ERR_INVALID_ARG, "%s is NULL", name);
  if (ld < cols) return fail(ctx, GP_ERR_INVALID_ARG, "%s: ld %lld < %d columns", name,
                             (long long)ld, cols);
  return GP_OK;
}

int check_precond(gp_ctx* ctx, const gp_solver_cfg& cfg) {
  if (cfg.precond_rank < 0 || cfg.precond_rank > kMaxPrecondRank)
    return fail(ctx, GP_ERR_INVALID_ARG, "precond_rank %d outside [0, %d]", cfg.precond_rank,
                kMaxPrecondRank);
  if (cfg.precond_rank > 0 && cfg.solver != GP_CG)
    return fail(ctx, GP_ERR_INVALID_ARG, "the pivoted-Cholesky preconditioner is for CG only");
  if (cfg.use_graph && cfg.solver != GP_CG)
    return fail(ctx, GP_ERR_INVALID_ARG, "graph-captured iterations are for CG only");
  if (cfg.precond_reuse < 0)
    return fail(ctx, GP_ERR_INVALID_ARG, "precond_reuse %d must be >= 0", cfg.precond_reuse);
  return GP_OK;
}

int check_prec(gp_ctx* ctx, int prec) {
  if (prec != GP_FP32 && prec != GP_BF16X3 && prec != GP_BF16)
    return fail(ctx, GP_ERR_INVALID_ARG, "unknown precision %d", prec);
  return GP_OK;
}

// ------------------------------------------------------------------ operator
// With a parent (the packed full set that X's selected rows belong to), the
// rows inherit its choice of distance form: the rows of a product over a subset
// are rows of the full product, with the same accuracy, and no norm statistics
// are read back (no host synchronisation).
int pack_points(gp_ctx* ctx, BufId id, const float* X, const int32_t* idx, int64_t n, int d,
                const double* theta, Packed* p, const Packed* parent = nullptr) {
  p->n = n;
  p->n_pad = round_up(std::max<int64_t>(n, 1), kRowAlign);
  p->D = select_D(d);
  p->DP = dp_of(p->D);
  DimScale sc{};
  for (int k = 0; k < d; ++k) sc.s[k] = (float)(kSqrt3Log2e / theta[k]);
  CHK(ensure(ctx, id, (size_t)(p->n_pad * p->DP), &p->xp));
  p->xt_ok = false;
  if (p->D > 3) {
    if (idx)
      HIPCHK(pack_x_rows(X, idx, n, d, p->DP, sc, p->xp, p->n_pad, ctx->stream));
    else
      HIPCHK(pack_x(X, n, d, p->DP, sc, p->xp, p->n_pad, ctx->stream));
    CHK(ensure(ctx, id == B_XP1 ? B_XT1 : B_XT2, (size_t)(p->n_pad * 4 * xt_chunks(p->D)),
               &p->xt));
  } else {
    p->xt = p->xp;  // the cross-term layout is the packed layout (DP = 4, norm in slot 3)
  }
  if (parent) {
    HIPCHK(pack_x_aug(X, idx, n, d, sc, xt_chunks(p->D), p->xt, p->n_pad, nullptr, ctx->stream));
    p->xt_ok = parent->xt_ok;
    p->xt_ok32 = parent->xt_ok32;
    return GP_OK;
  }
  // squared norms ride in the last slot of the cross-term layout; their maximum and
  // the count above the bulk bound decide whether the cross-term distance form is
  // accurate enough for these points
  unsigned* mx;
  CHK(ensure(ctx, B_XTMAX, 3, &mx));
  CHK(ensure_pinned(ctx, 2));
  HIPCHK(hipMemsetAsync(mx, 0, 3 * sizeof(unsigned), ctx->stream));
  // chunks for the kernel's dimension tier D (>= d), so kernel and layout agree
  HIPCHK(pack_x_aug(X, idx, n, d, sc, xt_chunks(p->D), p->xt, p->n_pad, mx, ctx->stream));
  HIPCHK(hipMemcpyAsync(ctx->hpin, mx, 3 * sizeof(unsigned), hipMemcpyDeviceToHost,
                        ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  unsigned st[3];
  std::memcpy(st, ctx->hpin, sizeof st);
  float m;
  std::memcpy(&m, &st[0], sizeof(float));
  p->xt_ok = std::isfinite(m) && m <= kXTHardNorm2 && (int64_t)st[1] * kXTOutlierShare <= n;
  p->xt_ok32 = std::isfinite(m) && m <= kXTHardNorm2F32 && (int64_t)st[2] * kXTOutlierShare <= n;
  return GP_OK;
}

// out[:, :cols] = scale * M(P1, P2) V (+ noise * vn); V has p2.n rows.
// With v_packed, the forward tiles of V (one pass of at most 80 columns, in the
// order kprod_v_perm gives) are already in the B_VHI / B_VLO workspace.
bool kprod_v_perm(const Packed& p1, const Packed& p2, int prec) {
  return prec == GP_FP32 ? (p1.xt_ok32 && p2.xt_ok32) : (p1.xt_ok && p2.xt_ok);
}

int kprod(gp_ctx* ctx, const Packed& p1, const Packed& p2, const float* V, int64_t ldv, int cols,
          float* out, int64_t ldo, int prec, float scale, const float* vn, int64_t ldvn,
          float noise, int fn = FN_MATERN, int fn_dim = 0, bool v_packed = false) {
  // Columns go in balanced passes of at most 80 (5 column tiles with 4 row
  // sub-tiles per wave): wider single passes (8 tiles, 2 sub-tiles) measured
  // slower than two such passes, although each pass re-evaluates the kernel.
  const int npass = (cols + 79) / 80;
  if (v_packed && (npass != 1 || fn != FN_MATERN))
    return fail(ctx, GP_ERR_INVALID_ARG, "pre-packed V needs one pass of the kernel product");
  const int per = (cols + npass - 1) / npass;
  for (int c0 = 0; c0 < cols; c0 += per) {
    const int cs = std::min(per, cols - c0);
    const int CT = select_CT(cs);
    FwdArgs a;
    a.prec = prec;
    a.fn = fn;
    a.fn_dim = fn_dim;
    a.D = p1.D;
    a.xp1 = p1.xp;
    a.xp2 = p2.xp;
    a.n1 = p1.n;
    a.n1_pad = p1.n_pad;
    a.steps = p2.n_pad / kJStep;
    a.CT = CT;
    a.c = cs;
    a.out = out + c0;
    a.ldo = ldo;
    a.scale = scale;
    a.vn = vn ? vn + c0 : nullptr;
    a.ldv = ldvn;
    a.noise = noise;
    a.xt = fn == FN_MATERN && kprod_v_perm(p1, p2, prec);
    a.xt1 = p1.xt;
    a.xt2 = p2.xt;
    a.n2_pad = p2.n_pad;
    const size_t vcount = (size_t)(p2.n_pad * 16 * CT);
    if (prec == GP_FP32) {
      float* vf;
      CHK(ensure(ctx, B_VHI, vcount, &vf));
      if (!v_packed)
        HIPCHK(pack_v_f32(V + c0, p2.n, ldv, cs, nullptr, CT, vf, p2.n_pad, a.xt != 0,
                          ctx->stream));
      a.vhi = vf;
    } else {
      uint16_t *hi, *lo = nullptr;
      CHK(ensure(ctx, B_VHI, vcount, &hi));
      if (prec == GP_BF16X3) CHK(ensure(ctx, B_VLO, vcount, &lo));
      if (!v_packed)
        HIPCHK(pack_v_bf16(V + c0, p2.n, ldv, cs, nullptr, CT, hi, lo, p2.n_pad, a.xt != 0,
                           ctx->stream));
      a.vhi = hi;
      a.vlo = lo;
    }
    const int64_t rowblocks =
        p1.n_pad / (64 * (a.xt ? fwd_xt_row_subtiles(CT, xt_chunks(p1.D)) : fwd_row_subtiles(CT)));
    a.S = choose_splits(rowblocks, a.steps);
    if (ctx->arena.on) {
      // allocation-free calls: as many column splits as the scratch left holds
      const size_t used = (ctx->arena.used + 255) & ~(size_t)255;
      const size_t left = ctx->arena.size[B_PART] > 0
                              ? ctx->arena.size[B_PART]
                              : (used < ctx->arena.cap ? ctx->arena.cap - used : 0);
      while (a.S > 1 && (size_t)(a.S * p1.n_pad * 16 * CT) * sizeof(float) > left) a.S /= 2;
    }
    if (a.S > 1) CHK(ensure(ctx, B_PART, (size_t)(a.S * p1.n_pad * 16 * CT), &a.part));
    {
      // the profile class times the forward kernel launch alone
      ProfScope ps(ctx, prec == GP_FP32 ? 4 : 0);
      HIPCHK(fwd(a, ctx->stream));
    }
    if (a.S > 1)
      HIPCHK(fwd_reduce(a.part, a.S, p1.n, p1.n_pad, 16 * CT, cs, scale, a.vn, ldvn, noise,
                        out + c0, ldo, ctx->stream));
  }
  return GP_OK;
}

float a2_of(const double* theta, int d) { return (float)(theta[d] * theta[d]); }
float s2_of(const double* theta, int d) { return (float)(theta[d + 1] * theta[d + 1]); }

// Column sums of A*B (or A*A) into host doubles out[c].
int col_sums(gp_ctx* ctx, const float* A, const float* B, int64_t n, int64_t lda, int64_t ldb,
             int c, double* out) {
  if (n == 0 || c == 0) {
    for (int k = 0; k < c; ++k) out[k] = 0.0;
    return GP_OK;
  }
  const int nb = reduce_blocks(n);
  double *partial, *res;
  CHK(ensure(ctx, B_PARTIAL, (size_t)nb * std::min(c, kMaxSolveC), &partial));
  CHK(ensure(ctx, B_SCALD, (size_t)6 * kMaxC, &res));
  // the column reductions take at most kMaxSolveC columns per launch
  for (int c0 = 0; c0 < c; c0 += kMaxSolveC) {
    const int cs = std::min(kMaxSolveC, c - c0);
    HIPCHK(col_dot_partial(A + c0, B ? B + c0 : nullptr, n, lda, ldb, cs, partial, nb,
                           ctx->stream));
    HIPCHK(col_reduce(partial, nb, cs, res + 5 * kMaxC + c0, ctx->stream));
  }
  CHK(ensure_pinned(ctx, kMaxC));
  HIPCHK(hipMemcpyAsync(ctx->hpin, res + 5 * kMaxC, c * sizeof(double), hipMemcpyDeviceToHost,
                        ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  std::memcpy(out, ctx->hpin, c * sizeof(double));
  return GP_OK;
}

// ------------------------------------------------------------------ solvers
struct SolveState {
  int64_t n;
  int c;
  float *Bt, *Ut, *R, *Dv, *HD, *Z = nullptr;
  double *scale_d, *gamma, *alpha, *beta, *rnorm;
  float* scale_f;
  int* status;
  int nb;
  double* partial;
};

int read_norms(gp_ctx* ctx, SolveState& s, double* ry, double* rz, int* status) {
  CHK(ensure_pinned(ctx, kMaxC + 2));
  HIPCHK(hipMemcpyAsync(ctx->hpin, s.rnorm, s.c * sizeof(double), hipMemcpyDeviceToHost,
                        ctx->stream));
  HIPCHK(hipMemcpyAsync(ctx->hpin + kMaxC, s.status, sizeof(int), hipMemcpyDeviceToHost,
                        ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  *ry = ctx->hpin[0];
  double z = 0.0;
  for (int k = 1; k < s.c; ++k) z += ctx->hpin[k];
  *rz = s.c > 1 ? z / (s.c - 1) : 0.0;
  int st;
  std::memcpy(&st, ctx->hpin + kMaxC, sizeof(int));
  *status = st;
  return GP_OK;
}

int status_to_error(gp_ctx* ctx, int st) {
  if (st & 1) return fail(ctx, GP_ERR_NONFINITE, "solver residual became non-finite");
  if (st & 2) return fail(ctx, GP_ERR_BREAKDOWN, "CG breakdown: d^T H d <= 0 on a live column");
  return GP_OK;
}

bool keep_going(double ry, double rz, double tol) { return ry > tol || rz > tol; }

// Opt-in progress lines on stderr for long solves: GPMI_PROGRESS=<seconds>.
struct Progress {
  double every = 0.0;
  std::chrono::steady_clock::time_point start, last;
  Progress() {
    const char* e = std::getenv("GPMI_PROGRESS");
    if (e) every = std::atof(e);
    start = last = std::chrono::steady_clock::now();
  }
  void tick(const char* what, int64_t it, double ry, double rz) {
    if (every <= 0.0) return;
    const auto now = std::chrono::steady_clock::now();
    if (std::chrono::duration<double>(now - last).count() < every) return;
    last = now;
    std::fprintf(stderr, "[gpmi] %s iter %lld  relres_y %.3e  relres_z %.3e  (%.1f s)\n", what,
                 (long long)it, ry, rz, std::chrono::duration<double>(now - start).count());
    std::fflush(stderr);
  }
  void count(const char* what, int64_t done, int64_t total) {
    if (every <= 0.0) return;
    const auto now = std::chrono::steady_clock::now();
    if (std::chrono::duration<double>(now - last).count() < every && done < total) return;
    last = now;
    std::fprintf(stderr, "[gpmi] %s %lld/%lld  (%.1f s)\n", what, (long long)done,
                 (long long)total, std::chrono::duration<double>(now - start).count());
    std::fflush(stderr);
  }
};

// Allocate solver vectors and normalise: Bt = B / (||B|| + eps), Ut = U0 / (||B|| + eps).
int solve_setup(gp_ctx* ctx, const float* B, int64_t ldb, const float* U, int64_t ldu,
                int64_t n, int c, SolveState& s) {
  s.n = n;
  s.c = c;
  const size_t vec = (size_t)std::max<int64_t>(n, 1) * c;
  CHK(ensure(ctx, B_BT, vec, &s.Bt));
  CHK(ensure(ctx, B_UT, vec, &s.Ut));
  CHK(ensure(ctx, B_R, vec, &s.R));
  CHK(ensure(ctx, B_DV, vec, &s.Dv));
  CHK(ensure(ctx, B_HD, vec, &s.HD));
  double* sc;
  CHK(ensure(ctx, B_SCALD, (size_t)6 * kMaxC, &sc));
  s.scale_d = sc;
  s.gamma = sc + kMaxC;
  s.alpha = sc + 2 * kMaxC;
  s.beta = sc + 3 * kMaxC;
  s.rnorm = sc + 4 * kMaxC;
  CHK(ensure(ctx, B_SCALF, (size_t)kMaxC, &s.scale_f));
  CHK(ensure(ctx, B_STATUS, 16, &s.status));
  s.nb = reduce_blocks(n);
  CHK(ensure(ctx, B_PARTIAL, (size_t)s.nb * c, &s.partial));
  HIPCHK(hipMemsetAsync(s.status, 0, sizeof(int), ctx->stream));
  HIPCHK(col_dot_partial(B, nullptr, n, ldb, ldb, c, s.partial, s.nb, ctx->stream));
  HIPCHK(col_reduce(s.partial, s.nb, c, s.gamma, ctx->stream));
  HIPCHK(norm_to_scale(s.gamma, c, kNormEps, s.scale_d, s.scale_f, ctx->stream));
  HIPCHK(scale_cols(B, ldb, n, c, s.scale_f, s.Bt, c, c, ctx->stream));
  HIPCHK(scale_cols(U, ldu, n, c, s.scale_f, s.Ut, c, c, ctx->stream));
  return GP_OK;
}

// ------------------------------------------------------------ preconditioner
// Rank-k pivoted-Cholesky preconditioner of CG (App. B): P = L L^T + sigma^2 I,
// applied as P^-1 through the Woodbury identity with M = (sigma^2 I + L^T L)^-1.
struct Precond {
  int k = 0;         // rank reached (0: P = sigma^2 I is not used, see `active`)
  int kp = 0;        // k rounded up to 32 (Cholesky / inverse tile)
  int64_t ldl = 0;   // leading dimension of the transposed factor L[t * ldl + i]
  int64_t n = 0;
  float* L32 = nullptr;  // FP32 factor (defines P; the products read it)
  double* M = nullptr;
  double s2 = 0.0;
  bool active = false;
};

// Greedy construction into L [k, ldl] (FP64) or, when L32 is given, L32 [k, ldl]
// (FP32); piv [k]; returns the rank reached.
int pc_construct(gp_ctx* ctx, const float* X, int64_t n, int d, const double* theta, int k,
                 double* L, float* L32, int64_t ldl, int32_t* piv, int* rank) {
  *rank = 0;
  if (k <= 0 || n <= 0) return GP_OK;
  double *diag, *lp, *pval, *ell;
  int64_t* pidx;
  PcState* st;
  CHK(ensure(ctx, B_PCDIAG, (size_t)n, &diag));
  CHK(ensure(ctx, B_PCLP, (size_t)k, &lp));
  CHK(ensure(ctx, B_PCPV, (size_t)pc_parts(n), &pval));
  CHK(ensure(ctx, B_PCPI, (size_t)pc_parts(n), &pidx));
  CHK(ensure(ctx, B_PCST, 1, &st));
  CHK(ensure(ctx, B_PCELL, (size_t)d, &ell));
  CHK(ensure_pinned(ctx, (size_t)std::max(d, 2)));
  std::memcpy(ctx->hpin, theta, (size_t)d * sizeof(double));
  HIPCHK(hipMemcpyAsync(ell, ctx->hpin, (size_t)d * sizeof(double), hipMemcpyHostToDevice,
                        ctx->stream));
  const double a2 = theta[d] * theta[d];
  HIPCHK(pc_init(diag, n, a2, st, piv, ctx->stream));
  for (int j = 0; j < k; ++j)
    HIPCHK(pc_step(X, n, d, ell, a2, L, L32, ldl, j, k, diag, st, lp, pval, pidx, piv,
                   ctx->stream));
  PcState hs;
  HIPCHK(hipMemcpyAsync(ctx->hpin, st, sizeof(PcState), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  std::memcpy(&hs, ctx->hpin, sizeof hs);
  *rank = hs.rank;
  return GP_OK;
}

// P for this solve.  The factor and its Gram matrix G = L^T L are kept in the
// context; with reuse > 0 a factor built for the same X (pointer and contents
// fingerprint), n, d and rank serves up to `reuse` later solves, and only
// sigma^2 I + G is factored again.
int pc_build(gp_ctx* ctx, const float* X, int64_t n, int d, const double* theta, int k_req,
             int reuse, Precond& pc) {
  pc = Precond{};
  pc.n = n;
  pc.s2 = theta[d + 1] * theta[d + 1];
  pc.active = true;
  const int k = (int)std::min<int64_t>(k_req, n);
  if (k <= 0) return GP_OK;
  pc.ldl = round_up(n, 64);
  auto& cc = ctx->pcc;
  unsigned long long sum = 0;
  {
    unsigned long long* dsum;
    CHK(ensure(ctx, B_PCSUM, 1, &dsum));
    CHK(ensure_pinned(ctx, 1));
    HIPCHK(hipMemsetAsync(dsum, 0, sizeof(unsigned long long), ctx->stream));
    HIPCHK(checksum_f32(X, n * d, dsum, ctx->stream));
    HIPCHK(hipMemcpyAsync(ctx->hpin, dsum, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                          ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    std::memcpy(&sum, ctx->hpin, sizeof sum);
  }
  const bool again = reuse > 0 && cc.valid && cc.X == X && cc.sum == sum && cc.n == n &&
                     cc.d == d && cc.k_req == k && cc.uses < reuse;
  double *part, *G;
  if (again) {
    CHK(ensure(ctx, B_PCL32, (size_t)k * pc.ldl, &pc.L32));  // present: no reallocation
    pc.k = cc.k;
    ++cc.uses;
  } else {
    cc.valid = false;
    int32_t* piv;
    CHK(ensure(ctx, B_PCL32, (size_t)k * pc.ldl, &pc.L32));
    CHK(ensure(ctx, B_PCPIV, (size_t)k, &piv));
    CHK(pc_construct(ctx, X, n, d, theta, k, nullptr, pc.L32, pc.ldl, piv, &pc.k));
    if (pc.k == 0) return GP_OK;
    const int64_t pcap = pc_gram_parts(n, pc.k);
    CHK(ensure(ctx, B_PCPART, (size_t)pcap, &part));
    CHK(ensure(ctx, B_PCG, (size_t)pc.k * pc.k, &G));
    HIPCHK(pc_gram(pc.L32, pc.ldl, pc.k, n, part, pcap, G, ctx->stream));
    cc.X = X;
    cc.sum = sum;
    cc.n = n;
    cc.d = d;
    cc.k_req = k;
    cc.k = pc.k;
    cc.uses = 0;
    cc.valid = true;
  }
  if (pc.k == 0) return GP_OK;
  // M = (sigma^2 I + L^T L)^-1 for this step's sigma: the recursive Cholesky with
  // inverse factor on the matrix cores (k^3 flops), padded with the identity to a
  // multiple of 64
  pc.kp = (int)round_up(pc.k, 64);
  double *A, *W, *dg;
  int* stat;
  CHK(ensure(ctx, B_PCG, (size_t)pc.k * pc.k, &G));
  CHK(ensure(ctx, B_PCA, (size_t)pc.kp * pc.kp, &A));
  CHK(ensure(ctx, B_PCW, (size_t)pc.kp * pc.kp, &W));
  CHK(ensure(ctx, B_PCM, (size_t)pc.kp * pc.kp, &pc.M));
  CHK(ensure(ctx, B_PCID, (size_t)pc.kp, &dg));
  CHK(ensure(ctx, B_PCSTAT, 1, &stat));
  HIPCHK(hipMemsetAsync(stat, 0, sizeof(int), ctx->stream));
  HIPCHK(pc_shift(G, pc.k, A, pc.kp, pc.s2, ctx->stream));
  HIPCHK(spd_inverse(A, W, pc.kp, dg, stat, ctx->stream));
  HIPCHK(pc_mirror(A, pc.kp, pc.M, ctx->stream));
  int hst = 0;
  HIPCHK(hipMemcpyAsync(ctx->hpin, stat, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  std::memcpy(&hst, ctx->hpin, sizeof(int));
  if (hst) return fail(ctx, GP_ERR_BREAKDOWN, "preconditioner: sigma^2 I + L^T L not positive definite");
  return GP_OK;
}

// Z = P^-1 R for the c columns of R (ld ldr).
int pc_apply_cols(gp_ctx* ctx, const Precond& pc, const float* R, int64_t ldr, int c, float* Z,
                  int64_t ldz) {
  double *part = nullptr, *T = nullptr, *S = nullptr;
  if (pc.k > 0) {
    CHK(ensure(ctx, B_PCPART, (size_t)std::max(pc_apply_parts(pc.n, pc.k, c),
                                               pc_gram_parts(pc.n, pc.k)), &part));
    CHK(ensure(ctx, B_PCT, (size_t)pc.k * c, &T));
    CHK(ensure(ctx, B_PCS, (size_t)pc.k * c, &S));
  }
  ProfScope ps(ctx, 5);
  HIPCHK(pc_apply(pc.L32, pc.ldl, pc.k, pc.n, pc.M, pc.kp, R, ldr, c, part, T, S, Z, ldz, pc.s2,
                  ctx->stream));
  return GP_OK;
}

// R = Bt - H Ut with the given precision; optionally D = R (or P^-1 R);
// gamma = R.R (or R.P^-1 R); rnorm = ||R||.
int true_residual(gp_ctx* ctx, const Packed& px, const double* theta, int d, SolveState& s,
                  int prec, bool set_d, const Precond* pc = nullptr) {
  CHK(kprod(ctx, px, px, s.Ut, s.c, s.c, s.HD, s.c, prec, a2_of(theta, d), s.Ut, s.c,
            s2_of(theta, d)));
  const bool use_pc = pc && pc->active;
  HIPCHK(residual_init(s.Bt, s.HD, s.R, s.Dv, s.n, s.c, s.c, s.partial, s.nb, set_d && !use_pc,
                       ctx->stream));
  HIPCHK(gamma_from_partial(s.partial, s.nb, s.c, use_pc ? nullptr : s.gamma, s.rnorm, s.status,
                            ctx->stream));
  if (use_pc) {
    CHK(pc_apply_cols(ctx, *pc, s.R, s.c, s.c, s.Z, s.c));
    HIPCHK(col_dot_partial(s.R, s.Z, s.n, s.c, s.c, s.c, s.partial, s.nb, ctx->stream));
    HIPCHK(col_reduce(s.partial, s.nb, s.c, s.gamma, ctx->stream));
    if (set_d) HIPCHK(copy_cols(s.Z, s.c, s.n, s.c, s.Dv, s.c, ctx->stream));
  }
  return GP_OK;
}

int solve_finish(gp_ctx* ctx, SolveState& s, float* U, int64_t ldu) {
  HIPCHK(unscale_cols(s.Ut, s.c, s.n, s.c, s.scale_d, U, ldu, ctx->stream));
  return GP_OK;
}

// Runs the solve on the library's own (capturable) stream, ordered after and
// before the caller's stream with events; restores the caller's stream on exit.
struct OwnStream {
  gp_ctx* ctx;
  hipStream_t user = nullptr;
  bool on = false;
  int enter(gp_ctx* c) {
    ctx = c;
    user = c->stream;
    if (!c->gstream) {
      HIPCHK(hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking));
      for (auto& e : c->gev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    HIPCHK(hipEventRecord(c->gev[0], user));
    HIPCHK(hipStreamWaitEvent(c->gstream, c->gev[0], 0));
    c->stream = c->gstream;
    on = true;
    return GP_OK;
  }
  ~OwnStream() {
    if (!on) return;
    (void)hipEventRecord(ctx->gev[1], ctx->gstream);
    (void)hipStreamWaitEvent(user, ctx->gev[1], 0);
    ctx->stream = user;
  }
};

int true_residual_stats(gp_ctx* ctx, const Packed& px, const double* theta, int d, SolveState& s,
                        gp_solve_stats& stats);

int cg_solve(gp_ctx* ctx, const Packed& px, const float* X, const double* theta, int d,
             SolveState& s, const gp_solver_cfg& cfg, gp_solve_stats& stats) {
  // the products' precision: the requested one, FP32 after an escalation
  int prec = cfg.precision;
  bool escalated = false;
  OwnStream own;
  if (cfg.use_graph) CHK(own.enter(ctx));
  Precond pcs;
  const Precond* pc = nullptr;
  if (cfg.precond_rank > 0) {
    {
      ProfScope ps(ctx, 5);
      CHK(pc_build(ctx, X, s.n, d, theta, cfg.precond_rank, cfg.precond_reuse, pcs));
    }
    CHK(ensure(ctx, B_Z, (size_t)s.n * s.c, &s.Z));
    pc = &pcs;
    stats.precond_rank = pcs.k;
  }
  const bool mixed = prec != GP_FP32;
  const int64_t cap = cfg.max_epochs > 0 ? (int64_t)std::ceil(cfg.max_epochs - 1e-9) : kSafetyCap;
  const int check = cfg.check_every > 0 ? cfg.check_every : 1;
  const float a2 = a2_of(theta, d), s2 = s2_of(theta, d);

  // Initial residual r = b~ - H u~ (FP32: it is the true residual).
  CHK(true_residual(ctx, px, theta, d, s, GP_FP32, true, pc));
  stats.matvecs += 1;
  int64_t t = 0, since_true = 0;
  double ry = 0, rz = 0;
  double last_true = std::numeric_limits<double>::infinity();
  // the recurrence's target: tol, lowered from the second failed acceptance on
  double tol_in = cfg.tol;
  int failed = 0;
  int st = 0;
  Progress prog;
  auto cg_iteration = [&]() -> int {
    CHK(kprod(ctx, px, px, s.Dv, s.c, s.c, s.HD, s.c, prec, a2, s.Dv, s.c, s2));
    {
      ProfScope ps(ctx, 3);
      HIPCHK(col_dot_partial(s.Dv, s.HD, s.n, s.c, s.c, s.c, s.partial, s.nb, ctx->stream));
      HIPCHK(cg_alpha(s.partial, s.nb, s.c, s.gamma, s.alpha, s.status, ctx->stream));
      HIPCHK(cg_update_ur(s.Ut, s.R, s.Dv, s.HD, s.alpha, s.n, s.c, s.c, s.partial, s.nb,
                          ctx->stream));
      if (!pc) {
        HIPCHK(cg_beta(s.partial, s.nb, s.c, s.gamma, s.beta, s.rnorm, s.status, ctx->stream));
        HIPCHK(cg_update_d(s.Dv, s.R, s.beta, s.n, s.c, s.c, ctx->stream));
      }
    }
    if (pc) {
      // p = P(r); beta = r.p / gamma; gamma = r.p; d = p + beta d
      HIPCHK(gamma_from_partial(s.partial, s.nb, s.c, nullptr, s.rnorm, s.status, ctx->stream));
      CHK(pc_apply_cols(ctx, *pc, s.R, s.c, s.c, s.Z, s.c));
      ProfScope ps(ctx, 3);
      HIPCHK(col_dot_partial(s.R, s.Z, s.n, s.c, s.c, s.c, s.partial, s.nb, ctx->stream));
      HIPCHK(cg_beta(s.partial, s.nb, s.c, s.gamma, s.beta, nullptr, s.status, ctx->stream));
      HIPCHK(cg_update_d(s.Dv, s.Z, s.beta, s.n, s.c, s.c, ctx->stream));
    }
    return GP_OK;
  };
  const bool use_graph = cfg.use_graph != 0;
  hipGraphExec_t graph_exec = nullptr;
  uint64_t graph_epoch = 0;
  struct ExecGuard {
    hipGraphExec_t* e;
    ~ExecGuard() {
      if (*e) (void)hipGraphExecDestroy(*e);
    }
  } exec_guard{&graph_exec};
  while (true) {
    if (since_true == 0 || t % check == 0 || t >= cap) {
      CHK(read_norms(ctx, s, &ry, &rz, &st));
      CHK(status_to_error(ctx, st));
      prog.tick("cg", t, ry, rz);
      // a true residual (since_true == 0) is tested against tol itself
      bool go = keep_going(ry, rz, since_true == 0 ? cfg.tol : tol_in);
      if (since_true == 0 && t == 0) last_true = std::max(ry, rz);
      if (!go && mixed && since_true > 0) {
        // The reduced-precision recurrence says converged: accept only on the
        // FP32 true residual.  If it is not yet below tol, restart CG from the
        // true residual (D = R): mixed-precision iterative refinement with CG
        // as the inner solver.  The first restart keeps the target; from the
        // second on, the target is halved at every restart (the recurrence
        // drifts from the true residual again after a restart, and a target just
        // under tol leaves the restart too little to do), and a restart with a
        // lowered target that gains less than 10 % on the true residual means
        // the attainable accuracy of the reduced-precision operator is reached.
        CHK(true_residual(ctx, px, theta, d, s, GP_FP32, true, pc));
        stats.matvecs += 1;
        stats.refinements += 1;
        since_true = 0;
        CHK(read_norms(ctx, s, &ry, &rz, &st));
        CHK(status_to_error(ctx, st));
        go = keep_going(ry, rz, cfg.tol);
        if (go) {
          const double now = std::max(ry, rz);
          ++failed;
          if (failed >= 3 && now > 0.9 * last_true) {
            if (!escalated && prec != GP_FP32) {
              // The reduced-precision operator's attainable accuracy lies above tol:
              // continue from this true residual (D = R or P^-1 R, just set) with
              // FP32 products, whose recurrence the true residual then follows.
              escalated = true;
              prec = GP_FP32;
              failed = 0;
              tol_in = cfg.tol;
              last_true = now;
              if (graph_exec) {
                HIPCHK(hipGraphExecDestroy(graph_exec));
                graph_exec = nullptr;
              }
            } else {
              stats.true_relres_y = ry;
              stats.true_relres_z = rz;
              stats.converged = 0;
              break;
            }
          } else {
            last_true = now;
            if (failed >= 2) tol_in *= 0.5;
          }
        }
      }
      if (since_true == 0) {
        stats.true_relres_y = ry;
        stats.true_relres_z = rz;
      } else {
        stats.true_relres_y = stats.true_relres_z = std::numeric_limits<double>::quiet_NaN();
      }
      if (!go || t >= cap) {
        stats.converged = !go;
        // a solve that the budget stopped reports the FP32 true residual of the
        // iterate it returns (early stopping, Sec. 5), as AP and SGD do
        if (go && since_true > 0) CHK(true_residual_stats(ctx, px, theta, d, s, stats));
        break;
      }
    }
    // One CG iteration (Algorithm 1), columns in parallel.
    if (graph_exec && ctx->alloc_epoch != graph_epoch) {
      // a workspace moved since the capture: the graph's pointers are stale
      HIPCHK(hipGraphExecDestroy(graph_exec));
      graph_exec = nullptr;
    }
    if (graph_exec) {
      HIPCHK(hipGraphLaunch(graph_exec, ctx->stream));
    } else if (use_graph && t >= 1) {
      // the first iteration ran eagerly, so every workspace has its final size:
      // capture the second one (no allocation, synchronisation or memset inside)
      const bool prof = ctx->prof;
      ctx->prof = false;
      HIPCHK(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeRelaxed));
      const int rc = cg_iteration();
      hipGraph_t g = nullptr;
      const hipError_t ec = hipStreamEndCapture(ctx->stream, &g);
      ctx->prof = prof;
      CHK(rc);
      HIPCHK(ec);
      const hipError_t ei = hipGraphInstantiate(&graph_exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      HIPCHK(ei);
      graph_epoch = ctx->alloc_epoch;
      HIPCHK(hipGraphLaunch(graph_exec, ctx->stream));
    } else {
      CHK(cg_iteration());
    }
    stats.matvecs += 1;
    if (escalated) stats.fp32_iterations += 1;
    ++t;
    ++since_true;
    if (mixed && cfg.refine_every > 0 && since_true >= cfg.refine_every) {
      CHK(true_residual(ctx, px, theta, d, s, GP_FP32, false, pc));
      stats.matvecs += 1;
      stats.refinements += 1;
      since_true = 0;
    }
  }
  stats.iterations = t;
  stats.epochs = (double)t;
  stats.relres_y = ry;
  stats.relres_z = rz;
  return GP_OK;
}

// Column norms of R into s.rnorm (and the stop-test values on the host).
int residual_norms(gp_ctx* ctx, SolveState& s, double* ry, double* rz, int* st) {
  HIPCHK(col_dot_partial(s.R, nullptr, s.n, s.c, s.c, s.c, s.partial, s.nb, ctx->stream));
  HIPCHK(gamma_from_partial(s.partial, s.nb, s.c, nullptr, s.rnorm, s.status, ctx->stream));
  return read_norms(ctx, s, ry, rz, st);
}

// FP32 true residual of the current iterate (for the statistics), leaving R intact.
int true_residual_stats(gp_ctx* ctx, const Packed& px, const double* theta, int d, SolveState& s,
                        gp_solve_stats& stats) {
  float* T;
  CHK(ensure(ctx, B_AUX, (size_t)s.n * s.c, &T));
  CHK(kprod(ctx, px, px, s.Ut, s.c, s.c, s.HD, s.c, GP_FP32, a2_of(theta, d), s.Ut, s.c,
            s2_of(theta, d)));
  HIPCHK(residual_init(s.Bt, s.HD, T, nullptr, s.n, s.c, s.c, s.partial, s.nb, false,
                       ctx->stream));
  HIPCHK(gamma_from_partial(s.partial, s.nb, s.c, nullptr, s.rnorm, s.status, ctx->stream));
  int st = 0;
  CHK(read_norms(ctx, s, &stats.true_relres_y, &stats.true_relres_z, &st));
  stats.matvecs += 1;
  return status_to_error(ctx, st);
}

// Alternating projections (App. B, Algorithm 2).  The diagonal blocks H[I, I]
// are factored once per solve and their Cholesky factors inverted in place, so
// each iteration's block solve is two triangular products.  An iteration: the
// block solve for the selected block, u[I] += delta, the column-block product
// H[:, I] delta, and one pass over R that applies it and yields every block's
// score and the column norms.
int ap_solve(gp_ctx* ctx, const Packed& px, const float* X, const double* theta, int d,
             SolveState& s, const gp_solver_cfg& cfg, gp_solve_stats& stats) {
  const int64_t n = s.n;
  const int c = s.c;
  const int b = (int)std::min<int64_t>(cfg.ap_block, n);
  if (b < 1) return fail(ctx, GP_ERR_INVALID_ARG, "ap_block must be >= 1");
  const int P = (int)round_up(b, 64);
  if (P > kMaxAPBlock)
    return fail(ctx, GP_ERR_INVALID_ARG, "ap_block %d exceeds the supported %d", b, kMaxAPBlock);
  const int nblk = (int)((n + b - 1) / b);
  const double limit = cfg.max_epochs > 0 ? (double)n / b * cfg.max_epochs
                                          : (double)kSafetyCap * nblk;
  const float a2 = a2_of(theta, d), s2 = s2_of(theta, d);
  // Factor every diagonal block once (cached for this solve) and invert the factors.
  double* M;
  CHK(ensure(ctx, B_APF, (size_t)nblk * P * P, &M));
  HIPCHK(ap_build_blocks(px.xp, px.DP, d, n, b, P, (double)theta[d] * theta[d],
                         (double)theta[d + 1] * theta[d + 1], M, ctx->stream));
  HIPCHK(ap_cholesky(M, nblk, P, s.status, ctx->stream));
  HIPCHK(ap_invert_factors(M, nblk, P, ctx->stream));
  // r = b~ - H u~ (FP32)
  CHK(true_residual(ctx, px, theta, d, s, GP_FP32, false));
  stats.matvecs += 1;
  float *delta, *G;
  double *y, *scores;
  CHK(ensure(ctx, B_G, (size_t)P * c, &delta));
  CHK(ensure(ctx, B_APY, (size_t)P * c, &y));
  CHK(ensure(ctx, B_AUX, (size_t)n * c, &G));
  // per part of a block: its share of the block's score, then its column sums of squares
  const int nsub = ap_subblocks(b);
  const int nparts = nblk * nsub;
  CHK(ensure(ctx, B_ADJP, (size_t)nparts * (c + 1), &scores));
  double* part = scores + nparts;
  CHK(ensure_pinned(ctx, (size_t)kMaxC + 2 + nparts));
  HIPCHK(ap_update(s.R, c, nullptr, 0, n, b, c, 0, 0, nullptr, 0, 0.f, scores, part,
                   ctx->stream));
  HIPCHK(gamma_from_partial(part, nparts, c, nullptr, s.rnorm, s.status, ctx->stream));
  Packed pb;  // the selected block's points as kernel columns
  int64_t t = 0;
  double ry = 0, rz = 0;
  int st = 0;
  Progress prog;
  while (true) {
    HIPCHK(hipMemcpyAsync(ctx->hpin + kMaxC + 2, scores, nparts * sizeof(double),
                          hipMemcpyDeviceToHost, ctx->stream));
    CHK(read_norms(ctx, s, &ry, &rz, &st));
    CHK(status_to_error(ctx, st));
    prog.tick("ap", t, ry, rz);
    if (!keep_going(ry, rz, cfg.tol) || !((double)t < limit)) {
      stats.converged = !keep_going(ry, rz, cfg.tol);
      break;
    }
    // the block with the largest score, the lowest index on ties
    int k = 0;
    double best = -1.0;
    const double* sc = ctx->hpin + kMaxC + 2;
    for (int q = 0; q < nblk; ++q) {
      double v = 0.0;
      for (int u = 0; u < nsub; ++u) v += sc[q * nsub + u];
      if (v > best) {
        best = v;
        k = q;
      }
    }
    const int64_t base = (int64_t)k * b;
    const int bk = (int)std::min<int64_t>(b, n - base);
    // delta = H[I,I]^-1 r[I];  u[I] += delta;  r -= H[:, I] delta
    HIPCHK(ap_solve_block(M, P, k, b, n, s.R, c, c, y, delta, c, ctx->stream));
    HIPCHK(add_block(s.Ut, c, base, bk, delta, c, c, 1.f, ctx->stream));
    CHK(pack_points(ctx, B_XP2, X + base * d, nullptr, bk, d, theta, &pb, &px));
    CHK(kprod(ctx, px, pb, delta, c, c, G, c, cfg.precision, a2, nullptr, 0, 0.f));
    HIPCHK(ap_update(s.R, c, G, c, n, b, c, base, bk, delta, c, s2, scores, part,
                     ctx->stream));
    HIPCHK(gamma_from_partial(part, nparts, c, nullptr, s.rnorm, s.status, ctx->stream));
    ++t;
  }
  stats.iterations = t;
  stats.epochs = (double)t * b / n;
  stats.relres_y = ry;
  stats.relres_z = rz;
  if (t > 0) CHK(true_residual_stats(ctx, px, theta, d, s, stats));
  return GP_OK;
}

// Floyd's sampling of b distinct indices from [0, n).
void draw_batch(std::mt19937_64& rng, int64_t n, int b, int32_t* out, std::vector<char>& seen) {
  if ((int64_t)seen.size() != n) seen.assign(n, 0);
  int cnt = 0;
  for (int64_t j = n - b; j < n; ++j) {
    std::uniform_int_distribution<int64_t> dist(0, j);
    int64_t v = dist(rng);
    if (seen[v]) v = j;
    seen[v] = 1;
    out[cnt++] = (int32_t)v;
  }
  for (int q = 0; q < cnt; ++q) seen[out[q]] = 0;
}

// Stochastic gradient descent (App. B, Algorithm 3).  An iteration is the row
// product H[I, :] u on the batch rows (u's forward tiles packed by the previous
// iteration), the gradient fix-up, ksgd_sparse (batch rows: momentum, residual
// estimate, running norms) and ksgd_update_pack (all rows: momentum decay,
// u += m, packing u for the next product).  The residual estimate's column norms
// are kept as running sums of squares in FP64, recomputed from R every
// kSgdRenorm iterations.
constexpr int64_t kSgdRenorm = 1024;

int sgd_solve(gp_ctx* ctx, const Packed& px, const float* X, const double* theta, int d,
              SolveState& s, const gp_solver_cfg& cfg, gp_solve_stats& stats) {
  const int64_t n = s.n;
  const int c = s.c;
  const int b = (int)std::min<int64_t>(cfg.sgd_batch, n);
  if (b < 1) return fail(ctx, GP_ERR_INVALID_ARG, "sgd_batch must be >= 1");
  double limit = cfg.max_epochs > 0 ? (double)n / b * cfg.max_epochs : (double)kSafetyCap;
  if (cfg.sgd_batches) limit = std::min(limit, (double)cfg.sgd_batches_count);
  const float a2 = a2_of(theta, d), s2 = s2_of(theta, d);
  const float rho = (float)cfg.sgd_momentum, lrb = (float)(cfg.sgd_lr / b);
  float *Mom, *G;
  int32_t *idx, *stamp;
  CHK(ensure(ctx, B_MOM, (size_t)n * c, &Mom));
  CHK(ensure(ctx, B_G, (size_t)round_up(b, kRowAlign) * c, &G));
  CHK(ensure(ctx, B_IDX, (size_t)b * 2, &idx));
  CHK(ensure(ctx, B_STAMP, (size_t)n, &stamp));
  HIPCHK(fill(Mom, n * c, 0.f, ctx->stream));
  HIPCHK(fill_i32(stamp, n, -1, ctx->stream));
  // residual estimate starts at b~ (as printed, also under warm start)
  HIPCHK(copy_cols(s.Bt, c, n, c, s.R, c, ctx->stream));
  double* sumsq = s.gamma;  // running column sums of squares of R
  auto renorm = [&]() -> int {
    HIPCHK(col_dot_partial(s.R, nullptr, n, c, c, c, s.partial, s.nb, ctx->stream));
    HIPCHK(gamma_from_partial(s.partial, s.nb, c, sumsq, s.rnorm, s.status, ctx->stream));
    return GP_OK;
  };
  CHK(renorm());
  // forward tiles of u for the product (one pass: c <= 80 columns), packed here
  // and then by every iteration's update
  const bool fused = c <= 80;
  const int CT = select_CT(c);
  uint16_t *vhi = nullptr, *vlo = nullptr;
  float* vf = nullptr;
  const bool perm = kprod_v_perm(px, px, cfg.precision);
  if (fused) {
    const size_t vcount = (size_t)(px.n_pad * 16 * CT);
    if (cfg.precision == GP_FP32) {
      CHK(ensure(ctx, B_VHI, vcount, &vf));
      HIPCHK(pack_v_f32(s.Ut, n, c, c, nullptr, CT, vf, px.n_pad, perm, ctx->stream));
    } else {
      CHK(ensure(ctx, B_VHI, vcount, &vhi));
      if (cfg.precision == GP_BF16X3) CHK(ensure(ctx, B_VLO, vcount, &vlo));
      HIPCHK(pack_v_bf16(s.Ut, n, c, c, nullptr, CT, vhi, vlo, px.n_pad, perm, ctx->stream));
    }
  }
  CHK(ensure_pinned(ctx, (size_t)kMaxC + 2 + b));
  int32_t* hidx = reinterpret_cast<int32_t*>(ctx->hpin + kMaxC + 2);
  std::mt19937_64 rng(cfg.sgd_seed);
  std::vector<char> seen;
  int64_t t = 0;
  double ry = 0, rz = 0;
  int st = 0;
  Progress prog;
  while (true) {
    if (t > 0 && t % kSgdRenorm == 0) CHK(renorm());
    CHK(read_norms(ctx, s, &ry, &rz, &st));
    CHK(status_to_error(ctx, st));
    prog.tick("sgd", t, ry, rz);
    if (!keep_going(ry, rz, cfg.tol) || !((double)t < limit)) {
      stats.converged = !keep_going(ry, rz, cfg.tol);
      break;
    }
    if (cfg.sgd_batches) {
      const int32_t* src = cfg.sgd_batches + t * b;
      if ((int64_t)seen.size() != n) seen.assign(n, 0);
      int bad = 0;
      for (int q = 0; q < b; ++q) {
        if (src[q] < 0 || src[q] >= n) {
          bad = 1;
          break;
        }
        if (seen[src[q]]) {
          bad = 2;
          break;
        }
        seen[src[q]] = 1;
        hidx[q] = src[q];
      }
      for (int q = 0; q < b; ++q)
        if (src[q] >= 0 && src[q] < n) seen[src[q]] = 0;
      if (bad == 1) return fail(ctx, GP_ERR_INVALID_ARG, "sgd batch %lld holds an index outside [0, n)", (long long)t);
      if (bad == 2) return fail(ctx, GP_ERR_INVALID_ARG, "sgd batch %lld repeats an index", (long long)t);
    } else {
      draw_batch(rng, n, b, hidx, seen);
    }
    // the pinned staging buffer is reused next iteration after the norm read syncs
    HIPCHK(hipMemcpyAsync(idx, hidx, b * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
    Packed pr;
    CHK(pack_points(ctx, B_XP2, X, idx, b, d, theta, &pr, &px));
    // g[I] = H[I, :] u - b~[I]
    CHK(kprod(ctx, pr, px, s.Ut, c, c, G, c, cfg.precision, a2, nullptr, 0, 0.f, FN_MATERN, 0,
              fused));
    HIPCHK(sgd_fix(G, c, s.Ut, s.Bt, c, idx, b, c, s2, ctx->stream));
    const int tag = (int)(t & 0x7fffffff);
    if (fused) {
      // m[I] = rho m[I] - (lr/b) g; r[I] = g;  m = rho m elsewhere;  u += m
      HIPCHK(sgd_sparse(G, c, idx, b, Mom, s.R, c, c, rho, lrb, stamp, tag, sumsq, s.rnorm,
                        s.status, ctx->stream));
      HIPCHK(sgd_update_pack(s.Ut, Mom, c, stamp, tag, rho, n, c, CT, perm, px.n_pad, vhi, vlo,
                             vf, ctx->stream));
    } else {
      HIPCHK(sgd_momentum(Mom, G, idx, b, n, c, c, rho, lrb, ctx->stream));
      HIPCHK(sgd_finish(s.Ut, s.R, Mom, G, idx, b, n, c, c, ctx->stream));
      CHK(renorm());
    }
    ++t;
  }
  stats.iterations = t;
  stats.epochs = (double)t * b / n;
  stats.relres_y = ry;
  stats.relres_z = rz;
  if (t > 0) CHK(true_residual_stats(ctx, px, theta, d, s, stats));
  return GP_OK;
}

int solve_dispatch(gp_ctx* ctx, const Packed& px, const float* X, const double* theta, int d,
                   const float* B, int64_t ldb, float* U, int64_t ldu, int c,
                   const gp_solver_cfg& cfg, gp_solve_stats& stats);

// ------------------------------------------------------------ workspace plan
// The largest request every workspace buffer receives during one call of an
// operation, in bytes, computed with the same counts as the ensure() calls of
// the code paths above (pack_points, kprod, solve_setup, the solvers, the
// preconditioner, the right-hand sides and the adjoint).  Where a size depends
// on the data (the cross-term distance form, the rank the factor reaches) the
// larger case is planned.
struct WsPlan {
  size_t bytes[B_COUNT] = {};
  size_t pinned = kMaxC + 2;  // doubles of pinned host staging (norm reads)
  void need(BufId id, size_t b) { bytes[id] = std::max(bytes[id], b); }
  void need_pinned(size_t doubles) { pinned = std::max(pinned, doubles); }
  size_t held() const {
    // ensure() allocates max(bytes, 256) plus one eighth
    size_t t = 0;
    for (size_t b : bytes)
      if (b) {
        const size_t v = std::max<size_t>(b, 256);
        t += v + v / 8;
      }
    return t;
  }
};

void plan_pack(WsPlan& p, BufId id, int64_t n, int d) {
  const int64_t n_pad = round_up(std::max<int64_t>(n, 1), kRowAlign);
  const int D = select_D(d);
  p.need(id, (size_t)(n_pad * dp_of(D)) * sizeof(float));
  if (D > 3)
    p.need(id == B_XP1 ? B_XT1 : B_XT2, (size_t)(n_pad * 4 * xt_chunks(D)) * sizeof(float));
  p.need(B_XTMAX, 3 * sizeof(unsigned));
}

void plan_kprod(WsPlan& p, int64_t n1, int64_t n2, int d, int cols, int prec) {
  const int64_t n1_pad = round_up(std::max<int64_t>(n1, 1), kRowAlign);
  const int64_t n2_pad = round_up(std::max<int64_t>(n2, 1), kRowAlign);
  const int D = select_D(d);
  const int npass = (cols + 79) / 80;
  const int per = (cols + npass - 1) / npass;
  for (int c0 = 0; c0 < cols; c0 += per) {
    const int cs = std::min(per, cols - c0);
    const int CT = select_CT(cs);
    const size_t vcount = (size_t)(n2_pad * 16 * CT);
    if (prec == GP_FP32) {
      p.need(B_VHI, vcount * sizeof(float));
    } else {
      p.need(B_VHI, vcount * sizeof(uint16_t));
      if (prec == GP_BF16X3) p.need(B_VLO, vcount * sizeof(uint16_t));
    }
    for (int xt = 0; xt < 2; ++xt) {
      const int rs = xt ? fwd_xt_row_subtiles(CT, xt_chunks(D)) : fwd_row_subtiles(CT);
      const int S = choose_splits(n1_pad / (64 * rs), n2_pad / kJStep);
      if (S > 1) p.need(B_PART, (size_t)(S * n1_pad * 16 * CT) * sizeof(float));
    }
  }
}

void plan_col_sums(WsPlan& p, int64_t n, int c) {
  p.need(B_PARTIAL, (size_t)reduce_blocks(n) * std::min(c, kMaxSolveC) * sizeof(double));
  p.need(B_SCALD, (size_t)6 * kMaxC * sizeof(double));
}

void plan_solve(WsPlan& p, int64_t n, int d, int c, const gp_solver_cfg& cfg) {
  plan_pack(p, B_XP1, n, d);
  const size_t vec = (size_t)std::max<int64_t>(n, 1) * c * sizeof(float);
  for (BufId id : {B_BT, B_UT, B_R, B_DV, B_HD}) p.need(id, vec);
  p.need(B_SCALD, (size_t)6 * kMaxC * sizeof(double));
  p.need(B_SCALF, (size_t)kMaxC * sizeof(float));
  p.need(B_STATUS, 16 * sizeof(int));
  p.need(B_PARTIAL, (size_t)reduce_blocks(n) * c * sizeof(double));
  plan_kprod(p, n, n, d, c, GP_FP32);  // true residuals
  plan_kprod(p, n, n, d, c, cfg.precision);
  if (cfg.solver == GP_CG) {
    p.need(B_AUX, vec);  // the true residual of a solve the budget stops
    const int k = (int)std::min<int64_t>(cfg.precond_rank, n);
    if (k > 0) {
      const int64_t ldl = round_up(n, 64);
      const int kp = (int)round_up(k, 64);
      p.need(B_Z, vec);
      p.need(B_PCSUM, sizeof(unsigned long long));
      p.need(B_PCL32, (size_t)k * ldl * sizeof(float));
      p.need(B_PCPIV, (size_t)k * sizeof(int32_t));
      p.need(B_PCDIAG, (size_t)n * sizeof(double));
      p.need(B_PCLP, (size_t)k * sizeof(double));
      p.need(B_PCPV, (size_t)pc_parts(n) * sizeof(double));
      p.need(B_PCPI, (size_t)pc_parts(n) * sizeof(int64_t));
      p.need(B_PCST, sizeof(PcState));
      p.need(B_PCELL, (size_t)d * sizeof(double));
      p.need(B_PCG, (size_t)k * k * sizeof(double));
      p.need(B_PCA, (size_t)kp * kp * sizeof(double));
      p.need(B_PCM, (size_t)kp * kp * sizeof(double));
      p.need(B_PCW, (size_t)kp * kp * sizeof(double));
      p.need(B_PCID, (size_t)kp * sizeof(double));
      p.need(B_PCSTAT, sizeof(int));
      const int64_t parts = std::max({pc_gram_parts(n, k),
                                      pc_apply_parts(n, k, c)});
      p.need(B_PCPART, (size_t)parts * sizeof(double));
      p.need(B_PCT, (size_t)k * c * sizeof(double));
      p.need(B_PCS, (size_t)k * c * sizeof(double));
    }
  } else if (cfg.solver == GP_AP) {
    const int b = (int)std::max<int64_t>(1, std::min<int64_t>(cfg.ap_block, n));
    const int P = (int)round_up(b, 64);
    const int nblk = (int)((n + b - 1) / b);
    p.need(B_APF, (size_t)nblk * P * P * sizeof(double));
    p.need(B_G, (size_t)P * c * sizeof(float));
    p.need(B_APY, (size_t)P * c * sizeof(double));
    p.need(B_AUX, vec);
    p.need(B_ADJP, (size_t)nblk * ap_subblocks(b) * (c + 1) * sizeof(double));
    p.need_pinned((size_t)kMaxC + 2 + (size_t)nblk * ap_subblocks(b));
    plan_pack(p, B_XP2, b, d);  // the selected block's points
    plan_kprod(p, n, b, d, c, cfg.precision);
  } else {
    const int b = (int)std::max<int64_t>(1, std::min<int64_t>(cfg.sgd_batch, n));
    p.need(B_MOM, vec);
    p.need(B_STAMP, (size_t)std::max<int64_t>(n, 1) * sizeof(int32_t));
    p.need(B_G, (size_t)round_up(b, kRowAlign) * c * sizeof(float));
    p.need(B_IDX, (size_t)b * 2 * sizeof(int32_t));
    p.need(B_AUX, vec);
    p.need_pinned((size_t)kMaxC + 2 + b);
    plan_pack(p, B_XP2, b, d);
    plan_kprod(p, b, n, d, c, cfg.precision);
  }
}

void plan_adjoint(WsPlan& p, int64_t n, int d, int c, int precision) {
  plan_pack(p, B_XP1, n, d);
  plan_col_sums(p, n, c);
  const int64_t n_pad = round_up(std::max<int64_t>(n, 1), kRowAlign);
  const int D = select_D(d);
  // per-parameter form
  p.need(B_AUX, (size_t)n * c * sizeof(float));
  plan_kprod(p, n, n, d, c, GP_FP32);
  // fused form
  p.need(B_SCALF, (size_t)kMaxC * sizeof(float));
  for (int g0 = 0; g0 < c; g0 += kAdjMaxCols) {
    const int CK = 32 * select_KT(std::min(kAdjMaxCols, c - g0));
    const size_t pc = (size_t)(n_pad * CK);
    if (precision == GP_BF16X3) {
      for (BufId id : {B_UHI, B_ULO, B_WHI, B_WLO}) p.need(id, pc * sizeof(uint16_t));
    } else {
      p.need(B_UHI, pc * 2 * sizeof(uint16_t));
      p.need(B_WHI, pc * 2 * sizeof(uint16_t));
    }
    const int64_t rowblocks = n_pad / kAdjRowsPerWG;
    int S = 1;
    while (rowblocks * S < 2048 && (n_pad / 16) / (2 * S) >= 32) S *= 2;
    p.need(B_ADJP, (size_t)(rowblocks * S * (D + 1)) * sizeof(double));
    p.need_pinned((size_t)(rowblocks * S * (D + 1)));
  }
}

int ws_plan(int op, int64_t n, int d, int c, const gp_solver_cfg* cfg, int M, WsPlan& p,
            gp_ctx* ctx) {
  if (n < 0) return fail(ctx, GP_ERR_INVALID_ARG, "n < 0");
  if (op == GP_WS_KMATVEC) {
    CHK(check_dims(ctx, d, c));
    const int prec = cfg ? cfg->precision : GP_FP32;
    CHK(check_prec(ctx, prec));
    if (n == 0 || c == 0) return GP_OK;
    plan_pack(p, B_XP1, n, d);
    plan_kprod(p, n, n, d, c, prec);
    return GP_OK;
  }
  if (op != GP_WS_SOLVE && op != GP_WS_MLL_GRAD)
    return fail(ctx, GP_ERR_INVALID_ARG, "unknown workspace operation %d", op);
  if (!cfg) return fail(ctx, GP_ERR_INVALID_ARG, "cfg is NULL");
  CHK(check_dims(ctx, d, c, kMaxSolveC));
  CHK(check_prec(ctx, cfg->precision));
  CHK(check_precond(ctx, *cfg));
  if (cfg->solver != GP_CG && cfg->solver != GP_AP && cfg->solver != GP_SGD)
    return fail(ctx, GP_ERR_INVALID_ARG, "solver %d not available", cfg->solver);
  if (n == 0 || c == 0) return GP_OK;
  plan_solve(p, n, d, c, *cfg);
  if (op == GP_WS_MLL_GRAD) {
    if (M < 0) return fail(ctx, GP_ERR_INVALID_ARG, "M = %d must be >= 0", M);
    p.need(B_RHS, (size_t)n * c * sizeof(float));
    p.need(B_WB, (size_t)n * c * sizeof(float));  // standard estimator
    if (M > 0) {
      p.need(B_OMEGA, (size_t)M * d * sizeof(double));
      p.need(B_INVELL, (size_t)kMaxD * sizeof(double));
    }
    plan_adjoint(p, n, d, c, cfg->precision == GP_FP32 ? GP_FP32 : GP_BF16X3);
  }
  return GP_OK;
}

}  // namespace

// ====================================================================== C ABI

extern "C" {

const char* gp_version(void) { return "gpmi 0.1 gfx950"; }

int gp_ctx_create(int device, void* stream, gp_ctx** out) {
  gp_ctx* ctx = nullptr;
  if (!out) return GP_ERR_INVALID_ARG;
  *out = nullptr;
  HIPCHK(hipSetDevice(device));
  if (device < 0 || device >= kMaxDevices) return GP_ERR_INVALID_ARG;
  {
    // the allocation-free entry point's scratch address on this device
    unsigned char* sp = nullptr;
    const int rs = scratch_address(device, &sp);
    if (rs != GP_OK) return rs;
  }
  ctx = new gp_ctx();
  ctx->device = device;
  ctx->stream = (hipStream_t)stream;
  *out = ctx;
  return GP_OK;
}

void gp_ctx_destroy(gp_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (int k = 0; k < kProfClasses; ++k)
    for (auto& p : ctx->ev[k]) {
      (void)hipEventDestroy(p.first);
      (void)hipEventDestroy(p.second);
    }
  for (auto e : ctx->pool) (void)hipEventDestroy(e);
  if (ctx->gstream) {
    (void)hipStreamSynchronize(ctx->gstream);
    (void)hipStreamDestroy(ctx->gstream);
  }
  for (auto e : ctx->gev)
    if (e) (void)hipEventDestroy(e);
  if (ctx->xstream) {
    (void)hipStreamSynchronize(ctx->xstream);
    (void)hipStreamDestroy(ctx->xstream);
  }
  for (auto e : ctx->xev) (void)hipEventDestroy(e);
  for (int i = 0; i < B_COUNT; ++i)
    if (ctx->buf[i]) (void)hipFree(ctx->buf[i]);
  if (ctx->hpin) (void)hipHostFree(ctx->hpin);
  delete ctx;
}

const char* gp_last_error(const gp_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int gp_profile_enable(gp_ctx* ctx, int enable) {
  if (!ctx) return GP_ERR_INVALID_ARG;
  ctx->err.clear();
  HIPCHK(hipSetDevice(ctx->device));
  CHK(harvest(ctx));
  ctx->prof = enable != 0;
  for (int k = 0; k < kProfClasses; ++k) {
    ctx->prof_ms[k] = 0.0;
    ctx->prof_n[k] = 0;
  }
  return GP_OK;
}

int gp_profile_read(gp_ctx* ctx, int which, double* total_ms, int64_t* launches) {
  if (!ctx || which < 0 || which >= kProfClasses) return GP_ERR_INVALID_ARG;
  ctx->err.clear();
  HIPCHK(hipSetDevice(ctx->device));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  CHK(harvest(ctx));
  if (total_ms) *total_ms = ctx->prof_ms[which];
  if (launches) *launches = ctx->prof_n[which];
  return GP_OK;
}

int gp_workspace_size(int op, int64_t n, int d, int c, const gp_solver_cfg* cfg, int M,
                      size_t* bytes) {
  if (!bytes) return GP_ERR_INVALID_ARG;
  WsPlan p;
  const int r = ws_plan(op, n, d, c, cfg, M, p, nullptr);
  if (r != GP_OK) return r;
  *bytes = p.held();
  return GP_OK;
}

int gp_workspace_reserve(gp_ctx* ctx, int op, int64_t n, int d, int c, const gp_solver_cfg* cfg,
                         int M) {
  if (!ctx) return GP_ERR_INVALID_ARG;
  ctx->err.clear();
  WsPlan p;
  CHK(ws_plan(op, n, d, c, cfg, M, p, ctx));
  HIPCHK(hipSetDevice(ctx->device));
  for (int id = 0; id < B_COUNT; ++id)
    if (p.bytes[id]) {
      unsigned char* ptr;
      CHK(ensure(ctx, (BufId)id, p.bytes[id], &ptr));
    }
  // the pinned host staging of the solvers' norm reads and of the adjoint partials
  CHK(ensure_pinned(ctx, p.pinned));
  return GP_OK;
}

int gp_workspace_held(const gp_ctx* ctx, size_t* bytes) {
  if (!ctx || !bytes) return GP_ERR_INVALID_ARG;
  size_t t = 0;
  for (int id = 0; id < B_COUNT; ++id) t += ctx->cap[id];
  *bytes = t;
  return GP_OK;
}

int gp_kmatvec(gp_ctx* ctx, const float* X1, int64_t n1, const float* X2, int64_t n2, int d,
               const double* theta, const float* V, int64_t ldv, int c, float* out, int64_t ldo,
               int precision, int add_noise) {
  if (!ctx) return GP_ERR_INVALID_ARG;
  ctx->err.clear();
  CHK(check_dims(ctx, d, c));
  CHK(check_theta(ctx, theta, d));
  CHK(check_prec(ctx, precision));
  CHK(check_mat(ctx, "X1", X1, n1, d, d));
  CHK(check_mat(ctx, "X2", X2, n2, d, d));
  CHK(check_mat(ctx, "V", V, n2, ldv, c));
  CHK(check_mat(ctx, "out", out, n1, ldo, c));
  if (add_noise && n1 != n2)
    return fail(ctx, GP_ERR_INVALID_ARG, "add_noise needs n1 == n2 (got %lld, %lld)",
                (long long)n1, (long long)n2);
  HIPCHK(hipSetDevice(ctx->device));
  if (n1 == 0 || c == 0) return GP_OK;
  if (n2 == 0) {
    for (int64_t i = 0; i < n1; ++i)
      HIPCHK(hipMemsetAsync(out + i * ldo, 0, c * sizeof(float), ctx->stream));
    return GP_OK;
  }
  Packed p1, p2;
  CHK(pack_points(ctx, B_XP1, X1, nullptr, n1, d, theta, &p1));
  if (X2 == X1 && n2 == n1)
    p2 = p1;
  else
    CHK(pack_points(ctx, B_XP2, X2, nullptr, n2, d, theta, &p2));
  return kprod(ctx, p1, p2, V, ldv, c, out, ldo, precision, a2_of(theta, d),
               add_noise ? V : nullptr, ldv, s2_of(theta, d));
}

int gp_kmatvec_static(gp_ctx* ctx, const float* X1, int64_t n1, const float* X2, int64_t n2,
                      int d, const double* theta, const float* V, int64_t ldv, int c, float* out,
                      int64_t ldo, int precision, int add_noise) {
  if (!ctx) return GP_ERR_INVALID_ARG;
  ctx->err.clear();
  unsigned char* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (ctx->device >= 0 && ctx->device < kMaxDevices) base = g_scratch_ptr[ctx->device];
  }
  if (!base) return fail(ctx, GP_ERR_HIP, "no static scratch address for device %d", ctx->device);
  // The same validation as gp_kmatvec, then the plan: every buffer of the call must
  // fit the scratch (column-split partial sums excepted: kprod fits their number).
  CHK(check_dims(ctx, d, c));
  CHK(check_prec(ctx, precision));
  WsPlan plan;
  plan_pack(plan, B_XP1, n1, d);
  if (!(X2 == X1 && n2 == n1)) plan_pack(plan, B_XP2, n2, d);
  {
    WsPlan v;
    plan_kprod(v, n1, n2, d, c, precision);
    plan.need(B_VHI, v.bytes[B_VHI]);
    plan.need(B_VLO, v.bytes[B_VLO]);
  }
  size_t need = 0;
  for (size_t b : plan.bytes)
    if (b) need += (std::max<size_t>(b, 256) + 255) & ~(size_t)255;
  if (need > kStaticScratchBytes)
    return fail(ctx, GP_ERR_INVALID_ARG,
                "n1 = %lld, n2 = %lld, d = %d, c = %d needs %zu bytes of scratch; the "
                "allocation-free product has %zu", (long long)n1, (long long)n2, d, c, need,
                kStaticScratchBytes);
  // arena scope: workspace from the scratch array, host staging in the context,
  // no per-launch profiling events (their creation could allocate)
  struct Scope {
    gp_ctx* c;
    double* hpin;
    size_t hcap;
    bool prof;
    Scope(gp_ctx* ctx, unsigned char* base) : c(ctx), hpin(ctx->hpin), hcap(ctx->hpin_cap),
                                             prof(ctx->prof) {
      c->arena.on = true;
      c->arena.base = base;
      c->arena.cap = kStaticScratchBytes;
      c->arena.used = 0;
      for (int i = 0; i < B_COUNT; ++i) {
        c->arena.ptr[i] = nullptr;
        c->arena.size[i] = 0;
      }
      c->hpin = c->arena_host;
      c->hpin_cap = sizeof(c->arena_host) / sizeof(double);
      c->prof = false;
    }
    ~Scope() {
      c->arena.on = false;
      c->hpin = hpin;
      c->hpin_cap = hcap;
      c->prof = prof;
    }
  } scope(ctx, base);
  return gp_kmatvec(ctx, X1, n1, X2, n2, d, theta, V, ldv, c, out, ldo, precision, add_noise);
}

int gp_kmatvec_adjoint(gp_ctx* ctx, const float* X, int64_t n, int d, const double* theta,
                       const float* U, int64_t ldu, const float* W, int64_t ldw, int c,
                       const double* col_weights, int precision, int mode, double* grad_out) {
  if (!ctx) return GP_ERR_INVALID_ARG;
  ctx->err.clear();
  CHK(check_dims(ctx, d, c));
  CHK(check_theta(ctx, theta, d));
  CHK(check_mat(ctx, "X", X, n, d, d));
  CHK(check_mat(ctx, "U", U, n, ldu, c));
  CHK(check_mat(ctx, "W", W, n, ldw, c));
  if (!grad_out) return fail(ctx, GP_ERR_INVALID_ARG, "grad_out is NULL");
  if (c > 0 && !col_weights) return fail(ctx, GP_ERR_INVALID_ARG, "col_weights is NULL");
  if (precision != GP_FP32 && precision != GP_BF16X3)
    return fail(ctx, GP_ERR_INVALID_ARG, "adjoint precision must be GP_FP32 or GP_BF16X3");
  if (mode != GP_ADJ_FUSED && mode != GP_ADJ_PER_PARAM)
    return fail(ctx, GP_ERR_INVALID_ARG, "unknown adjoint mode %d", mode);
  HIPCHK(hipSetDevice(ctx->device));
  for (int k = 0; k < d + 2; ++k) grad_out[k] = 0.0;
  if (n == 0 || c == 0) return GP_OK;
  Packed px;
  CHK(pack_points(ctx, B_XP1, X, nullptr, n, d, theta, &px));
  const double a = theta[d], sigma = theta[d + 1];
  const double log2e = 1.4426950408889634074;
  // sigma term: 2 sigma sum_c w_c U_c . W_c
  std::vector<double> uw(c);
  CHK(col_sums(ctx, U, W, n, ldu, ldw, c, uw.data()));
  double sw = 0.0;
  for (int k = 0; k < c; ++k) sw += col_weights[k] * uw[k];
  grad_out[d + 1] = 2.0 * sigma * sw;

  if (mode == GP_ADJ_PER_PARAM) {
    // d + 1 separate FP32 derivative-kernel products, each dotted with U.
    float* Y;
    CHK(ensure(ctx, B_AUX, (size_t)n * c, &Y));
    std::vector<double> dots(c);
    for (int k = 0; k <= d; ++k) {
      const bool amp = k == d;
      const float scale = amp ? (float)(2.0 * a) : (float)(a * a / (theta[k] * log2e * log2e));
      CHK(kprod(ctx, px, px, W, ldw, c, Y, c, GP_FP32, scale, nullptr, 0, 0.f,
                amp ? FN_MATERN : FN_DLEN, k));
      CHK(col_sums(ctx, U, Y, n, ldu, c, c, dots.data()));
      double g = 0.0;
      for (int j = 0; j < c; ++j) g += col_weights[j] * dots[j];
      grad_out[k] = g;
    }
    return GP_OK;
  }

  // Fused one-pass adjoint, over groups of at most 256 columns (the sum over
  // columns separates; one group holds 8 K-tiles of 32 columns).
  float* wf;
  CHK(ensure(ctx, B_SCALF, (size_t)kMaxC, &wf));
  CHK(ensure_pinned(ctx, kMaxC));
  {
    float* hw = reinterpret_cast<float*>(ctx->hpin);
    for (int k = 0; k < c; ++k) hw[k] = (float)col_weights[k];
    HIPCHK(hipMemcpyAsync(wf, hw, c * sizeof(float), hipMemcpyHostToDevice, ctx->stream));
  }
  const int nd = px.D + 1;
  std::vector<double> S(nd, 0.0);
  for (int g0 = 0; g0 < c; g0 += kAdjMaxCols) {
    const int cg = std::min(kAdjMaxCols, c - g0);
    const int KT = select_KT(cg);
    const int CK = 32 * KT;
    AdjArgs aa;
    aa.prec = precision;
    aa.D = px.D;
    aa.xp = px.xp;
    aa.n_pad = px.n_pad;
    aa.KT = KT;
    const size_t pc = (size_t)(px.n_pad * CK);
    if (precision == GP_BF16X3) {
      uint16_t *uh, *ul, *wh, *wl;
      CHK(ensure(ctx, B_UHI, pc, &uh));
      CHK(ensure(ctx, B_ULO, pc, &ul));
      CHK(ensure(ctx, B_WHI, pc, &wh));
      CHK(ensure(ctx, B_WLO, pc, &wl));
      HIPCHK(pack_rows_bf16(U + g0, n, ldu, cg, wf + g0, KT, uh, ul, px.n_pad, ctx->stream));
      HIPCHK(pack_rows_bf16(W + g0, n, ldw, cg, nullptr, KT, wh, wl, px.n_pad, ctx->stream));
      aa.uhi = uh; aa.ulo = ul; aa.whi = wh; aa.wlo = wl;
    } else {
      float *uf, *wf2;
      CHK(ensure(ctx, B_UHI, pc * 2, (uint16_t**)&uf));
      CHK(ensure(ctx, B_WHI, pc * 2, (uint16_t**)&wf2));
      HIPCHK(pack_rows_f32(U + g0, n, ldu, cg, wf + g0, KT, uf, px.n_pad, ctx->stream));
      HIPCHK(pack_rows_f32(W + g0, n, ldw, cg, nullptr, KT, wf2, px.n_pad, ctx->stream));
      aa.uhi = uf; aa.whi = wf2;
    }
    const int64_t rowblocks = px.n_pad / kAdjRowsPerWG;
    aa.S = 1;
    while (rowblocks * aa.S < 2048 && (px.n_pad / 16) / (2 * aa.S) >= 32) aa.S *= 2;
    double* part;
    CHK(ensure(ctx, B_ADJP, (size_t)(rowblocks * aa.S * nd), &part));
    aa.partial = part;
    int64_t rows = 0;
    {
      ProfScope ps(ctx, 1);
      HIPCHK(adj(aa, &rows, ctx->stream));
    }
    CHK(ensure_pinned(ctx, (size_t)rows * nd));
    HIPCHK(hipMemcpyAsync(ctx->hpin, part, rows * nd * sizeof(double), hipMemcpyDeviceToHost,
                          ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (int64_t r = 0; r < rows; ++r)
      for (int k = 0; k < nd; ++k) S[k] += ctx->hpin[r * nd + k];
  }
  for (int k = 0; k < d; ++k) grad_out[k] = a * a / (theta[k] * log2e * log2e) * S[k];
  grad_out[d] = 2.0 * a * S[px.D];
  return GP_OK;
}

void gp_solver_cfg_default(gp_solver_cfg* cfg) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof *cfg);
  cfg->solver = GP_CG;
  cfg->tol = 0.01;
  cfg->max_epochs = 0.0;
  cfg->precision = GP_FP32;
  cfg->refine_every = 0;
  cfg->check_every = 0;
  cfg->ap_block = 1000;
  cfg->sgd_batch = 500;
  cfg->sgd_lr = 10.0;
  cfg->sgd_momentum = 0.9;
  cfg->sgd_batches = nullptr;
  cfg->sgd_batches_count = 0;
  cfg->sgd_seed = 0;
  cfg->precond_rank = 0;
  cfg->use_graph = 0;
  cfg->precond_reuse = 0;
}

int gp_solve(gp_ctx* ctx, const float* X, int64_t n, int d, const double* theta, const float* B,
             int64_t ldb, float* U, int64_t ldu, int c, const gp_solver_cfg* cfg,
             gp_solve_stats* stats) {
  if (!ctx) return GP_ERR_INVALID_ARG;
  ctx->err.clear();
  gp_solve_stats local{};
  gp_solve_stats& s = stats ? *stats : local;
  std::memset(&s, 0, sizeof s);
  s.true_relres_y = s.true_relres_z = std::numeric_limits<double>::quiet_NaN();
  if (!cfg) return fail(ctx, GP_ERR_INVALID_ARG, "cfg is NULL");
  CHK(check_dims(ctx, d, c, kMaxSolveC));
  CHK(check_theta(ctx, theta, d));
  CHK(check_prec(ctx, cfg->precision));
  CHK(check_mat(ctx, "X", X, n, d, d));
  CHK(check_mat(ctx, "B", B, n, ldb, c));
  CHK(check_mat(ctx, "U", U, n, ldu, c));
  if (!(cfg->tol >= 0.0)) return fail(ctx, GP_ERR_INVALID_ARG, "tol must be >= 0");
  CHK(check_precond(ctx, *cfg));
  HIPCHK(hipSetDevice(ctx->device));
  if (n == 0 || c == 0) {
    s.converged = 1;
    return GP_OK;
  }
  Packed px;
  CHK(pack_points(ctx, B_XP1, X, nullptr, n, d, theta, &px));
  const int r = solve_dispatch(ctx, px, X, theta, d, B, ldb, U, ldu, c, *cfg, s);
  s.status = r;
  return r;
}

int gp_pivoted_cholesky(gp_ctx* ctx, const float* X, int64_t n, int d, const double* theta,
                        int k, double* L, int64_t ldl, int32_t* piv, int* rank) {
  if (!ctx) return GP_ERR_INVALID_ARG;
  ctx->err.clear();
  if (!rank) return fail(ctx, GP_ERR_INVALID_ARG, "rank is NULL");
  *rank = 0;
  CHK(check_dims(ctx, d, 1));
  CHK(check_theta(ctx, theta, d));
  if (k < 0 || k > kMaxPrecondRank)
    return fail(ctx, GP_ERR_INVALID_ARG, "k %d outside [0, %d]", k, kMaxPrecondRank);
  if (n < 0) return fail(ctx, GP_ERR_INVALID_ARG, "n < 0");
  if (k == 0 || n == 0) return GP_OK;
  CHK(check_mat(ctx, "X", X, n, d, d));
  if (!L || !piv) return fail(ctx, GP_ERR_INVALID_ARG, "L or piv is NULL");
  if (ldl < n) return fail(ctx, GP_ERR_INVALID_ARG, "ldl %lld < n %lld", (long long)ldl,
                           (long long)n);
  HIPCHK(hipSetDevice(ctx->device));
  return pc_construct(ctx, X, n, d, theta, (int)std::min<int64_t>(k, n), L, nullptr, ldl, piv,
                      rank);
}

int gp_prior_sample(gp_ctx* ctx, const float* Xq, int64_t m_rows, int d, const double* theta,
                    const float* t, int M, const float* W, int64_t ldw, int s, float* F,
                    int64_t ldf) {
  if (!ctx) return GP_ERR_INVALID_ARG;
  ctx->err.clear();
  CHK(check_dims(ctx, d, 0));
  CHK(check_theta(ctx, theta, d));
  if (M < 1) return fail(ctx, GP_ERR_INVALID_ARG, "M = %d must be >= 1", M);
  if (s < 0) return fail(ctx, GP_ERR_INVALID_ARG, "s must be >= 0");
  CHK(check_mat(ctx, "Xq", Xq, m_rows, d, d));
  CHK(check_mat(ctx, "t", t, M, d, d));
  CHK(check_mat(ctx, "W", W, 2 * (int64_t)M, ldw, s));
  CHK(check_mat(ctx, "F", F, m_rows, ldf, s));
  HIPCHK(hipSetDevice(ctx->device));
  if (m_rows == 0 || s == 0) return GP_OK;
  double *om, *inv;
  CHK(ensure(ctx, B_OMEGA, (size_t)M * d, &om));
  CHK(ensure(ctx, B_INVELL, (size_t)kMaxD, &inv));
  CHK(ensure_pinned(ctx, kMaxD));
  for (int k = 0; k < d; ++k) ctx->hpin[k] = 1.0 / theta[k];
  HIPCHK(hipMemcpyAsync(inv, ctx->hpin, d * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(rff_omega(t, M, d, inv, om, ctx->stream));
  RffArgs ra;
  ra.D = select_D(d);
  ra.x = Xq;
  ra.d = d;
  ra.m = m_rows;
  ra.omega = om;
  ra.M = M;
  ra.W = W;
  ra.ldw = ldw;
  ra.s = s;
  ra.amp = (float)(theta[d] / std::sqrt((double)M));
  ra.F = F;
  ra.ldf = ldf;
  {
    ProfScope ps(ctx, 2);
    HIPCHK(rff(ra, ctx->stream));
  }
  // the pinned buffer held inv_ell for the copy above: wait before it is reused
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return GP_OK;
}

int gp_posterior_sample(gp_ctx* ctx, const float* Xq, int64_t m_rows, const float* X, int64_t n,
                        int d, const double* theta, const float* t, int M, const float* W,
                        int64_t ldw, const float* U, int64_t ldu, int s, int precision, float* F,
                        int64_t ldf) {
  if (!ctx) return GP_ERR_INVALID_ARG;
  ctx->err.clear();
  CHK(check_prec(ctx, precision));
  CHK(check_dims(ctx, d, s));
  CHK(check_mat(ctx, "X", X, n, d, d));
  CHK(check_mat(ctx, "U", U, n, ldu, s + 1));
  CHK(gp_prior_sample(ctx, Xq, m_rows, d, theta, t, M, W, ldw, s, F, ldf));
  if (m_rows == 0 || s == 0 || n == 0) return GP_OK;
  float* Dd;
  CHK(ensure(ctx, B_POSTD, (size_t)n * s, &Dd));
  HIPCHK(post_diff(U, ldu, n, s, Dd, ctx->stream));
  Packed pq, px;
  CHK(pack_points(ctx, B_XP1, Xq, nullptr, m_rows, d, theta, &pq));
  CHK(pack_points(ctx, B_XP2, X, nullptr, n, d, theta, &px));
  // F = a^2 K(Xq, X) D + 1 * F  (the prior samples enter through the epilogue's added term)
  return kprod(ctx, pq, px, Dd, s, s, F, ldf, precision, a2_of(theta, d), F, ldf, 1.0f);
}

int gp_mll_grad(gp_ctx* ctx, const float* X, int64_t n, int d, const float* y,
                const double* theta, int estimator, int s, const float* Z, int64_t ldz,
                const float* rff_t, int M, const float* rff_W, int64_t ldw, const float* w_eps,
                int64_t ldeps, float* U, int64_t ldu, const gp_solver_cfg* cfg, int adjoint_mode,
                double* grad_out, gp_solve_stats* stats) {
  if (!ctx) return GP_ERR_INVALID_ARG;
  ctx->err.clear();
  if (!cfg) return fail(ctx, GP_ERR_INVALID_ARG, "cfg is NULL");
  if (!grad_out) return fail(ctx, GP_ERR_INVALID_ARG, "grad_out is NULL");
  if (s < 1) return fail(ctx, GP_ERR_INVALID_ARG, "s = %d must be >= 1", s);
  const int c = s + 1;
  CHK(check_dims(ctx, d, c, kMaxSolveC));
  CHK(check_theta(ctx, theta, d));
  CHK(check_mat(ctx, "X", X, n, d, d));
  CHK(check_mat(ctx, "y", y, n, 1, 1));
  CHK(check_mat(ctx, "U", U, n, ldu, c));
  if (estimator == GP_STANDARD) {
    CHK(check_mat(ctx, "Z", Z, n, ldz, s));
  } else if (estimator == GP_PATHWISE) {
    if (M < 1) return fail(ctx, GP_ERR_INVALID_ARG, "M = %d must be >= 1", M);
    CHK(check_mat(ctx, "rff_t", rff_t, M, d, d));
    CHK(check_mat(ctx, "rff_W", rff_W, 2 * (int64_t)M, ldw, s));
    CHK(check_mat(ctx, "w_eps", w_eps, n, ldeps, s));
  } else {
    return fail(ctx, GP_ERR_INVALID_ARG, "unknown estimator %d", estimator);
  }
  HIPCHK(hipSetDevice(ctx->device));
  for (int k = 0; k < d + 2; ++k) grad_out[k] = 0.0;
  if (n == 0) return GP_OK;

  // Right-hand sides B = [y, z_1..z_s] or [y, xi_1..xi_s].
  float* Bm;
  CHK(ensure(ctx, B_RHS, (size_t)n * c, &Bm));
  HIPCHK(set_col(y, n, Bm, c, 0, ctx->stream));
  if (estimator == GP_STANDARD) {
    HIPCHK(copy_cols(Z, ldz, n, s, Bm + 1, c, ctx->stream));
  } else {
    double *om, *inv;
    CHK(ensure(ctx, B_OMEGA, (size_t)M * d, &om));
    CHK(ensure(ctx, B_INVELL, (size_t)kMaxD, &inv));
    CHK(ensure_pinned(ctx, kMaxD));
    for (int k = 0; k < d; ++k) ctx->hpin[k] = 1.0 / theta[k];
    HIPCHK(hipMemcpyAsync(inv, ctx->hpin, d * sizeof(double), hipMemcpyHostToDevice,
                          ctx->stream));
    HIPCHK(rff_omega(rff_t, M, d, inv, om, ctx->stream));
    RffArgs ra;
    ra.D = select_D(d);
    ra.x = X;
    ra.d = d;
    ra.m = n;
    ra.omega = om;
    ra.M = M;
    ra.W = rff_W;
    ra.ldw = ldw;
    ra.s = s;
    ra.amp = (float)(theta[d] / std::sqrt((double)M));
    ra.F = Bm;
    ra.ldf = c;
    ra.f_col0 = 1;
    ra.weps = w_eps;
    ra.ldeps = ldeps;
    ra.sigma = (float)theta[d + 1];
    {
      ProfScope ps(ctx, 2);
      HIPCHK(rff(ra, ctx->stream));
    }
    HIPCHK(hipStreamSynchronize(ctx->stream));
  }
  // Solve H U = B (warm start: U holds the previous solution on entry).
  CHK(gp_solve(ctx, X, n, d, theta, Bm, c, U, ldu, c, cfg, stats));
  // Gradient: g_k = sum_c w_c U_c^T dH_k W_c, w = (1/2, -1/(2s), ...).
  std::vector<double> w(c, -1.0 / (2.0 * s));
  w[0] = 0.5;
  const float* W = U;
  int64_t ldW = ldu;
  if (estimator == GP_STANDARD) {
    float* Wb;
    CHK(ensure(ctx, B_WB, (size_t)n * c, &Wb));
    HIPCHK(copy_cols(U, ldu, n, 1, Wb, c, ctx->stream));
    HIPCHK(copy_cols(Z, ldz, n, s, Wb + 1, c, ctx->stream));
    W = Wb;
    ldW = c;
  }
  const int adj_prec = cfg->precision == GP_FP32 ? GP_FP32 : GP_BF16X3;
  return gp_kmatvec_adjoint(ctx, X, n, d, theta, U, ldu, W, ldW, c, w.data(), adj_prec,
                            adjoint_mode, grad_out);
}

int gp_nu_to_theta(int p, const double* nu, int transform, double* theta) {
  if (p < 0 || (p > 0 && (!nu || !theta))) return GP_ERR_INVALID_ARG;
  if (transform != GP_SOFTPLUS && transform != GP_LOG) return GP_ERR_INVALID_ARG;
  for (int k = 0; k < p; ++k) {
    const double v = nu[k];
    theta[k] = transform == GP_LOG ? std::exp(v)
                                   : (v > 0 ? v + std::log1p(std::exp(-v)) : std::log1p(std::exp(v)));
  }
  return GP_OK;
}

int gp_theta_to_nu(int p, const double* theta, int transform, double* nu) {
  if (p < 0 || (p > 0 && (!nu || !theta))) return GP_ERR_INVALID_ARG;
  if (transform != GP_SOFTPLUS && transform != GP_LOG) return GP_ERR_INVALID_ARG;
  for (int k = 0; k < p; ++k)
    if (!(theta[k] > 0.0) || !std::isfinite(theta[k])) return GP_ERR_INVALID_ARG;
  for (int k = 0; k < p; ++k) {
    const double t = theta[k];
    // softplus^-1(t) = log(e^t - 1) = t + log(1 - e^-t)
    nu[k] = transform == GP_LOG ? std::log(t) : t + std::log(-std::expm1(-t));
  }
  return GP_OK;
}

int gp_adam_ascent(int p, double* nu, double* m, double* v, int64_t* step,
                   const double* grad_theta, double lr, int transform) {
  if (p < 0 || (p > 0 && (!nu || !m || !v || !grad_theta)) || !step) return GP_ERR_INVALID_ARG;
  if (transform != GP_SOFTPLUS && transform != GP_LOG) return GP_ERR_INVALID_ARG;
  const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
  const int64_t t = ++(*step);
  const double c1 = 1.0 - std::pow(b1, (double)t);
  const double c2 = 1.0 - std::pow(b2, (double)t);
  for (int k = 0; k < p; ++k) {
    const double x = nu[k];
    double dth;
    if (transform == GP_LOG) {
      dth = std::exp(x);
    } else {
      const double e = std::exp(-std::fabs(x));
      dth = x >= 0 ? 1.0 / (1.0 + e) : e / (1.0 + e);
    }
    const double g = grad_theta[k] * dth;
    m[k] = b1 * m[k] + (1.0 - b1) * g;
    v[k] = b2 * v[k] + (1.0 - b2) * g * g;
    nu[k] = x + lr * (m[k] / c1) / (std::sqrt(v[k] / c2) + eps);
  }
  return GP_OK;
}

}  // extern "C"

namespace {

int solve_dispatch(gp_ctx* ctx, const Packed& px, const float* X, const double* theta, int d,
                   const float* B, int64_t ldb, float* U, int64_t ldu, int c,
                   const gp_solver_cfg& cfg, gp_solve_stats& stats) {
  SolveState s;
  CHK(solve_setup(ctx, B, ldb, U, ldu, px.n, c, s));
  switch (cfg.solver) {
    case GP_CG:
      CHK(cg_solve(ctx, px, X, theta, d, s, cfg, stats));
      break;
    case GP_AP:
      CHK(ap_solve(ctx, px, X, theta, d, s, cfg, stats));
      break;
    case GP_SGD:
      CHK(sgd_solve(ctx, px, X, theta, d, s, cfg, stats));
      break;
    default:
      return fail(ctx, GP_ERR_INVALID_ARG, "solver %d not available", cfg.solver);
  }
  return solve_finish(ctx, s, U, ldu);
}

}  // namespace

// ------------------------------------------- initial-hyperparameter heuristic
namespace {

struct ExactWs {
  double *A, *W, *xs, *ys, *diag, *v, *alpha, *part, *gpart, *out, *inv_ell;
  int* status;
  int64_t m, mp;
  int d;
};

// Workspace and the gathered rows (FP64) of one exact-likelihood subset.
int exact_prepare(gp_ctx* ctx, const float* X, int64_t n, int d, const float* y,
                  const int64_t* idx, int64_t m, ExactWs& ws) {
  ws.m = m;
  ws.d = d;
  ws.mp = round_up(m, kExactTile);
  const size_t mp = (size_t)ws.mp;
  CHK(ensure(ctx, B_EXA, mp * mp, &ws.A));
  CHK(ensure(ctx, B_EXW, mp * mp, &ws.W));
  CHK(ensure(ctx, B_EXXS, mp * d, &ws.xs));
  CHK(ensure(ctx, B_EXYS, mp, &ws.ys));
  CHK(ensure(ctx, B_EXDG, mp, &ws.diag));
  CHK(ensure(ctx, B_EXV, mp, &ws.v));
  CHK(ensure(ctx, B_EXAL, mp, &ws.alpha));
  CHK(ensure(ctx, B_EXPART, (size_t)exact_part_doubles(ws.mp), &ws.part));
  CHK(ensure(ctx, B_EXGP, (size_t)exact_gpart_doubles(ws.mp, d), &ws.gpart));
  CHK(ensure(ctx, B_EXOUT, (size_t)kMaxD + 4, &ws.out));
  CHK(ensure(ctx, B_EXIE, (size_t)kMaxD, &ws.inv_ell));
  CHK(ensure(ctx, B_EXST, 1, &ws.status));
  HIPCHK(hipMemsetAsync(ws.status, 0, sizeof(int), ctx->stream));
  HIPCHK(exact_gather(X, n, d, idx, m, ws.mp, y, ws.xs, ws.ys, ws.status, ctx->stream));
  return GP_OK;
}

// L and dL/dtheta at theta on the prepared subset (synchronises the stream).
int exact_run(gp_ctx* ctx, const ExactWs& ws, const double* theta, double* mll, double* grad) {
  const int d = ws.d;
  CHK(ensure_pinned(ctx, 2 * (size_t)kMaxD + 16));
  double* hin = ctx->hpin;
  double* hout = ctx->hpin + kMaxD;
  for (int k = 0; k < d; ++k) hin[k] = 1.0 / theta[k];
  HIPCHK(hipMemcpyAsync(ws.inv_ell, hin, d * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  if (!ctx->xstream) HIPCHK(hipStreamCreateWithFlags(&ctx->xstream, hipStreamNonBlocking));
  while ((int)ctx->xev.size() < exact_events(ws.mp)) {
    hipEvent_t e = nullptr;
    HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    ctx->xev.push_back(e);
  }
  {
    ProfScope ps(ctx, 7);
    HIPCHK(exact_factor(ws.xs, d, ws.m, ws.mp, ws.inv_ell, theta[d], theta[d + 1], ws.A, ws.W,
                        ws.diag, ws.status, ctx->stream, ctx->xstream, ctx->xev.data(),
                        (int)ctx->xev.size()));
  }
  {
    ProfScope ps(ctx, 8);
    HIPCHK(exact_finish(ws.xs, ws.ys, d, ws.m, ws.mp, ws.inv_ell, theta[d], theta[d + 1], ws.A,
                        ws.W, ws.diag, ws.v, ws.alpha, ws.part, ws.gpart, ws.out, ctx->stream));
  }
  HIPCHK(hipMemcpyAsync(hout, ws.out, (d + 4) * sizeof(double), hipMemcpyDeviceToHost,
                        ctx->stream));
  int* hst = reinterpret_cast<int*>(ctx->hpin + 2 * kMaxD + 8);
  HIPCHK(hipMemcpyAsync(hst, ws.status, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (*hst & 1) return fail(ctx, GP_ERR_INVALID_ARG, "a row index lies outside [0, n)");
  if (*hst & 2)
    return fail(ctx, GP_ERR_BREAKDOWN,
                "non-positive pivot in the Cholesky factorisation of H (m = %lld)",
                (long long)ws.m);
  if (mll) *mll = -0.5 * hout[0] - 0.5 * hout[1] - 0.5 * (double)ws.m * std::log(6.283185307179586477);
  if (grad)
    for (int k = 0; k < d + 2; ++k) grad[k] = hout[2 + k];
  return GP_OK;
}

int nearest_run(gp_ctx* ctx, const float* X, int64_t n, int d, int64_t centre, int64_t k,
                int64_t* idx) {
  if (k == 0) return GP_OK;
  uint64_t* key;
  SelState* st;
  int64_t* cnt;
  CHK(ensure(ctx, B_NRKEY, (size_t)n, &key));
  CHK(ensure(ctx, B_NRST, 1, &st));
  CHK(ensure(ctx, B_NRCNT, 2 * (size_t)nearest_blocks(n), &cnt));
  ProfScope ps(ctx, 6);
  HIPCHK(nearest(X, n, d, centre, k, key, st, cnt, idx, ctx->stream));
  return GP_OK;
}

int check_centre(gp_ctx* ctx, int64_t centre, int64_t n) {
  if (centre < 0 || centre >= n)
    return fail(ctx, GP_ERR_INVALID_ARG, "centre %lld outside [0, %lld)", (long long)centre,
                (long long)n);
  return GP_OK;
}

}  // namespace

extern "C" {

int gp_nearest(gp_ctx* ctx, const float* X, int64_t n, int d, int64_t centre, int64_t k,
               int64_t* idx) {
  if (!ctx) return GP_ERR_INVALID_ARG;
  ctx->err.clear();
  CHK(check_dims(ctx, d, 0));
  if (n < 0) return fail(ctx, GP_ERR_INVALID_ARG, "n < 0");
  if (k < 0 || k > n)
    return fail(ctx, GP_ERR_INVALID_ARG, "k = %lld outside [0, n = %lld]", (long long)k,
                (long long)n);
  if (k == 0) return GP_OK;
  CHK(check_centre(ctx, centre, n));
  CHK(check_mat(ctx, "X", X, n, d, d));
  if (!idx) return fail(ctx, GP_ERR_INVALID_ARG, "idx is NULL");
  HIPCHK(hipSetDevice(ctx->device));
  return nearest_run(ctx, X, n, d, centre, k, idx);
}

int gp_exact_mll(gp_ctx* ctx, const float* X, int64_t n, int d, const float* y,
                 const int64_t* idx, int64_t m, const double* theta, double* mll, double* grad) {
  if (!ctx) return GP_ERR_INVALID_ARG;
  ctx->err.clear();
  CHK(check_dims(ctx, d, 0));
  CHK(check_theta(ctx, theta, d));
  if (m < 1 || m > kExactMaxM)
    return fail(ctx, GP_ERR_INVALID_ARG, "m = %lld outside [1, %lld]", (long long)m,
                (long long)kExactMaxM);
  if (n < 1) return fail(ctx, GP_ERR_INVALID_ARG, "n < 1");
  if (!idx && m > n)
    return fail(ctx, GP_ERR_INVALID_ARG, "m = %lld > n = %lld without an index list",
                (long long)m, (long long)n);
  CHK(check_mat(ctx, "X", X, n, d, d));
  CHK(check_mat(ctx, "y", y, n, 1, 1));
  HIPCHK(hipSetDevice(ctx->device));
  ExactWs ws;
  CHK(exact_prepare(ctx, X, n, d, y, idx, m, ws));
  return exact_run(ctx, ws, theta, mll, grad);
}

void gp_init_cfg_default(gp_init_cfg* cfg) {
  if (!cfg) return;
  cfg->steps = 100;
  cfg->lr = 0.1;
  cfg->transform = GP_SOFTPLUS;
  cfg->theta0 = nullptr;
}

}  // extern "C"

namespace {

// One centroid subset of the heuristic: its own workspace, streams, dependency
// events and pinned staging, so the subsets' exact-likelihood evaluations run
// concurrently (the leaves and small GEMMs of one evaluation leave most of the
// chip idle).  Each lane issues exactly the kernels of the sequential path.
constexpr int kHeurLanes = 16;                    // concurrent subsets at most
constexpr int64_t kHeurLaneMemory = 64ll << 30;   // and their workspaces within 64 GiB

struct HeurLane {
  ExactWs ws{};
  int64_t* idx = nullptr;
  hipStream_t st = nullptr, side = nullptr;
  std::vector<hipEvent_t> ev;
  double* pin = nullptr;  // [0, kMaxD): 1/ell; [kMaxD, 2 kMaxD + 4): results; then status
  std::vector<void*> mem;
  std::vector<double> nu, mom, vel, th, g;
  int64_t step = 0;
};

struct LaneSet {
  std::vector<HeurLane> lanes;
  ~LaneSet() {
    for (auto& l : lanes) {
      if (l.st) (void)hipStreamSynchronize(l.st);
      if (l.side) (void)hipStreamSynchronize(l.side);
      for (auto e : l.ev) (void)hipEventDestroy(e);
      if (l.side) (void)hipStreamDestroy(l.side);
      if (l.st) (void)hipStreamDestroy(l.st);
      for (auto q : l.mem) (void)hipFree(q);
      if (l.pin) (void)hipHostFree(l.pin);
    }
  }
};

int64_t lane_bytes(int64_t m, int d) {
  const int64_t mp = round_up(m, kExactTile);
  return 8 * (2 * mp * mp + mp * (d + 5) + exact_part_doubles(mp) + exact_gpart_doubles(mp, d) +
              2 * kMaxD + 4) + 8 * m + 4096;
}

int lane_alloc(gp_ctx* ctx, HeurLane& l, int64_t m, int d) {
  auto dev = [&](size_t bytes, void** out) -> int {
    if (hipMalloc(out, std::max<size_t>(bytes, 256)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(ctx, GP_ERR_NO_WORKSPACE, "hipMalloc of %zu bytes for a heuristic lane failed",
                  bytes);
    }
    l.mem.push_back(*out);
    return GP_OK;
  };
  ExactWs& w = l.ws;
  w.m = m;
  w.d = d;
  w.mp = round_up(m, kExactTile);
  const size_t mp = (size_t)w.mp;
  CHK(dev(mp * mp * 8, (void**)&w.A));
  CHK(dev(mp * mp * 8, (void**)&w.W));
  CHK(dev(mp * d * 8, (void**)&w.xs));
  CHK(dev(mp * 8, (void**)&w.ys));
  CHK(dev(mp * 8, (void**)&w.diag));
  CHK(dev(mp * 8, (void**)&w.v));
  CHK(dev(mp * 8, (void**)&w.alpha));
  CHK(dev((size_t)exact_part_doubles(w.mp) * 8, (void**)&w.part));
  CHK(dev((size_t)exact_gpart_doubles(w.mp, d) * 8, (void**)&w.gpart));
  CHK(dev(((size_t)kMaxD + 4) * 8, (void**)&w.out));
  CHK(dev((size_t)kMaxD * 8, (void**)&w.inv_ell));
  CHK(dev(sizeof(int), (void**)&w.status));
  CHK(dev((size_t)m * 8, (void**)&l.idx));
  HIPCHK(hipHostMalloc((void**)&l.pin, (2 * kMaxD + 16) * sizeof(double), hipHostMallocDefault));
  HIPCHK(hipStreamCreateWithFlags(&l.st, hipStreamNonBlocking));
  HIPCHK(hipStreamCreateWithFlags(&l.side, hipStreamNonBlocking));
  l.ev.resize(exact_events(w.mp), nullptr);
  for (auto& e : l.ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  return GP_OK;
}

// Enqueue one evaluation of lane l at its current theta (results land in l.pin).
int lane_issue(gp_ctx* ctx, HeurLane& l) {
  const ExactWs& w = l.ws;
  const int d = w.d;
  for (int k = 0; k < d; ++k) l.pin[k] = 1.0 / l.th[k];
  HIPCHK(hipMemcpyAsync(w.inv_ell, l.pin, d * sizeof(double), hipMemcpyHostToDevice, l.st));
  HIPCHK(exact_factor(w.xs, d, w.m, w.mp, w.inv_ell, l.th[d], l.th[d + 1], w.A, w.W, w.diag,
                      w.status, l.st, l.side, l.ev.data(), (int)l.ev.size()));
  HIPCHK(exact_finish(w.xs, w.ys, d, w.m, w.mp, w.inv_ell, l.th[d], l.th[d + 1], w.A, w.W, w.diag,
                      w.v, w.alpha, w.part, w.gpart, w.out, l.st));
  HIPCHK(hipMemcpyAsync(l.pin + kMaxD, w.out, (d + 4) * sizeof(double), hipMemcpyDeviceToHost,
                        l.st));
  HIPCHK(hipMemcpyAsync(l.pin + 2 * kMaxD + 8, w.status, sizeof(int), hipMemcpyDeviceToHost, l.st));
  return GP_OK;
}

}  // namespace

extern "C" {

int gp_init_heuristic(gp_ctx* ctx, const float* X, int64_t n, int d, const float* y,
                      const int64_t* centres, int nc, int64_t m, const gp_init_cfg* cfg_in,
                      double* theta_out, double* theta_each) {
  if (!ctx) return GP_ERR_INVALID_ARG;
  ctx->err.clear();
  gp_init_cfg cfg;
  gp_init_cfg_default(&cfg);
  if (cfg_in) cfg = *cfg_in;
  CHK(check_dims(ctx, d, 0));
  if (nc < 1 || !centres) return fail(ctx, GP_ERR_INVALID_ARG, "need nc >= 1 centre rows");
  if (!theta_out) return fail(ctx, GP_ERR_INVALID_ARG, "theta_out is NULL");
  if (m < 1 || m > n || m > kExactMaxM)
    return fail(ctx, GP_ERR_INVALID_ARG, "m = %lld outside [1, min(n, %lld)]", (long long)m,
                (long long)kExactMaxM);
  if (cfg.steps < 0 || !(cfg.lr > 0.0) || !std::isfinite(cfg.lr))
    return fail(ctx, GP_ERR_INVALID_ARG, "steps must be >= 0 and lr > 0");
  if (cfg.transform != GP_SOFTPLUS && cfg.transform != GP_LOG)
    return fail(ctx, GP_ERR_INVALID_ARG, "unknown transform %d", cfg.transform);
  if (cfg.theta0) CHK(check_theta(ctx, cfg.theta0, d));
  for (int c = 0; c < nc; ++c) CHK(check_centre(ctx, centres[c], n));
  CHK(check_mat(ctx, "X", X, n, d, d));
  CHK(check_mat(ctx, "y", y, n, 1, 1));
  HIPCHK(hipSetDevice(ctx->device));
  const int p = d + 2;
  // concurrent lanes: at most kHeurLanes, and within kHeurLaneMemory of device memory
  const int64_t per = lane_bytes(m, d);
  const int group = (int)std::max<int64_t>(
      1, std::min<int64_t>({(int64_t)nc, (int64_t)kHeurLanes, kHeurLaneMemory / per}));
  std::vector<double> sum(p, 0.0);
  Progress pr;
  for (int c0 = 0; c0 < nc; c0 += group) {
    const int cn = std::min(group, nc - c0);
    LaneSet set;
    set.lanes.resize(cn);
    for (int q = 0; q < cn; ++q) {
      HeurLane& l = set.lanes[q];
      CHK(lane_alloc(ctx, l, m, d));
      // steps 1-2 on the context's stream: nearest rows, gathered subset
      CHK(nearest_run(ctx, X, n, d, centres[c0 + q], m, l.idx));
      HIPCHK(hipMemsetAsync(l.ws.status, 0, sizeof(int), ctx->stream));
      HIPCHK(exact_gather(X, n, d, l.idx, m, l.ws.mp, y, l.ws.xs, l.ws.ys, l.ws.status,
                          ctx->stream));
      l.nu.resize(p);
      l.mom.assign(p, 0.0);
      l.vel.assign(p, 0.0);
      l.th.resize(p);
      l.g.resize(p);
      for (int k = 0; k < p; ++k) {
        const double t0 = cfg.theta0 ? cfg.theta0[k] : 1.0;
        gp_theta_to_nu(1, &t0, cfg.transform, &l.nu[k]);
      }
    }
    HIPCHK(hipStreamSynchronize(ctx->stream));
    // step 3: Adam on the exact likelihood, all lanes of the group in lockstep
    for (int it = 0; it < cfg.steps; ++it) {
      for (auto& l : set.lanes) {
        gp_nu_to_theta(p, l.nu.data(), cfg.transform, l.th.data());
        CHK(lane_issue(ctx, l));
      }
      for (int q = 0; q < cn; ++q) {
        HeurLane& l = set.lanes[q];
        HIPCHK(hipStreamSynchronize(l.st));
        int stv;
        std::memcpy(&stv, l.pin + 2 * kMaxD + 8, sizeof(int));
        if (stv & 1) return fail(ctx, GP_ERR_INVALID_ARG, "a row index lies outside [0, n)");
        if (stv & 2)
          return fail(ctx, GP_ERR_BREAKDOWN,
                      "non-positive pivot in the Cholesky factorisation of H (centre %d)",
                      c0 + q);
        for (int k = 0; k < p; ++k) l.g[k] = l.pin[kMaxD + 2 + k];
        gp_adam_ascent(p, l.nu.data(), l.mom.data(), l.vel.data(), &l.step, l.g.data(), cfg.lr,
                       cfg.transform);
      }
    }
    for (int q = 0; q < cn; ++q) {
      HeurLane& l = set.lanes[q];
      gp_nu_to_theta(p, l.nu.data(), cfg.transform, l.th.data());
      for (int k = 0; k < p; ++k) {
        if (!std::isfinite(l.th[k]) || !(l.th[k] > 0.0))
          return fail(ctx, GP_ERR_NONFINITE,
                      "theta[%d] = %g after the maximisation for centre %d", k, l.th[k], c0 + q);
        sum[k] += l.th[k];
        if (theta_each) theta_each[(int64_t)(c0 + q) * p + k] = l.th[k];
      }
    }
    pr.count("init heuristic: centres done", c0 + cn, nc);
  }
  for (int k = 0; k < p; ++k) theta_out[k] = sum[k] / nc;
  return GP_OK;
}

}  // extern "C"
