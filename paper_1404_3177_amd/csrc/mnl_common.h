// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/mnl.h"

namespace mnl {

constexpr int kWave = 64;

// Copy n elements with nthr threads keeping U loads in flight per thread:
// all U loads of a batch are issued before any store, so a staging loop is
// not one memory latency per element.  ld(e) returns element e, st(e, v)
// stores it.
template <int U, typename Load, typename Store>
__device__ inline void batched_copy(int n, int tid, int nthr, Load ld,
                                    Store st) {
  for (int base = 0; base < n; base += U * nthr) {
    decltype(ld(0)) v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = base + tid + u * nthr;
      if (e < n) v[u] = ld(e);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = base + tid + u * nthr;
      if (e < n) st(e, v[u]);
    }
  }
}

// Asynchronous copy of n dwords from global memory to LDS by one wave: each
// instruction moves 64 consecutive dwords straight into LDS (no registers);
// the copy has landed after s_waitcnt vmcnt(0) (which __syncthreads
// includes).  src: 4-byte aligned; dst: LDS, 4-byte aligned.
typedef __attribute__((address_space(3))) void lds_void_t;
__device__ inline void wave_copy_lds(const void *src, void *dst, int n,
                                     int lane) {
  const uint32_t *s = static_cast<const uint32_t *>(src);
  char *dc = static_cast<char *>(dst);
  for (int c = 0; c < n; c += 64) {
    if (c + lane < n)
      __builtin_amdgcn_global_load_lds(s + c + lane,
                                       (lds_void_t *)(dc + 4 * c), 4, 0, 0);
  }
}

// Dimensions of a problem, validated.
struct Dims {
  int64_t N;
  int K, p, g, a;
  int64_t np;      // number of coefficients (Eq. 8)
  __host__ __device__ int64_t off_gamma() const { return int64_t(K - 1) * p; }
  __host__ __device__ int64_t off_alpha() const { return int64_t(K - 1) * p + int64_t(K) * a; }
};

// Device workspace: one growing allocation per named slot.
struct Buf {
  void *ptr = nullptr;
  size_t bytes = 0;
};

struct Ctx;

// Error helpers ---------------------------------------------------------------
int set_error(Ctx *c, int code, const char *fmt, ...);

#define MNL_HIP(ctx, call)                                                    \
  do {                                                                        \
    hipError_t _e = (call);                                                   \
    if (_e != hipSuccess)                                                     \
      return ::mnl::set_error((ctx), MNL_ERR_HIP, "%s failed: %s", #call,      \
                              hipGetErrorString(_e));                         \
  } while (0)

#define MNL_TRY(expr)                                                         \
  do {                                                                        \
    int _r = (expr);                                                          \
    if (_r != MNL_OK) return _r;                                              \
  } while (0)

// ---- fused pass (utility, probabilities, log-likelihood, gradient) ---------
struct PassPlan {
  int tb;            // observations per tile
  int grid;          // workgroups (fixed by the shape: deterministic sums)
  int ntw;           // beta-gradient MFMA tiles per wave (power of two)
  int cap;           // register slots for one alternative's z / y values
  int yl;            // 1: y rows staged through LDS one observation ahead
  size_t lds_bytes;
  int64_t stride;    // doubles per workgroup partial row
};

// Per-workgroup partial row layout: [0] loglik, [1 .. np] gradient.
int pass_plan(const Dims &d, PassPlan *plan);

struct PassArgs {
  Dims d;
  const double *X, *Y, *Z, *w;
  const int32_t *choice;
  const double *theta;
  double *P;         // [N][K] f64 or null
  float *P32;        // [N][K] f32 or null
  double *Ybar;      // [N][g] or null
  double *partial;   // [grid][stride]
  // Hessian-vector mode when set: P [N][K] at the current theta, theta
  // then holds v and the gradient rows sum to H v (l, P, Ybar not formed)
  const double *Pin = nullptr;
};

hipError_t launch_pass(const PassPlan &plan, const PassArgs &a,
                       hipStream_t s);
// Sum the partial rows in a fixed order: out[0] = loglik, out[1..] = grad.
hipError_t launch_pass_reduce(const PassPlan &plan, const double *partial,
                              double *loglik, double *grad, int64_t np,
                              hipStream_t s);

// ---- small vector kernels ----------------------------------------------------
// out = x + t * d
hipError_t launch_axpy(const double *x, const double *d, double t, double *out,
                       int64_t n, hipStream_t s);
// out[0] = sum(x^2) in a fixed order (single workgroup)
// out[0..2] = status[0] (0 if status is NULL), lg[0], sum of lg[1..n]^2
hipError_t launch_scalars(const double *lg, int64_t n, const int32_t *status,
                          double *out, hipStream_t s);
hipError_t launch_sumsq(const double *x, int64_t n, double *out,
                        hipStream_t s);
// Truncated CG on (-H) d = g (single workgroup each): init sets d = 0,
// r = p = g, scal[0] = g.g; update takes Hp = H p and does one step,
// scal[0] = r.r after it, scal[1] = p.(-H p) (no step when <= 0).
hipError_t launch_cg_init(const double *g, double *d, double *r, double *p,
                          int64_t n, double *scal, hipStream_t s);
hipError_t launch_cg_update(const double *Hp, double *d, double *r, double *p,
                            int64_t n, double *scal, hipStream_t s);
// Flags [0]: choice out of range count, [1]: non-finite data count.
hipError_t launch_validate(const Dims &d, const double *X, const double *Y,
                           const double *Z, const double *w,
                           const int32_t *choice, int32_t *flags,
                           hipStream_t s);

// ---- Hessian -------------------------------------------------------------------
struct HessPlan;
struct HessArgs {
  Dims d;
  const double *X, *Y, *Z, *w;
  const double *P;      // [N][K] f64
  const float *P32;     // [N][K] f32 (mixed precision)
  const double *Ybar;   // [N][g]
  double *H;            // [np][np] output (Hessian sign)
  int prec;
};
int hessian_run(Ctx *c, const HessArgs &a, hipStream_t s);
void hessian_cache_free(Ctx *c);
// Beta-beta blocks of H (k_bb.hip): written into a.H; the kernel is timed
// by the context's Hessian events.
int bb_run(Ctx *c, const HessArgs &a, hipStream_t s);
// Workspace (P blocks, split partials, chi operand) and table bytes of
// bb_run for a shape.
int bb_footprint(Ctx *c, const Dims &d, int prec, size_t *ws_bytes,
                 size_t *table_bytes);
void bb_cache_free(Ctx *c);
// Compute units of the context's device (256 when it cannot be queried).
int device_cus(Ctx *c);
// The context's library BLAS handle (rocBLAS, atomics off), bound to
// stream s; created on first use.
int blas_get(Ctx *c, hipStream_t s, void **handle);
// Destroy the context's library BLAS handle.
void blas_release(Ctx *c);
// Destroy the context's timing events.
void events_release(Ctx *c);
// Device bytes hessian_run takes for a shape: split partials (workspace
// slot S_HPART) and tile tables.
int hessian_footprint(Ctx *c, const Dims &d, int prec, size_t *part_bytes,
                      size_t *table_bytes);

// ---- Cholesky and solves ------------------------------------------------------
// Factor A = -H in place (lower triangle holds L) and solve L L^T delta = g;
// A has n + 1 + extra rows of n plus 64 doubles of padding (row n is
// scratch for g, NULL g reads as zeros; NULL delta skips the solve).
// extra = n appends identity rows that end up holding L^{-T} D^{-1}.
// info[0] receives 0 or (1 + index of the failed pivot).
int chol_solve_run(Ctx *c, double *A, int64_t n, const double *g,
                   double *delta, int32_t *info, hipStream_t s,
                   int64_t extra = 0);
// Scratch bytes chol_solve_run takes (workspace slot S_CHOL).
size_t chol_workspace_bytes(int64_t n, int64_t extra = 0);
// se_i = sqrt(diag((-H)^{-1})_i) from a factor with identity rows; z and
// pval (optional) the Wald statistic theta_i / se_i and its two-sided
// normal p-value.  Nothing is written when info[0] != 0.
hipError_t launch_inv_diag(const double *A, int64_t n, const double *theta,
                           double *se, double *z, double *pval,
                           const int32_t *info, hipStream_t s);
// V[a][b] = ((-H)^{-1})[idx[a]][idx[b]] (device idx [s], V [s][s]) from a
// factor with identity rows.
hipError_t launch_cov_sub(const double *A, int64_t n, const int32_t *idx,
                          int s, double *V, const int32_t *info,
                          hipStream_t st);
// out[0..n^2) = sgn (A - B) (B may be NULL), out[n^2 .. n^2 + n) = x - x0
// (x0 may be NULL): the matrix and g rows of a factorisation buffer.
hipError_t launch_signed_copy(const double *A, const double *B,
                              const double *x, const double *x0, double sgn,
                              int64_t n, double *out, hipStream_t s);
// out[0] = sum_k D_k y_k^2 over the factor's g row: x^T A^{-1} x when x
// was the g row of A's factorisation (0 when info[0] != 0).
hipError_t launch_quad(const double *A, int64_t n, double *out,
                       const int32_t *info, hipStream_t s);

// ---- collinearity check -------------------------------------------------------
// Keep flags (host int32, 1 = keep) of the X, Y and Z variables: column-order
// selection at tolerance tol on X, each Z_k (a Z variable must pass for every
// k) and the differenced generic data stacked over alternatives.
// Synchronises s.
int collinear_run(Ctx *c, const Dims &d, const mnl_problem *pr, double tol,
                  int32_t *keep_x, int32_t *keep_y, int32_t *keep_z,
                  hipStream_t s);
// Copies of X, Y, Z with only the kept columns (device outputs).
int select_columns_run(Ctx *c, const Dims &d, const mnl_problem *pr,
                       const int32_t *keep_x, const int32_t *keep_y,
                       const int32_t *keep_z, double *X_out, double *Y_out,
                       double *Z_out, hipStream_t s);

// ---- batched small fits (k_small.hip) ---------------------------------------
// Whether one workgroup can hold a fit of this shape (LDS and register
// limits of k_fit_small).
bool small_fit_shape_ok(const Dims &d);
// Fit nfits problems (device data) with one persistent kernel; opts may be
// NULL (defaults), else nfits entries, each FP64 Newton without validation.
// Synchronises s.
int small_fit_run(Ctx *c, int nfits, const mnl_problem *probs,
                  const double *const *theta0, const mnl_fit_opts *opts,
                  double *const *theta_out, mnl_fit_info *infos,
                  hipStream_t s);
// Whether the server runs a fit of this shape and options through
// small_fit_run (mnl_batch_eligible).
bool batch_eligible(const Dims &d, const mnl_fit_opts &o);
// Workspace bytes (slot S_BATCH) of a batch of nfits fits.
size_t small_fit_workspace_bytes(int nfits);

// Context ---------------------------------------------------------------------
struct Ctx {
  int device = 0;
  std::string last_error;
  std::vector<Buf> bufs;
  size_t total_bytes = 0;
  size_t ws_cap = 0;   // most bytes the workspace may hold (0: no cap)
  // HIP events bracketing the Hessian MFMA kernel and the fused pass
  // kernel on the caller's stream (read after the driver's next sync)
  hipEvent_t ev_h0 = nullptr, ev_h1 = nullptr, ev_p0 = nullptr,
             ev_p1 = nullptr;
  hipEvent_t ev_q[4] = {nullptr, nullptr, nullptr, nullptr};  // phases
  bool ev_ready = false;
  // captured Newton steps of the current fit, one per parity of the
  // alternating P / gradient buffers, and the page-locked host scalars
  // their last copy writes
  hipGraphExec_t step_exec[2] = {nullptr, nullptr};
  double *pinned = nullptr;
  // a step is being captured: nothing may allocate (an allocation would be
  // recorded into the graph instead of happening)
  bool capturing = false;
  bool hess_pending = false, pass_pending = false;
  // host-side caches of Hessian tile tables (keyed by shape)
  void *hess_cache = nullptr;
  void *bb_cache = nullptr;
  // stream-ordered mode (server slots): device memory comes from `pool`,
  // allocated and freed in the order of `ostream`, the only stream the
  // context's work runs on
  hipMemPool_t pool = nullptr;
  hipStream_t ostream = nullptr;
  int ncu = 0;   // compute units of `device` (0: not queried yet)
  // library GEMM handle (rocBLAS), created on first use
  void *blas = nullptr;
  // the beta-beta operand chi = x_a x_b (k_bb.hip), valid within one call
  // epoch (one top-level API call: a fit reuses it across its Hessians);
  // [0]: FP64 (workspace slot S_XX), [1]: FP32 / BF16 (slot S_XX_LP).  A
  // mixed-precision fit's FP64 retries keep their own copy, so a captured
  // mixed step never reads an operand of the other type
  uint64_t call_epoch = 0;
  struct XXState {
    uint64_t epoch = ~uint64_t(0);
    const double *X = nullptr, *w = nullptr;
    const void *buf = nullptr;
    int64_t N = 0;
    int p = 0, prec = -1;
  } xx[2];
};

// Raise a kernel's dynamic-LDS limit on the current device to at least
// `bytes`.  The limit only grows, so launches from several host threads
// never see it lowered under them.
hipError_t raise_lds_limit(const void *kernel, int bytes);

// Validate a problem description and fill its dimensions.
// (choices may be NULL when need_choice is false: the pass then reads
// alternative 0 for every observation and its l and g are meaningless)
int check_problem(Ctx *c, const mnl_problem *pr, Dims *d,
                  bool need_choice = true);
int check_opts(Ctx *c, const mnl_fit_opts *o);
// Newton-Raphson loop on device data (theta in/out on the device).
int fit_impl(Ctx *c, const mnl_problem *prob, double *theta,
             const mnl_fit_opts &o, mnl_fit_info *info, bool one_step,
             hipStream_t s);
// Upper bound of the device bytes a fit of this shape allocates in its
// context (workspace and tables; not the caller's data).
int fit_workspace_footprint(Ctx *c, const Dims &d, int prec, size_t *bytes);
// Free the context's workspace and tables (stream-ordered in pool mode).
void ctx_release(Ctx *c);
double now_ms();

// Workspace slots
enum Slot {
  S_PARTIAL = 0,   // pass partial rows
  S_LG,            // [0] loglik, [1..np] grad (current)
  S_LG_TRIAL,      // same for the line-search trial
  S_P,             // P f64 [N][K] (current theta)
  S_P_TRIAL,       // P f64 for the trial
  S_P32,           // P f32
  S_P32_TRIAL,
  S_YBAR,          // Ybar [N][g]
  S_YBAR_TRIAL,
  S_H,             // Hessian / Cholesky factor [np][np]
  S_DELTA,         // Newton direction [np]
  S_THETA_TRIAL,   // trial theta [np]
  S_SCAL,          // scalars (norms, flags)
  S_HPART,         // Hessian split-K partials
  S_HTAB,          // Hessian tile tables
  S_CHOL,          // Cholesky scratch
  S_THETA0,        // zero start
  S_XX,            // chi = x_a x_b operand of the beta-beta product, FP64
  S_XX_LP,         // the same in FP32 / BF16
  S_PT,            // P by observation blocks (beta-beta)
  S_BBPART,        // beta-beta split partials
  S_CG,            // inexact Newton: r, p, H p [np] each, scalars
  S_COLLIN,        // collinearity check: Gram matrices, masks, indices
  S_BATCH,         // batched small fits: descriptors, options, reports
  S_NSLOTS
};

int ws_get(Ctx *c, int slot, size_t bytes, void **ptr);

}  // namespace mnl
