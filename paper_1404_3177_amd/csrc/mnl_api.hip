// C ABI entry points and the Newton-Raphson driver (Sec. 3.1).
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <utility>

#include <rocblas/rocblas.h>

#include "mnl_common.h"

struct mnl_ctx {
  mnl::Ctx c;
};

namespace mnl {

int set_error(Ctx *c, int code, const char *fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->last_error = buf;
  }
  return code;
}

void graphs_release(Ctx *c);

int ws_get(Ctx *c, int slot, size_t bytes, void **ptr) {
  if (bytes == 0) bytes = 256;
  bytes = (bytes + 255) & ~size_t(255);
  Buf &b = c->bufs[slot];
  if (b.bytes < bytes) {
    if (c->capturing)
      return set_error(c, MNL_ERR_HIP, "workspace growth inside a capture");
    if (c->ws_cap && c->total_bytes - b.bytes + bytes > c->ws_cap)
      return set_error(c, MNL_ERR_OOM,
                       "workspace of %zu bytes would exceed the context's "
                       "cap of %zu bytes",
                       c->total_bytes - b.bytes + bytes, c->ws_cap);
    // captured steps hold the workspace's addresses: a buffer that moves
    // (a mixed-precision fit's FP64 retry grows the Hessian partials, for
    // one) makes them stale, so they are dropped and captured again
    graphs_release(c);
    if (b.ptr) {
      if (c->pool) {
        // stream-ordered: later work on ostream cannot see the old buffer
        MNL_HIP(c, hipFreeAsync(b.ptr, c->ostream));
      } else {
        // the old buffer may still be in use by enqueued work
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess)
          return set_error(c, MNL_ERR_HIP, "hipDeviceSynchronize: %s",
                           hipGetErrorString(e));
        (void)hipFree(b.ptr);
      }
      c->total_bytes -= b.bytes;
      b.ptr = nullptr;
      b.bytes = 0;
    }
    void *p = nullptr;
    const hipError_t e =
        c->pool ? hipMallocFromPoolAsync(&p, bytes, c->pool, c->ostream)
                : hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return set_error(c, MNL_ERR_OOM, "device allocation of %zu bytes failed",
                       bytes);
    }
    b.ptr = p;
    b.bytes = bytes;
    c->total_bytes += bytes;
  }
  *ptr = b.ptr;
  return MNL_OK;
}

void ctx_release(Ctx *c) {
  for (auto &b : c->bufs) {
    if (!b.ptr) continue;
    if (c->pool) (void)hipFreeAsync(b.ptr, c->ostream);
    else (void)hipFree(b.ptr);
    b.ptr = nullptr;
    b.bytes = 0;
  }
  c->total_bytes = 0;
  hessian_cache_free(c);
  bb_cache_free(c);
}

int blas_get(Ctx *c, hipStream_t s, void **handle) {
  if (!c->blas) {
    rocblas_handle hb;
    if (rocblas_create_handle(&hb) != rocblas_status_success)
      return set_error(c, MNL_ERR_HIP, "rocblas_create_handle failed");
    // no atomics: every library product is bitwise reproducible
    (void)rocblas_set_atomics_mode(hb, rocblas_atomics_not_allowed);
    c->blas = hb;
  }
  rocblas_handle hb = static_cast<rocblas_handle>(c->blas);
  if (rocblas_set_stream(hb, s) != rocblas_status_success)
    return set_error(c, MNL_ERR_HIP, "rocblas_set_stream failed");
  *handle = c->blas;
  return MNL_OK;
}

void graphs_release(Ctx *c) {
  for (auto &g : c->step_exec) {
    if (g) (void)hipGraphExecDestroy(g);
    g = nullptr;
  }
}

void events_release(Ctx *c) {
  graphs_release(c);
  if (c->pinned) {
    (void)hipHostFree(c->pinned);
    c->pinned = nullptr;
  }
  if (!c->ev_ready) return;
  (void)hipEventDestroy(c->ev_h0);
  (void)hipEventDestroy(c->ev_h1);
  (void)hipEventDestroy(c->ev_p0);
  (void)hipEventDestroy(c->ev_p1);
  for (auto &e : c->ev_q) (void)hipEventDestroy(e);
  c->ev_ready = false;
}

void blas_release(Ctx *c) {
  if (c->blas) {
    (void)rocblas_destroy_handle(static_cast<rocblas_handle>(c->blas));
    c->blas = nullptr;
  }
}

hipError_t raise_lds_limit(const void *kernel, int bytes) {
  static std::mutex mu;
  static std::map<std::pair<const void *, int>, int> limit;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(mu);
  int &cur = limit[{kernel, dev}];
  if (cur >= bytes) return hipSuccess;
  e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                          bytes);
  if (e == hipSuccess) cur = bytes;
  return e;
}

int check_problem(Ctx *c, const mnl_problem *pr, Dims *d, bool need_choice) {
  if (!pr) return set_error(c, MNL_ERR_ARG, "problem is NULL");
  if (pr->N < 1) return set_error(c, MNL_ERR_ARG, "N must be >= 1");
  if (pr->K < 2) return set_error(c, MNL_ERR_ARG, "K must be >= 2");
  if (pr->p < 0 || pr->g < 0 || pr->a < 0)
    return set_error(c, MNL_ERR_ARG, "negative dimension");
  if (pr->p > 0 && !pr->X) return set_error(c, MNL_ERR_ARG, "X is NULL");
  if (pr->g > 0 && !pr->Y) return set_error(c, MNL_ERR_ARG, "Y is NULL");
  if (pr->a > 0 && !pr->Z) return set_error(c, MNL_ERR_ARG, "Z is NULL");
  if (need_choice && !pr->choice)
    return set_error(c, MNL_ERR_ARG, "choice is NULL");
  d->N = pr->N;
  d->K = pr->K;
  d->p = pr->p;
  d->g = pr->g;
  d->a = pr->a;
  d->np = int64_t(pr->K - 1) * pr->p + int64_t(pr->K) * pr->a + pr->g;
  if (d->np < 1) return set_error(c, MNL_ERR_ARG, "model has no coefficients");
  if (int64_t(pr->K) * (pr->g + pr->a + 1) > (int64_t(1) << 24) ||
      pr->p > 4096)
    return set_error(c, MNL_ERR_UNSUPPORTED, "shape too large");
  return MNL_OK;
}

int check_opts(Ctx *c, const mnl_fit_opts *o) {
  if (o->maxiter < 0 || o->ls_max < 0 || o->ls_max > 1000 ||
      !(o->gtol >= 0) || !(o->ftol >= 0) || !(o->ls_tol_ulps >= 0) ||
      o->prec < MNL_PREC_FP64 || o->prec > MNL_PREC_BF16 ||
      o->method < MNL_METHOD_NEWTON || o->method > MNL_METHOD_NEWTON_CG ||
      o->cg_maxiter < 1)
    return set_error(c, MNL_ERR_ARG, "invalid fit options");
  return MNL_OK;
}

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch())
      .count();
}

namespace {

// One full pass (l, g, P, Ybar at theta) into the given workspace slots.
int run_pass(Ctx *c, const Dims &d, const mnl_problem *pr, const double *theta,
             double *lg, int slotP, int slotP32, int slotYbar, bool want_p32,
             hipStream_t s) {
  PassPlan plan;
  int rc = pass_plan(d, &plan);
  if (rc != MNL_OK)
    return set_error(c, rc, "shape beyond the fused-pass limits");
  void *partial, *P, *P32 = nullptr, *Ybar = nullptr;
  MNL_TRY(ws_get(c, S_PARTIAL, size_t(plan.grid) * plan.stride * 8, &partial));
  MNL_TRY(ws_get(c, slotP, size_t(d.N) * d.K * 8, &P));
  if (want_p32) MNL_TRY(ws_get(c, slotP32, size_t(d.N) * d.K * 4, &P32));
  if (d.g) MNL_TRY(ws_get(c, slotYbar, size_t(d.N) * d.g * 8, &Ybar));
  PassArgs A;
  A.d = d;
  A.X = pr->X;
  A.Y = pr->Y;
  A.Z = pr->Z;
  A.w = pr->w;
  A.choice = pr->choice;
  A.theta = theta;
  A.P = (double *)P;
  A.P32 = (float *)P32;
  A.Ybar = (double *)Ybar;
  A.partial = (double *)partial;
  if (c->ev_ready) MNL_HIP(c, hipEventRecord(c->ev_p0, s));
  MNL_HIP(c, launch_pass(plan, A, s));
  if (c->ev_ready) {
    MNL_HIP(c, hipEventRecord(c->ev_p1, s));
    c->pass_pending = true;
  }
  MNL_HIP(c, launch_pass_reduce(plan, (double *)partial, lg, lg + 1, d.np, s));
  return MNL_OK;
}

// Add the GPU times of the last bracketed kernels (call after a sync).
void collect_timing(Ctx *c, mnl_fit_info *info) {
  float ms = 0.0f;
  if (c->hess_pending) {
    if (hipEventElapsedTime(&ms, c->ev_h0, c->ev_h1) == hipSuccess) {
      info->t_hess_kernel += ms;
      info->n_hess += 1;
    }
    c->hess_pending = false;
  }
  if (c->pass_pending) {
    if (hipEventElapsedTime(&ms, c->ev_p0, c->ev_p1) == hipSuccess) {
      info->t_pass_kernel += ms;
      info->n_pass += 1;
    }
    c->pass_pending = false;
  }
  (void)hipGetLastError();
}

int ensure_events(Ctx *c) {
  if (c->ev_ready) return MNL_OK;
  MNL_HIP(c, hipEventCreate(&c->ev_h0));
  MNL_HIP(c, hipEventCreate(&c->ev_h1));
  MNL_HIP(c, hipEventCreate(&c->ev_p0));
  MNL_HIP(c, hipEventCreate(&c->ev_p1));
  for (auto &e : c->ev_q) MNL_HIP(c, hipEventCreate(&e));
  c->ev_ready = true;
  return MNL_OK;
}

// milliseconds between two recorded (and completed) events, 0 on error
double event_ms(hipEvent_t a, hipEvent_t b) {
  float ms = 0.0f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
    (void)hipGetLastError();
    return 0.0;
  }
  return double(ms);
}

struct StepState {
  double *lg;        // [0] l, [1..] g at theta
  double *lg_trial;
  int cur;           // which P/Ybar slots hold theta's values (0 or 1)
  double g2 = 0.0;   // |g|^2 at theta after an accepted step
};

// Hessian at the current theta (its P/Ybar in slot set `cur`) into S_H.
int form_hessian(Ctx *c, const Dims &d, const mnl_problem *pr, int cur,
                 int prec, double *H, hipStream_t s) {
  void *P, *P32 = nullptr, *Ybar = nullptr;
  MNL_TRY(ws_get(c, cur ? S_P_TRIAL : S_P, size_t(d.N) * d.K * 8, &P));
  if (prec != MNL_PREC_FP64)
    MNL_TRY(ws_get(c, cur ? S_P32_TRIAL : S_P32, size_t(d.N) * d.K * 4, &P32));
  if (d.g)
    MNL_TRY(ws_get(c, cur ? S_YBAR_TRIAL : S_YBAR, size_t(d.N) * d.g * 8,
                   &Ybar));
  HessArgs h;
  h.d = d;
  h.X = pr->X;
  h.Y = pr->Y;
  h.Z = pr->Z;
  h.w = pr->w;
  h.P = (const double *)P;
  h.P32 = (const float *)P32;
  h.Ybar = (const double *)Ybar;
  h.H = H;
  h.prec = prec;
  return hessian_run(c, h, s);
}

int copy_d2h(Ctx *c, void *dst, const void *src, size_t n, hipStream_t s) {
  MNL_HIP(c, hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToHost, s));
  MNL_HIP(c, hipStreamSynchronize(s));
  return MNL_OK;
}

int validate_data(Ctx *c, const Dims &d, const mnl_problem *pr,
                  hipStream_t s) {
  void *f;
  MNL_TRY(ws_get(c, S_SCAL, 256, &f));
  int32_t *flags = (int32_t *)f + 16;
  MNL_HIP(c, hipMemsetAsync(flags, 0, 8, s));
  MNL_HIP(c, launch_validate(d, pr->X, pr->Y, pr->Z, pr->w, pr->choice, flags,
                             s));
  int32_t h[2];
  MNL_TRY(copy_d2h(c, h, flags, 8, s));
  if (h[0]) return set_error(c, MNL_ERR_ARG, "%d choices out of range", h[0]);
  if (h[1])
    return set_error(c, MNL_ERR_NONFINITE,
                     "%d observations with non-finite data or bad weight",
                     h[1]);
  return MNL_OK;
}

// Inexact Newton direction (Sec. 5): truncated CG on (-H) d = g from d = 0
// with Hessian-vector passes at the P of slot set `cur`; stops when
// ||r|| <= eta ||g||, eta = min(1/2, sqrt(||g|| / ||g_0||)) with g_0 the
// gradient where the call started, after cg_maxiter
// products, or at p^T (-H) p <= 0 (d = g when that happens first).  One
// host round trip per product carries r.r and p^T (-H) p.
int cg_direction(Ctx *c, const Dims &d, const mnl_problem *pr,
                 const StepState &st, const mnl_fit_opts &o, double gnorm,
                 double gnorm0, double *delta, int *ncg, hipStream_t s) {
  PassPlan plan;
  int rc = pass_plan(d, &plan);
  if (rc != MNL_OK)
    return set_error(c, rc, "shape beyond the fused-pass limits");
  void *cv, *partial, *Pv;
  const int64_t n = d.np;
  MNL_TRY(ws_get(c, S_CG, size_t(3 * n + 8) * 8, &cv));
  MNL_TRY(ws_get(c, S_PARTIAL, size_t(plan.grid) * plan.stride * 8, &partial));
  MNL_TRY(ws_get(c, st.cur ? S_P_TRIAL : S_P, size_t(d.N) * d.K * 8, &Pv));
  double *r = (double *)cv, *p = r + n, *Hp = p + n, *scal = Hp + n;
  const double *g = st.lg + 1;
  MNL_HIP(c, launch_cg_init(g, delta, r, p, n, scal, s));
  const double eta = std::min(0.5, std::sqrt(gnorm / gnorm0));
  PassArgs A;
  A.d = d;
  A.X = pr->X;
  A.Y = pr->Y;
  A.Z = pr->Z;
  A.w = pr->w;
  A.choice = nullptr;
  A.theta = p;
  A.P = nullptr;
  A.P32 = nullptr;
  A.Ybar = nullptr;
  A.partial = (double *)partial;
  A.Pin = (const double *)Pv;
  double rr = gnorm * gnorm;
  int j = 0;
  for (; j < o.cg_maxiter; ++j) {
    if (j > 0 && std::sqrt(rr) <= eta * gnorm) break;
    MNL_HIP(c, launch_pass(plan, A, s));
    MNL_HIP(c, launch_pass_reduce(plan, (double *)partial, scal + 2, Hp, n, s));
    MNL_HIP(c, launch_cg_update(Hp, delta, r, p, n, scal, s));
    double h[2];
    MNL_TRY(copy_d2h(c, h, scal, sizeof h, s));
    rr = h[0];
    if (!(h[1] > 0.0)) {
      if (j == 0)
        MNL_HIP(c, hipMemcpyAsync(delta, g, size_t(n) * 8,
                                  hipMemcpyDeviceToDevice, s));
      ++j;
      break;
    }
  }
  *ncg = j;
  return MNL_OK;
}

// Core of one Newton iteration, given l and g at theta (in lg, P/Ybar in
// slot set `cur`).  On an accepted step theta is updated in place and lg,
// cur describe the new point.  Returns MNL_OK with *reason set.
int newton_core(Ctx *c, const Dims &d, const mnl_problem *pr, double *theta,
                const mnl_fit_opts &o, StepState &st, double l_old,
                double gnorm, double gnorm0, bool use_graph,
                mnl_fit_info *info, int *reason, hipStream_t s) {
  void *Hv, *dv, *tv, *sv;
  // n_p + 1 rows: the factorisation carries g as an extra row; 64 doubles
  // of padding let its kernels load whole panel rows unconditionally
  MNL_TRY(ws_get(c, S_H, (size_t(d.np + 1) * d.np + 64) * 8, &Hv));
  MNL_TRY(ws_get(c, S_DELTA, size_t(d.np) * 8, &dv));
  MNL_TRY(ws_get(c, S_THETA_TRIAL, size_t(d.np) * 8, &tv));
  MNL_TRY(ws_get(c, S_SCAL, 256, &sv));
  double *H = (double *)Hv, *delta = (double *)dv, *th_t = (double *)tv;
  int32_t *cinfo = (int32_t *)sv + 32;
  double *sc = (double *)sv + 24;   // status, l and |g|^2 of a trial
  const int nxt = st.cur ^ 1;
  const bool want32 = o.prec != MNL_PREC_FP64;
  // one trial of the line search at step t: theta + t delta, its pass and
  // the decision scalars (with the factorisation status when asked)
  auto trial_at = [&](double t, const int32_t *status) -> int {
    MNL_HIP(c, launch_axpy(theta, delta, t, th_t, d.np, s));
    MNL_TRY(run_pass(c, d, pr, th_t, st.lg_trial, nxt ? S_P_TRIAL : S_P,
                     nxt ? S_P32_TRIAL : S_P32, nxt ? S_YBAR_TRIAL : S_YBAR,
                     want32, s));
    MNL_HIP(c, launch_scalars(st.lg_trial, d.np, status, sc, s));
    return MNL_OK;
  };

  // Hessian and Newton direction (Eq. 6): delta = (-H)^{-1} g; the full
  // step's trial runs behind the factorisation, so one copy to the host
  // brings the factorisation status and the trial's l and |g|^2
  int prec = o.prec;
  int32_t fail = 0;
  double sh[3] = {0.0, 0.0, 0.0};
  bool done = false;
  if (use_graph) {
    // the step of this parity: captured on first use (every buffer it
    // touches exists by now), then replayed; eager on any capture error
    hipGraphExec_t &ex = c->step_exec[st.cur];
    if (!ex) {
      const bool ev = c->ev_ready;
      c->ev_ready = false;   // no timing events inside the graph
      hipGraph_t gr = nullptr;
      int rc = MNL_OK;
      if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) ==
          hipSuccess) {
        c->capturing = true;
        rc = form_hessian(c, d, pr, st.cur, prec, H, s);
        if (rc == MNL_OK) rc = chol_solve_run(c, H, d.np, st.lg + 1, delta,
                                              cinfo, s);
        if (rc == MNL_OK) rc = trial_at(1.0, cinfo);
        if (rc == MNL_OK &&
            hipMemcpyAsync(c->pinned, sc, 3 * sizeof(double),
                           hipMemcpyDeviceToHost, s) != hipSuccess)
          rc = MNL_ERR_HIP;
        const hipError_t ee = hipStreamEndCapture(s, &gr);
        c->capturing = false;
        if (ee != hipSuccess) rc = MNL_ERR_HIP;
        if (rc == MNL_OK &&
            hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0) != hipSuccess)
          ex = nullptr;
        if (gr) (void)hipGraphDestroy(gr);
      }
      (void)hipGetLastError();
      c->ev_ready = ev;
      if (!ex) use_graph = false;
    }
    if (ex) {
      MNL_HIP(c, hipGraphLaunch(ex, s));
      MNL_HIP(c, hipStreamSynchronize(s));
      info->graph_steps += 1;
      std::memcpy(sh, c->pinned, sizeof sh);
      fail = int32_t(sh[0]);
      done = fail == 0 || prec == MNL_PREC_FP64;
      if (!done) {
        prec = MNL_PREC_FP64;   // the FP64 retry runs eagerly
        info->hess_fallbacks += 1;
      }
    }
  }
  if (!done && o.method == MNL_METHOD_NEWTON_CG) {
    // inexact Newton: the inner solve's time is reported as t_hessian
    int ncg = 0;
    MNL_HIP(c, hipEventRecord(c->ev_q[0], s));
    MNL_TRY(cg_direction(c, d, pr, st, o, gnorm, gnorm0, delta, &ncg, s));
    info->cg_iters += ncg;
    MNL_HIP(c, hipEventRecord(c->ev_q[2], s));
    MNL_TRY(trial_at(1.0, nullptr));
    MNL_HIP(c, hipEventRecord(c->ev_q[3], s));
    MNL_TRY(copy_d2h(c, sh, sc, sizeof sh, s));
    collect_timing(c, info);
    info->t_hessian += event_ms(c->ev_q[0], c->ev_q[2]);
    info->t_ls += event_ms(c->ev_q[2], c->ev_q[3]);
  }
  for (int attempt = 0; !done && o.method == MNL_METHOD_NEWTON && attempt < 2;
       ++attempt) {
    MNL_HIP(c, hipEventRecord(c->ev_q[0], s));
    MNL_TRY(form_hessian(c, d, pr, st.cur, prec, H, s));
    MNL_HIP(c, hipEventRecord(c->ev_q[1], s));
    // the factorisation works on A = -H in place
    MNL_TRY(chol_solve_run(c, H, d.np, st.lg + 1, delta, cinfo, s));
    MNL_HIP(c, hipEventRecord(c->ev_q[2], s));
    MNL_TRY(trial_at(1.0, cinfo));
    MNL_HIP(c, hipEventRecord(c->ev_q[3], s));
    MNL_TRY(copy_d2h(c, sh, sc, sizeof sh, s));
    collect_timing(c, info);
    info->t_hessian += event_ms(c->ev_q[0], c->ev_q[1]);
    info->t_chol += event_ms(c->ev_q[1], c->ev_q[2]);
    fail = int32_t(sh[0]);
    if (fail == 0) info->t_ls += event_ms(c->ev_q[2], c->ev_q[3]);
    if (fail == 0 || prec == MNL_PREC_FP64) break;
    // a rounded Hessian that is not positive definite: redo it in FP64
    prec = MNL_PREC_FP64;
    info->hess_fallbacks += 1;
  }
  if (fail != 0) {
    *reason = MNL_STOP_NOT_PD;
    return MNL_OK;
  }

  // halving line search (Sec. 3.1); the full step is already evaluated
  const double tau =
      o.ls_tol_ulps * std::numeric_limits<double>::epsilon() * std::fabs(l_old);
  double t = 1.0;
  for (int trial = 1; trial <= o.ls_max + 1; ++trial) {
    if (trial > 1) {
      MNL_HIP(c, hipEventRecord(c->ev_q[2], s));
      MNL_TRY(trial_at(t, nullptr));
      MNL_HIP(c, hipEventRecord(c->ev_q[3], s));
      MNL_TRY(copy_d2h(c, sh, sc, sizeof sh, s));
      collect_timing(c, info);
      info->t_ls += event_ms(c->ev_q[2], c->ev_q[3]);
    }
    const double l_new = sh[1];
    info->ls_iters += 1;
    if (std::isfinite(l_new) && l_new >= l_old - tau) {
      info->ls_backtracks += trial - 1;
      MNL_HIP(c, hipMemcpyAsync(theta, th_t, size_t(d.np) * 8,
                                hipMemcpyDeviceToDevice, s));
      std::swap(st.lg, st.lg_trial);
      st.cur = nxt;
      st.g2 = sh[2];
      info->loglik_diff = l_new - l_old;
      info->loglik = l_new;
      *reason = MNL_STOP_NONE;
      return MNL_OK;
    }
    t *= 0.5;
  }
  info->ls_backtracks += o.ls_max;
  *reason = MNL_STOP_LS_FAIL;
  return MNL_OK;
}

}  // namespace
int fit_impl(Ctx *c, const mnl_problem *prob, double *theta,
             const mnl_fit_opts &o, mnl_fit_info *info, bool one_step,
             hipStream_t s) {
  Dims d;
  MNL_TRY(check_problem(c, prob, &d));
  MNL_TRY(check_opts(c, &o));
  MNL_HIP(c, hipSetDevice(c->device));
  const double t_start = now_ms();
  ++c->call_epoch;  // data-derived caches are valid within one call only
  std::memset(info, 0, sizeof *info);
  MNL_TRY(ensure_events(c));
  c->hess_pending = c->pass_pending = false;
  if (o.validate) MNL_TRY(validate_data(c, d, prob, s));
  void *a, *b;
  MNL_TRY(ws_get(c, S_LG, size_t(d.np + 1) * 8, &a));
  MNL_TRY(ws_get(c, S_LG_TRIAL, size_t(d.np + 1) * 8, &b));
  void *sv;
  MNL_TRY(ws_get(c, S_SCAL, 256, &sv));
  double *gn2 = (double *)sv;
  StepState st{(double *)a, (double *)b, 0};

  double t0 = now_ms();
  MNL_TRY(run_pass(c, d, prob, theta, st.lg, S_P, S_P32, S_YBAR,
                   o.prec != MNL_PREC_FP64, s));
  double l = 0.0, gnorm = 0.0;
  {
    MNL_HIP(c, launch_scalars(st.lg, d.np, nullptr, gn2, s));
    double h[3];
    MNL_TRY(copy_d2h(c, h, gn2, sizeof h, s));
    collect_timing(c, info);
    l = h[1];
    gnorm = std::sqrt(h[2]);
  }
  info->t_loglik_grad = now_ms() - t0;
  const double gnorm0 = gnorm;   // scale of the inexact Newton forcing term
  // captured steps: only on a non-default stream, for exact Newton steps
  // below the outer-panel factorisation's size; by default only for small
  // fits, whose steps are launch-bound
  const bool graph_on =
      o.graph > 0 || (o.graph < 0 && d.np <= MNL_GRAPH_AUTO_MAX_NP);
  bool graph_ok = graph_on && s != nullptr && o.method == MNL_METHOD_NEWTON &&
                  d.np < 2048 && !one_step;
  if (graph_ok && !c->pinned) {
    if (hipHostMalloc(reinterpret_cast<void **>(&c->pinned), 256) !=
        hipSuccess) {
      (void)hipGetLastError();
      c->pinned = nullptr;
      graph_ok = false;
    }
  }
  graphs_release(c);   // graphs hold the previous fit's pointers
  info->loglik_diff = std::numeric_limits<double>::quiet_NaN();
  int reason = MNL_STOP_NONE;
  for (;;) {
    if (!std::isfinite(l) || !std::isfinite(gnorm)) {
      reason = MNL_STOP_NONFINITE;
      break;
    }
    if (gnorm <= o.gtol) {
      reason = MNL_STOP_GTOL;
      break;
    }
    if (!one_step && info->iters >= o.maxiter) {
      reason = MNL_STOP_MAXITER;
      break;
    }
    if (one_step && info->iters >= 1) break;
    int r = MNL_STOP_NONE;
    const double step_gnorm = gnorm;
    // graph replay from the second iteration (the first allocates)
    const bool g_now = graph_ok && info->iters >= 1;
    const int rcn = newton_core(c, d, prob, theta, o, st, l, step_gnorm,
                                gnorm0, g_now, info, &r, s);
    if (rcn != MNL_OK) {
      graphs_release(c);
      return rcn;
    }
    if (r != MNL_STOP_NONE) {
      reason = r;
      if (one_step) info->grad_norm = step_gnorm;
      break;
    }
    info->iters += 1;
    l = info->loglik;
    gnorm = std::sqrt(st.g2);   // from the accepted trial's scalars
    if (one_step) {
      info->grad_norm = step_gnorm;
      info->loglik = l;
      info->stop_reason = MNL_STOP_NONE;
      info->t_total = now_ms() - t_start;
      return MNL_OK;
    }
    if (std::fabs(info->loglik_diff) < o.ftol) {
      reason = MNL_STOP_FTOL;
      break;
    }
  }
  info->stop_reason = reason;
  info->loglik = l;
  if (!one_step || reason == MNL_STOP_GTOL || reason == MNL_STOP_NONFINITE)
    info->grad_norm = gnorm;
  info->t_total = now_ms() - t_start;
  graphs_release(c);
  return MNL_OK;
}


int fit_workspace_footprint(Ctx *c, const Dims &d, int prec, size_t *bytes) {
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  PassPlan plan;
  if (pass_plan(d, &plan) != MNL_OK)
    return set_error(c, MNL_ERR_UNSUPPORTED, "shape beyond the fused-pass limits");
  const size_t np = size_t(d.np), N = size_t(d.N), K = size_t(d.K);
  size_t t = al(size_t(plan.grid) * plan.stride * 8);  // S_PARTIAL
  t += 2 * al((np + 1) * 8);                            // S_LG, S_LG_TRIAL
  t += 2 * al(N * K * 8);                               // S_P, S_P_TRIAL
  if (prec != MNL_PREC_FP64) t += 2 * al(N * K * 4);   // S_P32 pair
  if (d.g) t += 2 * al(N * size_t(d.g) * 8);            // S_YBAR pair
  t += al(((np + 1) * np + 64) * 8);                    // S_H
  t += 2 * al(np * 8) + al(256);                        // delta, trial, scalars
  t += al(chol_workspace_bytes(int64_t(np)));           // Cholesky scratch
  t += al((3 * np + 8) * 8);                            // inexact Newton
  // Hessian partials and tables; a mixed fit may redo the Hessian in FP64
  size_t part = 0, tab = 0;
  MNL_TRY(hessian_footprint(c, d, prec, &part, &tab));
  t += al(part) + al(tab);
  if (prec != MNL_PREC_FP64) {
    size_t part64 = 0, tab64 = 0;
    MNL_TRY(hessian_footprint(c, d, MNL_PREC_FP64, &part64, &tab64));
    // an upper bound: the FP64 retry's partials, P blocks, chi operand
    // (a slot of its own) and tables on top of the mixed ones
    t += al(part64) + al(tab64);
  }
  *bytes = t;
  return MNL_OK;
}

}  // namespace mnl

namespace mnl {

// Upper tail of the chi-square distribution, Q(df/2, x/2) with Q the
// regularised upper incomplete gamma function: the power series of the
// lower function for x < a + 1, else Legendre's continued fraction for the
// upper one evaluated by the modified Lentz method (Abramowitz & Stegun
// 6.5.29 and 6.5.31).
double chi2_upper_tail(double x, double df) {
  if (!(df > 0.0) || std::isnan(x)) return std::numeric_limits<double>::quiet_NaN();
  if (x <= 0.0) return 1.0;
  const double a = 0.5 * df, z = 0.5 * x;
  const double lpre = a * std::log(z) - z - std::lgamma(a);
  const double eps = 1e-16;
  if (z < a + 1.0) {
    // P(a, z) = z^a e^{-z} / Gamma(a + 1) sum_n z^n / ((a+1)...(a+n))
    double term = 1.0 / a, sum = term;
    for (int n = 1; n < 100000; ++n) {
      term *= z / (a + n);
      sum += term;
      if (std::fabs(term) < std::fabs(sum) * eps) break;
    }
    return 1.0 - std::exp(lpre) * sum;
  }
  // Q(a, z) = z^a e^{-z} / Gamma(a) * 1 / (z + 1 - a - 1 (1 - a) /
  //           (z + 3 - a - 2 (2 - a) / (z + 5 - a - ...)))
  const double tiny = 1e-300;
  double b = z + 1.0 - a, cc = 1.0 / tiny, dd = 1.0 / b, h = dd;
  for (int n = 1; n < 100000; ++n) {
    const double an = -n * (n - a);
    b += 2.0;
    dd = an * dd + b;
    if (std::fabs(dd) < tiny) dd = tiny;
    cc = b + an / cc;
    if (std::fabs(cc) < tiny) cc = tiny;
    dd = 1.0 / dd;
    const double del = dd * cc;
    h *= del;
    if (std::fabs(del - 1.0) < eps) break;
  }
  return std::exp(lpre) * h;
}

namespace {
// FP64 Hessian at theta factored as -H = L D L^T with n_p identity rows
// appended (they end as L^{-T} D^{-1}); *H_out is the matrix buffer,
// *cinfo_out the device status.
int factor_with_identity(Ctx *c, const Dims &d, const mnl_problem *prob,
                         const double *theta, double **H_out,
                         int32_t **cinfo_out, hipStream_t s) {
  void *lg, *Hv, *sv;
  MNL_TRY(ws_get(c, S_LG, size_t(d.np + 1) * 8, &lg));
  // 2 n_p + 1 rows: H, the (zero) g row and n_p identity rows, plus the
  // factorisation's padding
  MNL_TRY(ws_get(c, S_H, (size_t(2 * d.np + 1) * d.np + 64) * 8, &Hv));
  MNL_TRY(ws_get(c, S_SCAL, 256, &sv));
  int32_t *cinfo = (int32_t *)sv + 32;
  double *H = (double *)Hv;
  MNL_TRY(run_pass(c, d, prob, theta, (double *)lg, S_P, S_P32, S_YBAR, false,
                   s));
  MNL_TRY(form_hessian(c, d, prob, 0, MNL_PREC_FP64, H, s));
  MNL_TRY(chol_solve_run(c, H, d.np, nullptr, nullptr, cinfo, s, d.np));
  *H_out = H;
  *cinfo_out = cinfo;
  return MNL_OK;
}
}  // namespace

// Static device scratch of the entry point that allocates nothing
// (mnl_loglik_grad_noalloc): the fused pass's per-workgroup partial rows.
// Every device the library runs on holds its own copy from the module's
// load until the process ends.  Host code never passes the array's name to
// a kernel: its device address on each device comes from
// hipGetSymbolAddress (scratch_setup, called by mnl_create with the device
// current) and is kept per device.
constexpr size_t kScratchBytes = MNL_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[kScratchBytes / 8];
std::mutex scratch_mu;
void *scratch_ptr[kMaxDevices] = {};

int scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return MNL_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (scratch_ptr[device]) return MNL_OK;
  void *p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
    (void)hipGetLastError();
    return MNL_ERR_HIP;
  }
  scratch_ptr[device] = p;
  return MNL_OK;
}

void *scratch_get(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(scratch_mu);
  return scratch_ptr[device];
}

}  // namespace mnl

using namespace mnl;

extern "C" {

const char *mnl_version(void) { return "0.1"; }

const char *mnl_strerror(int code) {
  switch (code) {
    case MNL_OK: return "ok";
    case MNL_ERR_ARG: return "invalid argument";
    case MNL_ERR_OOM: return "out of device memory";
    case MNL_ERR_NOT_PD: return "Hessian not negative definite";
    case MNL_ERR_NONFINITE: return "non-finite value";
    case MNL_ERR_LS_FAIL: return "line search failed";
    case MNL_ERR_HIP: return "HIP runtime error";
    case MNL_ERR_UNSUPPORTED: return "unsupported shape";
    default: return "unknown error";
  }
}

void mnl_default_opts(mnl_fit_opts *o) {
  if (!o) return;
  o->maxiter = 50;
  o->ftol = 1e-6;
  o->gtol = 1e-6;
  o->prec = MNL_PREC_FP64;
  o->ls_max = 30;
  o->ls_tol_ulps = 64.0;
  o->validate = 0;
  o->method = MNL_METHOD_NEWTON;
  o->cg_maxiter = 250;
  o->graph = MNL_GRAPH_AUTO;
}

int64_t mnl_num_params(int32_t K, int32_t p, int32_t g, int32_t a) {
  if (K < 2 || p < 0 || g < 0 || a < 0) return -1;
  return int64_t(K - 1) * p + int64_t(K) * a + g;
}

int mnl_create(mnl_ctx **ctx, int device, size_t workspace_bytes) {
  if (!ctx) return MNL_ERR_ARG;
  *ctx = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess) {
    (void)hipGetLastError();
    return MNL_ERR_HIP;
  }
  if (device < 0 || device >= n) return MNL_ERR_ARG;
  if (hipSetDevice(device) != hipSuccess) return MNL_ERR_HIP;
  // this device's address of the static scratch (with the device current)
  const int rs = scratch_setup(device);
  if (rs != MNL_OK) return rs;
  mnl_ctx *h = new mnl_ctx;
  h->c.device = device;
  h->c.bufs.resize(S_NSLOTS);
  h->c.ws_cap = workspace_bytes;
  *ctx = h;
  return MNL_OK;
}

void mnl_destroy(mnl_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->c.device);
  (void)hipDeviceSynchronize();
  for (auto &b : ctx->c.bufs)
    if (b.ptr) (void)hipFree(b.ptr);
  hessian_cache_free(&ctx->c);
  blas_release(&ctx->c);
  events_release(&ctx->c);
  delete ctx;
}

size_t mnl_workspace_bytes(const mnl_ctx *ctx) {
  return ctx ? ctx->c.total_bytes : 0;
}

const char *mnl_last_error(const mnl_ctx *ctx) {
  return ctx ? ctx->c.last_error.c_str() : "";
}

int mnl_loglik_grad(mnl_ctx *ctx, const mnl_problem *prob, const double *theta,
                    double *loglik, double *grad, double *P, void *stream) {
  if (!ctx) return MNL_ERR_ARG;
  Ctx *c = &ctx->c;
  Dims d;
  MNL_TRY(check_problem(c, prob, &d));
  if (!theta || !loglik) return set_error(c, MNL_ERR_ARG, "NULL output");
  MNL_HIP(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  PassPlan plan;
  int rc = pass_plan(d, &plan);
  if (rc != MNL_OK) return set_error(c, rc, "shape beyond pass limits");
  void *partial, *Pw = P, *Yb = nullptr;
  MNL_TRY(ws_get(c, S_PARTIAL, size_t(plan.grid) * plan.stride * 8, &partial));
  if (d.g) MNL_TRY(ws_get(c, S_YBAR, size_t(d.N) * d.g * 8, &Yb));
  PassArgs A;
  A.d = d;
  A.X = prob->X;
  A.Y = prob->Y;
  A.Z = prob->Z;
  A.w = prob->w;
  A.choice = prob->choice;
  A.theta = theta;
  A.P = (double *)Pw;
  A.P32 = nullptr;
  A.Ybar = (double *)Yb;
  A.partial = (double *)partial;
  MNL_HIP(c, launch_pass(plan, A, s));
  MNL_HIP(c, launch_pass_reduce(plan, (double *)partial, loglik, grad, d.np,
                                s));
  return MNL_OK;
}

int mnl_loglik_grad_noalloc(mnl_ctx *ctx, const mnl_problem *prob,
                            const double *theta, double *loglik, double *grad,
                            double *P, void *stream) {
  if (!ctx) return MNL_ERR_ARG;
  Ctx *c = &ctx->c;
  Dims d;
  MNL_TRY(check_problem(c, prob, &d));
  if (!theta || !loglik) return set_error(c, MNL_ERR_ARG, "NULL output");
  MNL_HIP(c, hipSetDevice(c->device));
  PassPlan plan;
  int rc = pass_plan(d, &plan);
  if (rc != MNL_OK) return set_error(c, rc, "shape beyond pass limits");
  const size_t need = size_t(plan.grid) * size_t(plan.stride) * 8;
  if (need > kScratchBytes)
    return set_error(c, MNL_ERR_UNSUPPORTED,
                     "the pass needs %zu bytes of scratch (%d workgroup rows "
                     "of %lld values), more than the %zu-byte static buffer",
                     need, plan.grid, (long long)plan.stride, kScratchBytes);
  void *sp = scratch_get(c->device);
  if (!sp) return set_error(c, MNL_ERR_HIP, "no scratch address for device");
  PassArgs A;
  A.d = d;
  A.X = prob->X;
  A.Y = prob->Y;
  A.Z = prob->Z;
  A.w = prob->w;
  A.choice = prob->choice;
  A.theta = theta;
  A.P = P;
  A.P32 = nullptr;
  A.Ybar = nullptr;
  A.partial = static_cast<double *>(sp);
  hipStream_t s = (hipStream_t)stream;
  MNL_HIP(c, launch_pass(plan, A, s));
  MNL_HIP(c, launch_pass_reduce(plan, A.partial, loglik, grad, d.np, s));
  return MNL_OK;
}

int mnl_hessian(mnl_ctx *ctx, const mnl_problem *prob, const double *theta,
                int32_t prec, double *H, void *stream) {
  if (!ctx) return MNL_ERR_ARG;
  Ctx *c = &ctx->c;
  Dims d;
  MNL_TRY(check_problem(c, prob, &d));
  if (!theta || !H) return set_error(c, MNL_ERR_ARG, "NULL argument");
  if (prec < MNL_PREC_FP64 || prec > MNL_PREC_BF16)
    return set_error(c, MNL_ERR_ARG, "bad precision");
  MNL_HIP(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  ++c->call_epoch;
  void *lg;
  MNL_TRY(ws_get(c, S_LG, size_t(d.np + 1) * 8, &lg));
  MNL_TRY(run_pass(c, d, prob, theta, (double *)lg, S_P, S_P32, S_YBAR,
                   prec != MNL_PREC_FP64, s));
  return form_hessian(c, d, prob, 0, prec, H, s);
}

int mnl_hessvec(mnl_ctx *ctx, const mnl_problem *prob, const double *theta,
                const double *v, double *Hv, void *stream) {
  if (!ctx) return MNL_ERR_ARG;
  Ctx *c = &ctx->c;
  Dims d;
  MNL_TRY(check_problem(c, prob, &d, false));
  if (!theta || !v || !Hv) return set_error(c, MNL_ERR_ARG, "NULL argument");
  MNL_HIP(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  ++c->call_epoch;
  PassPlan plan;
  int rc = pass_plan(d, &plan);
  if (rc != MNL_OK) return set_error(c, rc, "shape beyond pass limits");
  void *lg, *Pv, *partial;
  MNL_TRY(ws_get(c, S_LG, size_t(d.np + 1) * 8, &lg));
  // P at theta (slot S_P), then the pass of v with P read back
  MNL_TRY(run_pass(c, d, prob, theta, (double *)lg, S_P, S_P32, S_YBAR, false,
                   s));
  MNL_TRY(ws_get(c, S_P, size_t(d.N) * d.K * 8, &Pv));
  MNL_TRY(ws_get(c, S_PARTIAL, size_t(plan.grid) * plan.stride * 8, &partial));
  PassArgs A;
  A.d = d;
  A.X = prob->X;
  A.Y = prob->Y;
  A.Z = prob->Z;
  A.w = prob->w;
  A.choice = nullptr;
  A.theta = v;
  A.P = nullptr;
  A.P32 = nullptr;
  A.Ybar = nullptr;
  A.partial = (double *)partial;
  A.Pin = (const double *)Pv;
  MNL_HIP(c, launch_pass(plan, A, s));
  // l of this pass is meaningless: it goes to the scratch l slot
  MNL_HIP(c, launch_pass_reduce(plan, (double *)partial, (double *)lg, Hv,
                                d.np, s));
  c->pass_pending = false;
  return MNL_OK;
}

int mnl_collinear(mnl_ctx *ctx, const mnl_problem *prob, double tol,
                  int32_t *keep_x, int32_t *keep_y, int32_t *keep_z,
                  void *stream) {
  if (!ctx) return MNL_ERR_ARG;
  Ctx *c = &ctx->c;
  Dims d;
  MNL_TRY(check_problem(c, prob, &d, false));
  if (!(tol >= 0.0) || !(tol < 1.0))
    return set_error(c, MNL_ERR_ARG, "tol must lie in [0, 1)");
  if ((d.p && !keep_x) || (d.g && !keep_y) || (d.a && !keep_z))
    return set_error(c, MNL_ERR_ARG, "NULL keep array");
  MNL_HIP(c, hipSetDevice(c->device));
  ++c->call_epoch;
  return collinear_run(c, d, prob, tol, keep_x, keep_y, keep_z,
                       (hipStream_t)stream);
}

int mnl_select_columns(mnl_ctx *ctx, const mnl_problem *prob,
                       const int32_t *keep_x, const int32_t *keep_y,
                       const int32_t *keep_z, double *X_out, double *Y_out,
                       double *Z_out, void *stream) {
  if (!ctx) return MNL_ERR_ARG;
  Ctx *c = &ctx->c;
  Dims d;
  MNL_TRY(check_problem(c, prob, &d, false));
  if ((d.p && !keep_x) || (d.g && !keep_y) || (d.a && !keep_z))
    return set_error(c, MNL_ERR_ARG, "NULL keep array");
  MNL_HIP(c, hipSetDevice(c->device));
  return select_columns_run(c, d, prob, keep_x, keep_y, keep_z, X_out, Y_out,
                            Z_out, (hipStream_t)stream);
}

int mnl_predict(mnl_ctx *ctx, const mnl_problem *prob, const double *theta,
                double *P, void *stream) {
  if (!ctx) return MNL_ERR_ARG;
  Ctx *c = &ctx->c;
  Dims d;
  MNL_TRY(check_problem(c, prob, &d, false));
  if (!theta || !P) return set_error(c, MNL_ERR_ARG, "NULL argument");
  MNL_HIP(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  PassPlan plan;
  int rc = pass_plan(d, &plan);
  if (rc != MNL_OK) return set_error(c, rc, "shape beyond pass limits");
  // the fused pass with no choices: P is its output, the partial rows of
  // l and g are left unreduced
  void *partial;
  MNL_TRY(ws_get(c, S_PARTIAL, size_t(plan.grid) * plan.stride * 8, &partial));
  PassArgs A;
  A.d = d;
  A.X = prob->X;
  A.Y = prob->Y;
  A.Z = prob->Z;
  A.w = nullptr;
  A.choice = nullptr;
  A.theta = theta;
  A.P = P;
  A.P32 = nullptr;
  A.Ybar = nullptr;
  A.partial = (double *)partial;
  MNL_HIP(c, launch_pass(plan, A, s));
  return MNL_OK;
}


int mnl_covariance(mnl_ctx *ctx, const mnl_problem *prob, const double *theta,
                   const int32_t *idx, int32_t nidx, double *V,
                   void *stream) {
  if (!ctx) return MNL_ERR_ARG;
  Ctx *c = &ctx->c;
  Dims d;
  MNL_TRY(check_problem(c, prob, &d, false));
  if (!theta || !V || (nidx > 0 && !idx) || nidx < 0)
    return set_error(c, MNL_ERR_ARG, "NULL argument or negative count");
  const int32_t s_n = nidx ? nidx : int32_t(d.np);
  std::vector<int32_t> sel(s_n);
  for (int32_t j = 0; j < s_n; ++j) {
    sel[j] = nidx ? idx[j] : j;
    if (sel[j] < 0 || sel[j] >= d.np)
      return set_error(c, MNL_ERR_ARG, "coefficient index out of range");
  }
  MNL_HIP(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  ++c->call_epoch;
  double *H;
  int32_t *cinfo;
  MNL_TRY(factor_with_identity(c, d, prob, theta, &H, &cinfo, s));
  void *iv;
  MNL_TRY(ws_get(c, S_COLLIN, size_t(s_n) * 4 + 8, &iv));
  MNL_HIP(c, hipMemcpyAsync(iv, sel.data(), size_t(s_n) * 4,
                            hipMemcpyHostToDevice, s));
  MNL_HIP(c, launch_cov_sub(H, d.np, (const int32_t *)iv, s_n, V, cinfo, s));
  int32_t fail = 0;
  MNL_TRY(copy_d2h(c, &fail, cinfo, sizeof fail, s));
  c->hess_pending = c->pass_pending = false;
  if (fail)
    return set_error(c, MNL_ERR_NOT_PD,
                     "-H not positive definite (pivot %d)", int(fail) - 1);
  return MNL_OK;
}

int mnl_quadform(mnl_ctx *ctx, const double *A, const double *B,
                 const double *x, const double *x0, int64_t n,
                 int32_t hessian_sign, double *out, void *stream) {
  if (!ctx) return MNL_ERR_ARG;
  Ctx *c = &ctx->c;
  if (!A || !x || !out || n < 1)
    return set_error(c, MNL_ERR_ARG, "NULL argument or empty matrix");
  MNL_HIP(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  void *bv, *sv;
  // matrix rows, then d = x - x0 as the g row, plus padding
  MNL_TRY(ws_get(c, S_H, (size_t(n + 1) * n + 64) * 8, &bv));
  MNL_TRY(ws_get(c, S_SCAL, 256, &sv));
  int32_t *cinfo = (int32_t *)sv + 32;
  double *qd = (double *)sv + 8;
  double *Bf = (double *)bv;
  // the factorisation takes a Hessian-signed matrix and factors its
  // negation: a positive definite A goes in negated
  MNL_HIP(c, launch_signed_copy(A, B, x, x0, hessian_sign ? 1.0 : -1.0, n,
                                Bf, s));
  // d = x - x0 is already in the g row (its copy into that row is then
  // element by element onto itself)
  MNL_TRY(chol_solve_run(c, Bf, n, Bf + n * n, nullptr, cinfo, s));
  MNL_HIP(c, launch_quad(Bf, n, qd, cinfo, s));
  struct {
    double q;
    int32_t fail;
  } h;
  MNL_HIP(c, hipMemcpyAsync(&h.q, qd, 8, hipMemcpyDeviceToHost, s));
  MNL_HIP(c, hipMemcpyAsync(&h.fail, cinfo, 4, hipMemcpyDeviceToHost, s));
  MNL_HIP(c, hipStreamSynchronize(s));
  if (h.fail)
    return set_error(c, MNL_ERR_NOT_PD,
                     "matrix not positive definite (pivot %d)",
                     int(h.fail) - 1);
  *out = h.q;
  return MNL_OK;
}

double mnl_chi2_sf(double x, double df) { return chi2_upper_tail(x, df); }

int mnl_lrtest(double loglik_full, double loglik_restricted, int32_t df,
               double *stat, double *pval) {
  if (!stat || df <= 0) return MNL_ERR_ARG;
  *stat = 2.0 * (loglik_full - loglik_restricted);
  if (pval) *pval = chi2_upper_tail(*stat, double(df));
  return MNL_OK;
}

int mnl_stderr(mnl_ctx *ctx, const mnl_problem *prob, const double *theta,
               double *se, double *zval, double *pval, void *stream) {
  if (!ctx) return MNL_ERR_ARG;
  Ctx *c = &ctx->c;
  Dims d;
  MNL_TRY(check_problem(c, prob, &d, false));
  if (!theta || !se) return set_error(c, MNL_ERR_ARG, "NULL argument");
  MNL_HIP(c, hipSetDevice(c->device));
  hipStream_t s = (hipStream_t)stream;
  ++c->call_epoch;
  double *H;
  int32_t *cinfo;
  MNL_TRY(factor_with_identity(c, d, prob, theta, &H, &cinfo, s));
  MNL_HIP(c, launch_inv_diag(H, d.np, theta, se, zval, pval, cinfo, s));
  int32_t fail = 0;
  MNL_TRY(copy_d2h(c, &fail, cinfo, sizeof fail, s));
  c->hess_pending = c->pass_pending = false;
  if (fail)
    return set_error(c, MNL_ERR_NOT_PD,
                     "-H not positive definite (pivot %d)", int(fail) - 1);
  return MNL_OK;
}

int mnl_newton_step(mnl_ctx *ctx, const mnl_problem *prob, double *theta,
                    const mnl_fit_opts *opts, mnl_fit_info *step,
                    void *stream) {
  if (!ctx) return MNL_ERR_ARG;
  Ctx *c = &ctx->c;
  if (!theta || !step) return set_error(c, MNL_ERR_ARG, "NULL argument");
  mnl_fit_opts o;
  if (opts) o = *opts;
  else mnl_default_opts(&o);
  return fit_impl(c, prob, theta, o, step, true, (hipStream_t)stream);
}

int mnl_fit(mnl_ctx *ctx, const mnl_problem *prob, const double *theta0,
            const mnl_fit_opts *opts, double *theta_out, mnl_fit_info *info,
            void *stream) {
  if (!ctx) return MNL_ERR_ARG;
  Ctx *c = &ctx->c;
  if (!theta_out || !info) return set_error(c, MNL_ERR_ARG, "NULL argument");
  mnl_fit_opts o;
  if (opts) o = *opts;
  else mnl_default_opts(&o);
  Dims d;
  MNL_TRY(check_problem(c, prob, &d));
  hipStream_t s = (hipStream_t)stream;
  MNL_HIP(c, hipSetDevice(c->device));
  if (theta0) {
    if (theta0 != theta_out)
      MNL_HIP(c, hipMemcpyAsync(theta_out, theta0, size_t(d.np) * 8,
                                hipMemcpyDeviceToDevice, s));
  } else {
    MNL_HIP(c, hipMemsetAsync(theta_out, 0, size_t(d.np) * 8, s));
  }
  int rc = fit_impl(c, prob, theta_out, o, info, false, s);
  (void)hipStreamSynchronize(s);
  return rc;
}

int mnl_fit_batch(mnl_ctx *ctx, int32_t nfits, const mnl_problem *probs,
                  const double *const *theta0, const mnl_fit_opts *opts,
                  double *const *theta_out, mnl_fit_info *info,
                  void *stream) {
  if (!ctx) return MNL_ERR_ARG;
  Ctx *c = &ctx->c;
  ++c->call_epoch;
  return small_fit_run(c, nfits, probs, theta0, opts, theta_out, info,
                       (hipStream_t)stream);
}

int mnl_batch_eligible(const mnl_problem *shape, const mnl_fit_opts *opts) {
  if (!shape) return 0;
  mnl_fit_opts o;
  if (opts) o = *opts;
  else mnl_default_opts(&o);
  Ctx c;
  if (check_opts(&c, &o) != MNL_OK) return 0;
  // only the sizes matter: stand-in pointers pass the NULL checks
  static const double dummy = 0.0;
  static const int32_t dummy_c = 0;
  mnl_problem pr = *shape;
  pr.X = pr.Y = pr.Z = &dummy;
  pr.choice = &dummy_c;
  Dims d;
  if (check_problem(&c, &pr, &d) != MNL_OK) return 0;
  return batch_eligible(d, o) ? 1 : 0;
}

}  // extern "C"
