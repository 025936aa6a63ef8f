// Continuous-batching server: many independent Newton-Raphson fits in
// flight on one device, admitted by device-memory footprint.
//
// Each slot is a host thread with its own library context and HIP stream.
// A slot takes the oldest queued request once the request's footprint fits
// in the budget that running fits leave, copies the request's host data into
// memory from the server's stream-ordered pool, runs the fit on its stream,
// copies theta back and returns every byte to the pool.  Slots run
// concurrently, so the kernels of different fits overlap on the device and a
// request that arrives while others run starts as soon as a slot and memory
// are free.  The arithmetic of a fit depends only on its own shape and data
// (fixed reduction partitions), never on the slot or on the other fits.
// Small fits run in groups: a slot that admits a request the batched kernel
// takes (batch_eligible) also admits the eligible requests right behind it
// at the head of the queue (arrival order kept, up to max_group and the
// budget) and runs them as one small_fit_run, a persistent kernel with one
// workgroup per fit.  A host-only mode runs the same scheduler with no device (admitted
// requests wait a given time instead of fitting), so admission, slot and
// budget accounting can be tested anywhere.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "mnl_common.h"

namespace mnl {
namespace {

constexpr size_t kAlign = 256;
size_t al(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// Offsets of one request's device copy of its data.
struct DataLayout {
  size_t oX, oY, oZ, oC, oW, oT, total;
};

DataLayout data_layout(const Dims &d, bool has_w) {
  DataLayout L;
  const size_t N = size_t(d.N), K = size_t(d.K);
  L.oX = 0;
  L.oY = L.oX + al(N * size_t(d.p) * 8);
  L.oZ = L.oY + al(N * K * size_t(d.g) * 8);
  L.oC = L.oZ + al(N * K * size_t(d.a) * 8);
  L.oW = L.oC + al(N * 4);
  L.oT = L.oW + (has_w ? al(N * 8) : 0);
  L.total = L.oT + al(size_t(d.np) * 8);
  return L;
}

struct Request {
  int64_t id;
  mnl_problem hp;          // host pointers
  const double *theta0;    // host or NULL
  double *theta_out;       // host
  mnl_fit_opts opts;
  Dims d;
  double t_arrival;
  size_t footprint;
  bool batch;              // runs through small_fit_run
};

constexpr int kDefaultGroup = 1024;

}  // namespace
}  // namespace mnl

struct mnl_server {
  int device = 0;
  size_t budget = 0;
  int max_group = 1;
  bool host_only = false;
  double host_fit_ms = 0.0;
  hipMemPool_t pool = nullptr;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<mnl::Request> queue;
  std::deque<mnl_server_result> done;
  size_t in_use = 0, peak_in_use = 0;
  int running = 0, max_running = 0;
  int64_t next_id = 0, submitted = 0, completed = 0;
  bool stop = false;
  struct Slot {
    mnl::Ctx ctx;
    hipStream_t stream = nullptr;
    std::thread th;
  };
  std::vector<Slot *> slots;
  // footprint queries use a context of their own (host work only)
  std::mutex probe_mu;
  mnl::Ctx probe;
};

namespace mnl {
namespace {

// Run one admitted request on a slot; fills res.
void run_request(mnl_server *sv, mnl_server::Slot *sl, const Request &r,
                 mnl_server_result *res) {
  Ctx *c = &sl->ctx;
  hipStream_t s = sl->stream;
  res->status = MNL_OK;
  const Dims &d = r.d;
  const bool has_w = r.hp.w != nullptr;
  const DataLayout L = data_layout(d, has_w);
  void *buf = nullptr;
  int rc = MNL_OK;
  auto hip_fail = [&](hipError_t e, const char *what) {
    (void)hipGetLastError();
    rc = set_error(c, MNL_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
  };
  hipError_t e = hipMallocFromPoolAsync(&buf, L.total, sv->pool, s);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    rc = set_error(c, MNL_ERR_OOM, "data copy of %zu bytes", L.total);
  }
  char *b = static_cast<char *>(buf);
  mnl_problem dp = r.hp;
  auto h2d = [&](size_t off, const void *src, size_t n) -> void * {
    if (rc != MNL_OK || n == 0 || src == nullptr) return nullptr;
    hipError_t e2 = hipMemcpyAsync(b + off, src, n, hipMemcpyHostToDevice, s);
    if (e2 != hipSuccess) hip_fail(e2, "host-to-device copy");
    return b + off;
  };
  const size_t N = size_t(d.N), K = size_t(d.K);
  dp.X = (const double *)h2d(L.oX, r.hp.X, N * d.p * 8);
  dp.Y = (const double *)h2d(L.oY, r.hp.Y, N * K * d.g * 8);
  dp.Z = (const double *)h2d(L.oZ, r.hp.Z, N * K * d.a * 8);
  dp.choice = (const int32_t *)h2d(L.oC, r.hp.choice, N * 4);
  dp.w = has_w ? (const double *)h2d(L.oW, r.hp.w, N * 8) : nullptr;
  double *theta = rc == MNL_OK ? (double *)(b + L.oT) : nullptr;
  if (rc == MNL_OK) {
    if (r.theta0)
      h2d(L.oT, r.theta0, size_t(d.np) * 8);
    else if ((e = hipMemsetAsync(theta, 0, size_t(d.np) * 8, s)) != hipSuccess)
      hip_fail(e, "zero start");
  }
  if (rc == MNL_OK)
    rc = fit_impl(c, &dp, theta, r.opts, &res->info, false, s);
  if (rc == MNL_OK) {
    e = hipMemcpyAsync(r.theta_out, theta, size_t(d.np) * 8,
                       hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) hip_fail(e, "device-to-host copy");
  }
  // every byte goes back to the pool in stream order
  ctx_release(c);
  if (buf) (void)hipFreeAsync(buf, s);
  e = hipStreamSynchronize(s);
  if (e != hipSuccess && rc == MNL_OK) hip_fail(e, "stream synchronize");
  res->status = rc;
}

// Run an admitted group of batch-eligible requests as one small_fit_run:
// one pool allocation holds every request's data and, at its end, all the
// thetas (one copy back).  Fills res[0 .. n).
void run_group(mnl_server::Slot *sl, const std::vector<Request> &g,
               mnl_server_result *res) {
  Ctx *c = &sl->ctx;
  hipStream_t s = sl->stream;
  const int n = int(g.size());
  std::vector<size_t> off(n + 1), toff(n + 1);
  std::vector<DataLayout> L(n);
  off[0] = 0;
  toff[0] = 0;
  for (int f = 0; f < n; ++f) {
    L[f] = data_layout(g[f].d, g[f].hp.w != nullptr);
    off[f + 1] = off[f] + L[f].oT;   // data only; thetas go at the end
    toff[f + 1] = toff[f] + size_t(g[f].d.np);
  }
  const size_t bytes = off[n] + al(toff[n] * 8);
  void *buf = nullptr;
  int rc = MNL_OK;
  auto hip_fail = [&](hipError_t e, const char *what) {
    (void)hipGetLastError();
    if (rc == MNL_OK)
      rc = set_error(c, MNL_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
  };
  hipError_t e = hipMallocFromPoolAsync(&buf, bytes, c->pool, s);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    rc = set_error(c, MNL_ERR_OOM, "group data copy of %zu bytes", bytes);
  }
  char *b = static_cast<char *>(buf);
  double *thetas = rc == MNL_OK ? reinterpret_cast<double *>(b + off[n])
                                : nullptr;
  std::vector<mnl_problem> dp(n);
  std::vector<const double *> th0(n, nullptr);
  std::vector<double *> th(n, nullptr);
  std::vector<mnl_fit_opts> opts(n);
  std::vector<mnl_fit_info> infos(n);
  auto h2d = [&](size_t o, const void *src, size_t nb) -> void * {
    if (rc != MNL_OK || nb == 0 || src == nullptr) return nullptr;
    hipError_t e2 = hipMemcpyAsync(b + o, src, nb, hipMemcpyHostToDevice, s);
    if (e2 != hipSuccess) hip_fail(e2, "host-to-device copy");
    return b + o;
  };
  for (int f = 0; f < n && rc == MNL_OK; ++f) {
    const Request &r = g[f];
    const Dims &d = r.d;
    const size_t N = size_t(d.N), K = size_t(d.K), o = off[f];
    dp[f] = r.hp;
    dp[f].X = (const double *)h2d(o + L[f].oX, r.hp.X, N * d.p * 8);
    dp[f].Y = (const double *)h2d(o + L[f].oY, r.hp.Y, N * K * d.g * 8);
    dp[f].Z = (const double *)h2d(o + L[f].oZ, r.hp.Z, N * K * d.a * 8);
    dp[f].choice = (const int32_t *)h2d(o + L[f].oC, r.hp.choice, N * 4);
    dp[f].w = r.hp.w ? (const double *)h2d(o + L[f].oW, r.hp.w, N * 8)
                     : nullptr;
    th[f] = thetas + toff[f];
    // a start is copied into the theta slot itself (NULL: zeros)
    if (r.theta0) th0[f] = (const double *)h2d(off[n] + toff[f] * 8,
                                               r.theta0, size_t(d.np) * 8);
    opts[f] = r.opts;
  }
  if (rc == MNL_OK)
    rc = small_fit_run(c, n, dp.data(), th0.data(), opts.data(), th.data(),
                       infos.data(), s);
  std::vector<double> hth;
  if (rc == MNL_OK) {
    hth.resize(toff[n]);
    e = hipMemcpyAsync(hth.data(), thetas, toff[n] * 8, hipMemcpyDeviceToHost,
                       s);
    if (e != hipSuccess) hip_fail(e, "device-to-host copy");
  }
  ctx_release(c);
  if (buf) (void)hipFreeAsync(buf, s);
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) hip_fail(e, "stream synchronize");
  for (int f = 0; f < n; ++f) {
    res[f].status = rc;
    if (rc == MNL_OK) {
      res[f].info = infos[f];
      std::memcpy(g[f].theta_out, hth.data() + toff[f],
                  size_t(g[f].d.np) * 8);
    }
  }
}

// host-only mode: the request "runs" for host_fit_ms and returns theta = 0
// (a group together: its fits run at once, as in one batched launch)
void run_group_host(mnl_server *sv, const std::vector<Request> &g,
                    mnl_server_result *res) {
  std::this_thread::sleep_for(
      std::chrono::duration<double, std::milli>(sv->host_fit_ms));
  for (size_t f = 0; f < g.size(); ++f) {
    res[f].status = MNL_OK;
    std::memset(g[f].theta_out, 0, size_t(g[f].d.np) * 8);
    res[f].info.stop_reason = MNL_STOP_NONE;
  }
}

void slot_main(mnl_server *sv, int i) {
  mnl_server::Slot *sl = sv->slots[i];
  if (!sv->host_only) (void)hipSetDevice(sv->device);
  std::vector<Request> grp;
  std::vector<mnl_server_result> res;
  for (;;) {
    grp.clear();
    double t_admit = 0.0;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      sv->cv_work.wait(lk, [&] {
        return sv->stop || (!sv->queue.empty() &&
                            sv->in_use + sv->queue.front().footprint <=
                                sv->budget);
      });
      if (sv->stop) return;
      // the head of the queue, and with a batch-eligible head the eligible
      // requests right behind it while they fit (never one further back)
      do {
        const Request &r = sv->queue.front();
        grp.push_back(r);
        sv->queue.pop_front();
        sv->in_use += r.footprint;
      } while (grp[0].batch && int(grp.size()) < sv->max_group &&
               !sv->queue.empty() && sv->queue.front().batch &&
               sv->in_use + sv->queue.front().footprint <= sv->budget);
      sv->peak_in_use = std::max(sv->peak_in_use, sv->in_use);
      sv->running += int(grp.size());
      sv->max_running = std::max(sv->max_running, sv->running);
      // taken under the lock: admission times follow the queue order
      t_admit = now_ms();
    }
    res.assign(grp.size(), mnl_server_result{});
    for (size_t f = 0; f < grp.size(); ++f) {
      std::memset(&res[f], 0, sizeof res[f]);
      res[f].id = grp[f].id;
      res[f].slot = i;
      res[f].t_arrival = grp[f].t_arrival;
      res[f].t_admit = t_admit;
      res[f].footprint = grp[f].footprint;
    }
    if (sv->host_only) run_group_host(sv, grp, res.data());
    else if (grp[0].batch) run_group(sl, grp, res.data());
    else run_request(sv, sl, grp[0], &res[0]);
    const double t_done = now_ms();
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      for (size_t f = 0; f < grp.size(); ++f) {
        res[f].t_done = t_done;
        sv->in_use -= grp[f].footprint;
        sv->done.push_back(res[f]);
      }
      sv->running -= int(grp.size());
      sv->completed += int64_t(grp.size());
    }
    // freed memory may admit the next request on any idle slot
    sv->cv_work.notify_all();
    sv->cv_done.notify_all();
  }
}

int64_t footprint_of(Ctx *c, const mnl_problem *shape, int32_t prec) {
  Dims d;
  mnl_problem pr = *shape;
  // only the sizes matter here: stand-in pointers pass the NULL checks
  static const double dummy = 0.0;
  static const int32_t dummy_c = 0;
  pr.X = pr.Y = pr.Z = &dummy;
  pr.choice = &dummy_c;
  if (check_problem(c, &pr, &d) != MNL_OK) return -1;
  if (prec < MNL_PREC_FP64 || prec > MNL_PREC_BF16) return -1;
  size_t ws = 0;
  if (fit_workspace_footprint(c, d, prec, &ws) != MNL_OK) return -1;
  return int64_t(ws + data_layout(d, shape->w != nullptr).total);
}

}  // namespace
}  // namespace mnl

using namespace mnl;

extern "C" {

double mnl_server_now_ms(void) { return now_ms(); }

int64_t mnl_fit_footprint(const mnl_problem *shape, int32_t prec) {
  if (!shape) return -1;
  Ctx c;
  return footprint_of(&c, shape, prec);
}

int mnl_server_create(mnl_server **out, const mnl_server_opts *o) {
  if (!out || !o) return MNL_ERR_ARG;
  *out = nullptr;
  if (o->slots < 1 || o->slots > 256 || o->max_group < 0) return MNL_ERR_ARG;
  const int max_group = o->max_group == 0 ? kDefaultGroup : o->max_group;
  if (o->host_only) {
    if (o->hbm_budget == 0 || !(o->host_fit_ms >= 0.0)) return MNL_ERR_ARG;
    mnl_server *sv = new mnl_server;
    sv->host_only = true;
    sv->max_group = max_group;
    sv->host_fit_ms = o->host_fit_ms;
    sv->budget = o->hbm_budget;
    for (int i = 0; i < o->slots; ++i)
      sv->slots.push_back(new mnl_server::Slot);
    for (int i = 0; i < o->slots; ++i)
      sv->slots[i]->th = std::thread(slot_main, sv, i);
    *out = sv;
    return MNL_OK;
  }
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess) {
    (void)hipGetLastError();
    return MNL_ERR_HIP;
  }
  if (o->device < 0 || o->device >= n) return MNL_ERR_ARG;
  if (hipSetDevice(o->device) != hipSuccess) return MNL_ERR_HIP;
  mnl_server *sv = new mnl_server;
  sv->device = o->device;
  sv->max_group = max_group;
  sv->budget = o->hbm_budget;
  if (sv->budget == 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      delete sv;
      return MNL_ERR_HIP;
    }
    sv->budget = fr / 10 * 8;
  }
  hipMemPoolProps props;
  std::memset(&props, 0, sizeof props);
  props.allocType = hipMemAllocationTypePinned;
  props.handleTypes = hipMemHandleTypeNone;
  props.location.type = hipMemLocationTypeDevice;
  props.location.id = o->device;
  if (hipMemPoolCreate(&sv->pool, &props) != hipSuccess) {
    (void)hipGetLastError();
    delete sv;
    return MNL_ERR_HIP;
  }
  // keep freed memory in the pool (no return to the system at each
  // synchronisation): the budget caps what the pool holds
  uint64_t keep = sv->budget;
  (void)hipMemPoolSetAttribute(sv->pool, hipMemPoolAttrReleaseThreshold,
                               &keep);
  for (int i = 0; i < o->slots; ++i) {
    auto *sl = new mnl_server::Slot;
    sl->ctx.device = o->device;
    sl->ctx.bufs.resize(S_NSLOTS);
    if (hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking) !=
        hipSuccess) {
      (void)hipGetLastError();
      delete sl;
      mnl_server_destroy(sv);
      return MNL_ERR_HIP;
    }
    sl->ctx.pool = sv->pool;
    sl->ctx.ostream = sl->stream;
    sv->slots.push_back(sl);
  }
  for (int i = 0; i < o->slots; ++i)
    sv->slots[i]->th = std::thread(slot_main, sv, i);
  *out = sv;
  return MNL_OK;
}

void mnl_server_destroy(mnl_server *sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
    sv->queue.clear();
  }
  sv->cv_work.notify_all();
  for (auto *sl : sv->slots)
    if (sl->th.joinable()) sl->th.join();
  if (sv->host_only) {
    for (auto *sl : sv->slots) delete sl;
    delete sv;
    return;
  }
  (void)hipSetDevice(sv->device);
  for (auto *sl : sv->slots) {
    if (sl->stream) {
      (void)hipStreamSynchronize(sl->stream);
      ctx_release(&sl->ctx);
      blas_release(&sl->ctx);
      (void)hipStreamSynchronize(sl->stream);
      events_release(&sl->ctx);
      (void)hipStreamDestroy(sl->stream);
    }
    delete sl;
  }
  if (sv->pool) (void)hipMemPoolDestroy(sv->pool);
  delete sv;
}

int mnl_server_submit(mnl_server *sv, const mnl_problem *prob,
                      const double *theta0, const mnl_fit_opts *opts,
                      double *theta_out, double t_arrival, int64_t *id) {
  if (!sv || !prob || !theta_out || !id) return MNL_ERR_ARG;
  Request r;
  std::memset(&r, 0, sizeof r);
  {
    std::lock_guard<std::mutex> lk(sv->probe_mu);
    Ctx *c = &sv->probe;
    MNL_TRY(check_problem(c, prob, &r.d));
    if (opts) r.opts = *opts;
    else mnl_default_opts(&r.opts);
    MNL_TRY(check_opts(c, &r.opts));
    const int64_t f = footprint_of(c, prob, r.opts.prec);
    if (f < 0) return MNL_ERR_UNSUPPORTED;
    r.footprint = size_t(f);
    r.batch = batch_eligible(r.d, r.opts);
  }
  if (r.footprint > sv->budget) return MNL_ERR_OOM;
  r.hp = *prob;
  r.theta0 = theta0;
  r.theta_out = theta_out;
  r.t_arrival = t_arrival < 0 ? now_ms() : t_arrival;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop) return MNL_ERR_ARG;
    r.id = sv->next_id++;
    sv->submitted += 1;
    sv->queue.push_back(r);
  }
  *id = r.id;
  sv->cv_work.notify_all();
  return MNL_OK;
}

int mnl_server_wait(mnl_server *sv, mnl_server_result *out,
                    int32_t max_results, double timeout_ms, int32_t *n_out) {
  if (!sv || !n_out || (max_results > 0 && !out) || max_results < 0)
    return MNL_ERR_ARG;
  *n_out = 0;
  std::unique_lock<std::mutex> lk(sv->mu);
  auto ready = [&] { return !sv->done.empty(); };
  if (timeout_ms < 0) {
    sv->cv_done.wait(lk, ready);
  } else if (timeout_ms > 0) {
    sv->cv_done.wait_for(
        lk, std::chrono::duration<double, std::milli>(timeout_ms), ready);
  }
  int32_t k = 0;
  while (k < max_results && !sv->done.empty()) {
    out[k++] = sv->done.front();
    sv->done.pop_front();
  }
  *n_out = k;
  return MNL_OK;
}

int mnl_server_get_stats(mnl_server *sv, mnl_server_stats *st) {
  if (!sv || !st) return MNL_ERR_ARG;
  std::lock_guard<std::mutex> lk(sv->mu);
  std::memset(st, 0, sizeof *st);
  st->submitted = sv->submitted;
  st->completed = sv->completed;
  st->queued = int32_t(sv->queue.size());
  st->running = sv->running;
  st->max_running = sv->max_running;
  st->budget = sv->budget;
  st->in_use = sv->in_use;
  st->peak_in_use = sv->peak_in_use;
  return MNL_OK;
}

}  // extern "C"
