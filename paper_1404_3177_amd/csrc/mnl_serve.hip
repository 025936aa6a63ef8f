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
// A host-only mode runs the same scheduler with no device (admitted
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
};

}  // namespace
}  // namespace mnl

struct mnl_server {
  int device = 0;
  size_t budget = 0;
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

// host-only mode: the request "runs" for host_fit_ms and returns theta = 0
void run_request_host(mnl_server *sv, const Request &r,
                      mnl_server_result *res) {
  res->status = MNL_OK;
  std::this_thread::sleep_for(
      std::chrono::duration<double, std::milli>(sv->host_fit_ms));
  std::memset(r.theta_out, 0, size_t(r.d.np) * 8);
  res->info.stop_reason = MNL_STOP_NONE;
}

void slot_main(mnl_server *sv, int i) {
  mnl_server::Slot *sl = sv->slots[i];
  if (!sv->host_only) (void)hipSetDevice(sv->device);
  for (;;) {
    Request r;
    double t_admit = 0.0;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      sv->cv_work.wait(lk, [&] {
        return sv->stop || (!sv->queue.empty() &&
                            sv->in_use + sv->queue.front().footprint <=
                                sv->budget);
      });
      if (sv->stop) return;
      r = sv->queue.front();
      sv->queue.pop_front();
      sv->in_use += r.footprint;
      sv->peak_in_use = std::max(sv->peak_in_use, sv->in_use);
      sv->running += 1;
      sv->max_running = std::max(sv->max_running, sv->running);
      // taken under the lock: admission times follow the queue order
      t_admit = now_ms();
    }
    mnl_server_result res;
    std::memset(&res, 0, sizeof res);
    res.id = r.id;
    res.slot = i;
    res.t_arrival = r.t_arrival;
    res.t_admit = t_admit;
    res.footprint = r.footprint;
    if (sv->host_only) run_request_host(sv, r, &res);
    else run_request(sv, sl, r, &res);
    res.t_done = now_ms();
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      sv->in_use -= r.footprint;
      sv->running -= 1;
      sv->completed += 1;
      sv->done.push_back(res);
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
  if (o->slots < 1 || o->slots > 256) return MNL_ERR_ARG;
  if (o->host_only) {
    if (o->hbm_budget == 0 || !(o->host_fit_ms >= 0.0)) return MNL_ERR_ARG;
    mnl_server *sv = new mnl_server;
    sv->host_only = true;
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
