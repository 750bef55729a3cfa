// Serving runtime: continuous batching of identification requests on one GPU.
//
// Requests (one monitoring window each: host samples, channel count, lags,
// orders, rank, precision) are queued by ssi_server_submit and return a
// ticket at once.  A dispatcher admits queued requests to free slots in
// arrival order, skipping ahead past a request that does not fit, as long as
// the device memory the slots hold stays within the budget.  Each slot owns a
// library context on its own non-blocking stream, a pinned staging buffer and
// device buffers for y and the outputs, all grown on demand and kept; a slot
// thread copies y to the device, enqueues the identification, copies the
// outputs back and marks the request done.  Work of different slots overlaps
// on the device, and a request that arrives while others run is admitted as
// soon as a slot and memory free up.
//
// Memory accounting is exact for what the server holds: a slot holds its
// context workspace and one buffer for y and the outputs, each grown to the
// largest request it ran (the workspace with the context's growth margin).
// Admitting request r to idle slot s needs  used - hold(s) + hold'(s, r) <=
// budget, with hold'(s, r) what s will hold after running r.  If no idle
// slot qualifies but one would after releasing its buffers, that slot is
// reset first, so a request that fits the budget alone is never starved by
// idle slots.
#include "../../include/ssicov.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

namespace {

thread_local std::string g_srv_error;

ssi_status srv_fail(ssi_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_srv_error = buf;
  return s;
}

using Clock = std::chrono::steady_clock;

size_t round_up(size_t b) { return (b + 255) & ~size_t(255); }

// Device output buffer sizes of one request, in the ssi_output order.
struct OutSizes {
  size_t sigma, count, f, xi, mu, phi, flags;
  size_t total() const {
    return round_up(sigma) + round_up(count) + round_up(f) + round_up(xi) + round_up(mu) +
           round_up(phi) + round_up(flags);
  }
};

OutSizes out_sizes(const ssi_layout &lay) {
  OutSizes o{};
  const size_t nl = lay.n_lags, no = lay.n_orders, cap = lay.pole_cap;
  o.sigma = sizeof(double) * nl * lay.sigma_per_lag;
  o.count = sizeof(int32_t) * nl * no;
  o.f = sizeof(double) * nl * cap;
  o.xi = sizeof(double) * nl * cap;
  o.mu = 2 * sizeof(double) * nl * cap;
  o.phi = 2 * sizeof(float) * nl * cap * lay.l;
  o.flags = sizeof(int32_t) * nl * no;
  return o;
}

struct Request {
  uint64_t ticket = 0;
  ssi_params params{};
  std::vector<int32_t> lags;
  int32_t l = 0;
  int64_t n = 0;
  std::vector<float> y;          // l x n, dense (ld n)
  ssi_layout layout{};
  size_t footprint = 0;          // ssi_footprint: ws_need + margin + io_need
  size_t ws_need = 0;            // workspace of one identification
  size_t io_need = 0;            // y and output buffers
  // result
  enum State { QUEUED, RUNNING, DONE } state = QUEUED;
  ssi_status status = SSI_OK;
  std::string error;
  Clock::time_point t_submit, t_start, t_done;
  int slot = -1;
  std::vector<double> sigma, f, xi, mu;
  std::vector<int32_t> count, flags;
  std::vector<float> phi;
  ssi_host_result host{};
};

struct Slot {
  int index = 0;
  ssi_ctx *ctx = nullptr;
  hipStream_t stream = nullptr;
  size_t cap = 0;                // device bytes held or reserved (workspace + io)
  size_t ws_cap = 0;             // context workspace held
  char *io_dev = nullptr;        // y, then the output buffers
  size_t io_cap = 0;
  float *pinned = nullptr;
  size_t pinned_cap = 0;
  std::shared_ptr<Request> job;
  std::thread th;
};

}  // namespace

struct ssi_server {
  int device = 0;
  size_t budget = 0;
  size_t used = 0;               // sum of slot capacities
  std::mutex mu;
  std::condition_variable cv_work;     // slots and dispatcher wait here
  std::condition_variable cv_done;     // ssi_server_wait
  std::deque<std::shared_ptr<Request>> queue;
  std::map<uint64_t, std::shared_ptr<Request>> all;
  std::vector<std::unique_ptr<Slot>> slots;
  uint64_t next_ticket = 1;
  bool stop = false;
  Clock::time_point t0;
  int running = 0;
  ssi_server_stats stats{};
  std::thread dispatcher;
};

namespace {

double us_since(const ssi_server *s, Clock::time_point t) {
  return std::chrono::duration<double, std::micro>(t - s->t0).count();
}

// Grow a device buffer (contents discarded).
hipError_t grow(void **p, size_t *cap, size_t need) {
  if (need <= *cap) return hipSuccess;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  *cap = 0;
  hipError_t e = hipMalloc(p, need);
  if (e == hipSuccess) *cap = need;
  return e;
}

// Runs one admitted request on its slot.  Called without the server lock.
void execute(ssi_server *S, Slot &sl, Request &r) {
  auto set_err = [&r](ssi_status st, const std::string &msg) {
    r.status = st;
    r.error = msg;
  };
  hipError_t e = hipSetDevice(S->device);
  const size_t ybytes = sizeof(float) * (size_t)r.l * (size_t)r.n;
  const OutSizes os = out_sizes(r.layout);
  if (e == hipSuccess) e = grow((void **)&sl.io_dev, &sl.io_cap, r.io_need);
  float *y_dev = reinterpret_cast<float *>(sl.io_dev);
  if (e == hipSuccess && ybytes > sl.pinned_cap) {
    if (sl.pinned) (void)hipHostFree(sl.pinned);
    sl.pinned = nullptr;
    sl.pinned_cap = 0;
    e = hipHostMalloc((void **)&sl.pinned, ybytes, hipHostMallocDefault);
    if (e == hipSuccess) sl.pinned_cap = ybytes;
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    set_err(SSI_ENOMEM, std::string("slot buffers: ") + hipGetErrorString(e));
    return;
  }
  std::memcpy(sl.pinned, r.y.data(), ybytes);
  e = hipMemcpyAsync(y_dev, sl.pinned, ybytes, hipMemcpyHostToDevice, sl.stream);
  if (e != hipSuccess) {
    set_err(SSI_EDEVICE, std::string("H2D: ") + hipGetErrorString(e));
    return;
  }
  char *q = sl.io_dev + round_up(ybytes);
  ssi_output out{};
  out.sigma = reinterpret_cast<double *>(q);  q += round_up(os.sigma);
  out.count = reinterpret_cast<int32_t *>(q); q += round_up(os.count);
  out.f = reinterpret_cast<double *>(q);      q += round_up(os.f);
  out.xi = reinterpret_cast<double *>(q);     q += round_up(os.xi);
  out.mu = reinterpret_cast<double *>(q);     q += round_up(os.mu);
  out.phi = reinterpret_cast<float *>(q);     q += round_up(os.phi);
  out.flags = reinterpret_cast<int32_t *>(q);
  r.params.lags = r.lags.data();
  ssi_status st = ssi_identify(sl.ctx, y_dev, r.l, r.n, r.n, &r.params, &out);
  if (st == SSI_OK) st = ssi_synchronize(sl.ctx);
  if (st != SSI_OK) {
    set_err(st, ssi_last_error());
    return;
  }
  r.sigma.resize(os.sigma / sizeof(double));
  r.count.resize(os.count / sizeof(int32_t));
  r.f.resize(os.f / sizeof(double));
  r.xi.resize(os.xi / sizeof(double));
  r.mu.resize(os.mu / sizeof(double));
  r.phi.resize(os.phi / sizeof(float));
  r.flags.resize(os.flags / sizeof(int32_t));
  struct { void *h; const void *d; size_t b; } cp[] = {
      {r.sigma.data(), out.sigma, os.sigma}, {r.count.data(), out.count, os.count},
      {r.f.data(), out.f, os.f},             {r.xi.data(), out.xi, os.xi},
      {r.mu.data(), out.mu, os.mu},          {r.phi.data(), out.phi, os.phi},
      {r.flags.data(), out.flags, os.flags}};
  for (auto &c : cp) {
    e = hipMemcpyAsync(c.h, c.d, c.b, hipMemcpyDeviceToHost, sl.stream);
    if (e != hipSuccess) break;
  }
  if (e == hipSuccess) e = hipStreamSynchronize(sl.stream);
  if (e != hipSuccess) {
    set_err(SSI_EDEVICE, std::string("D2H: ") + hipGetErrorString(e));
    return;
  }
  r.host.layout = r.layout;
  r.host.sigma = r.sigma.data();
  r.host.count = r.count.data();
  r.host.f = r.f.data();
  r.host.xi = r.xi.data();
  r.host.mu = r.mu.data();
  r.host.phi = r.phi.data();
  r.host.flags = r.flags.data();
}

void slot_loop(ssi_server *S, Slot *sl) {
  (void)hipSetDevice(S->device);
  for (;;) {
    std::shared_ptr<Request> job;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_work.wait(lk, [&] { return S->stop || sl->job; });
      if (!sl->job) return;          // stopping and idle
      job = sl->job;
    }
    execute(S, *sl, *job);
    {
      std::lock_guard<std::mutex> lk(S->mu);
      job->t_done = Clock::now();
      job->state = Request::DONE;
      // the slot keeps its buffers: its capacity is what ssi_identify's
      // workspace and the request's buffers needed
      sl->ws_cap = ssi_workspace_bytes(sl->ctx);
      const size_t held = sl->ws_cap + sl->io_cap;
      S->used = S->used - sl->cap + held;
      sl->cap = held;
      S->stats.peak_bytes = std::max<uint64_t>(S->stats.peak_bytes, S->used);
      sl->job.reset();
      --S->running;
      ++S->stats.completed;
      if (job->status != SSI_OK) ++S->stats.failed;
    }
    S->cv_work.notify_all();
    S->cv_done.notify_all();
  }
}

// What slot s holds after running r (the context grows its workspace to
// need + need / 8 when need exceeds what it has).
size_t hold_after(const Slot &s, const Request &r) {
  const size_t ws = s.ws_cap >= r.ws_need ? s.ws_cap : r.ws_need + (r.ws_need >> 3);
  return ws + std::max(s.io_cap, r.io_need);
}

// Release an idle slot's device buffers (new context, no io buffer).
bool reset_slot(ssi_server *S, Slot &s) {
  ssi_destroy(s.ctx);
  s.ctx = nullptr;
  if (s.io_dev) (void)hipFree(s.io_dev);
  s.io_dev = nullptr;
  s.io_cap = 0;
  s.ws_cap = 0;
  S->used -= s.cap;
  s.cap = 0;
  return ssi_create(S->device, s.stream, &s.ctx) == SSI_OK;
}

void dispatch_loop(ssi_server *S) {
  (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    if (S->stop) return;
    bool admitted = false;
    for (auto it = S->queue.begin(); it != S->queue.end() && !admitted; ++it) {
      const auto &r = *it;
      // the idle slot that needs the least extra memory for r; failing that,
      // an idle slot that would fit r once its buffers are released
      Slot *best = nullptr, *reset = nullptr;
      size_t best_used = 0;
      for (auto &sp : S->slots) {
        if (sp->job || !sp->ctx) continue;
        const size_t u = S->used - sp->cap + hold_after(*sp, *r);
        if (u <= S->budget && (!best || u < best_used)) {
          best = sp.get();
          best_used = u;
        }
        if (!reset && S->used - sp->cap + r->footprint <= S->budget) reset = sp.get();
      }
      if (!best && reset) {
        if (!reset_slot(S, *reset)) continue;
        best = reset;
        best_used = S->used + hold_after(*reset, *r);
      }
      if (!best) continue;
      // reserve the memory now; the slot settles its exact holding at the end
      S->used = best_used;
      best->cap = hold_after(*best, *r);
      S->stats.peak_bytes = std::max<uint64_t>(S->stats.peak_bytes, S->used);
      r->state = Request::RUNNING;
      r->slot = best->index;
      r->t_start = Clock::now();
      best->job = r;
      ++S->running;
      S->stats.peak_inflight = std::max<int32_t>(S->stats.peak_inflight, S->running);
      S->queue.erase(it);
      admitted = true;
    }
    if (admitted) {
      S->cv_work.notify_all();
      continue;
    }
    if (!S->queue.empty() && S->running == 0) {
      // Nothing runs and nothing fits: idle slots together hold too much.
      // Release them all; if that frees nothing, the head cannot run at all.
      bool freed = false;
      for (auto &sp : S->slots)
        if (sp->cap > 0) freed = reset_slot(S, *sp) || freed;
      if (freed) continue;
      auto r = S->queue.front();
      S->queue.pop_front();
      r->status = SSI_ENOMEM;
      r->error = "request does not fit the memory budget";
      r->t_start = r->t_done = Clock::now();
      r->state = Request::DONE;
      ++S->stats.completed;
      ++S->stats.failed;
      S->cv_done.notify_all();
      continue;
    }
    S->cv_work.wait(lk);
  }
}

}  // namespace

extern "C" {

ssi_status ssi_footprint(const ssi_params *p, int32_t l, int64_t n, size_t *bytes) {
  if (!bytes) return srv_fail(SSI_EINVAL, "ssi_footprint: bytes is NULL");
  size_t ws = 0;
  ssi_status s = ssi_workspace_estimate(p, l, n, &ws);
  if (s != SSI_OK) return s;
  ssi_layout lay;
  s = ssi_output_layout(p, l, n, &lay);
  if (s != SSI_OK) return s;
  // the context arena grows by an eighth over what a call needs
  *bytes = ws + (ws >> 3) + round_up(sizeof(float) * (size_t)l * (size_t)n) +
           out_sizes(lay).total();
  return SSI_OK;
}

ssi_status ssi_server_create(const ssi_server_config *cfg, ssi_server **out) {
  if (!cfg || !out) return srv_fail(SSI_EINVAL, "ssi_server_create: NULL argument");
  if (cfg->max_inflight < 1 || cfg->max_inflight > 64)
    return srv_fail(SSI_EINVAL, "ssi_server_create: max_inflight must be in [1, 64]");
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || cfg->device < 0 || cfg->device >= count) {
    (void)hipGetLastError();
    return srv_fail(SSI_EDEVICE, "ssi_server_create: device %d absent", cfg->device);
  }
  if (hipSetDevice(cfg->device) != hipSuccess)
    return srv_fail(SSI_EDEVICE, "ssi_server_create: hipSetDevice failed");
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess)
    return srv_fail(SSI_EDEVICE, "ssi_server_create: hipMemGetInfo failed");
  auto S = std::make_unique<ssi_server>();
  S->device = cfg->device;
  S->budget = cfg->hbm_budget ? std::min(cfg->hbm_budget, free_b) : free_b / 10 * 8;
  S->t0 = Clock::now();
  for (int i = 0; i < cfg->max_inflight; ++i) {
    auto sl = std::make_unique<Slot>();
    sl->index = i;
    if (hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking) != hipSuccess ||
        ssi_create(cfg->device, sl->stream, &sl->ctx) != SSI_OK) {
      for (auto &o : S->slots) {
        ssi_destroy(o->ctx);
        (void)hipStreamDestroy(o->stream);
      }
      if (sl->stream) (void)hipStreamDestroy(sl->stream);
      return srv_fail(SSI_EDEVICE, "ssi_server_create: slot %d: %s", i, ssi_last_error());
    }
    S->slots.push_back(std::move(sl));
  }
  ssi_server *raw = S.release();
  for (auto &sl : raw->slots) sl->th = std::thread(slot_loop, raw, sl.get());
  raw->dispatcher = std::thread(dispatch_loop, raw);
  *out = raw;
  return SSI_OK;
}

void ssi_server_destroy(ssi_server *S) {
  if (!S) return;
  {
    // let admitted and queued work finish
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv_done.wait(lk, [&] { return S->queue.empty() && S->running == 0; });
    S->stop = true;
  }
  S->cv_work.notify_all();
  S->dispatcher.join();
  for (auto &sl : S->slots) sl->th.join();
  (void)hipSetDevice(S->device);
  for (auto &sl : S->slots) {
    ssi_destroy(sl->ctx);
    (void)hipStreamDestroy(sl->stream);
    if (sl->io_dev) (void)hipFree(sl->io_dev);
    if (sl->pinned) (void)hipHostFree(sl->pinned);
  }
  delete S;
}

ssi_status ssi_server_submit(ssi_server *S, const float *y, int32_t l, int64_t n, int64_t ldy,
                             const ssi_params *p, uint64_t *ticket) {
  if (!S || !y || !p || !ticket) return srv_fail(SSI_EINVAL, "ssi_server_submit: NULL argument");
  if (ldy < n) return srv_fail(SSI_EINVAL, "ssi_server_submit: ldy < n");
  ssi_status s = ssi_validate(p, l, n);
  if (s != SSI_OK) return srv_fail(s, "%s", ssi_last_error());
  if (p->omega)
    return srv_fail(SSI_EINVAL, "ssi_server_submit: requests draw their sketch from the seed "
                                "(omega must be NULL)");
  auto r = std::make_shared<Request>();
  r->params = *p;
  r->lags.assign(p->lags, p->lags + p->n_lags);
  r->params.lags = r->lags.data();
  r->l = l;
  r->n = n;
  s = ssi_output_layout(&r->params, l, n, &r->layout);
  if (s != SSI_OK) return srv_fail(s, "%s", ssi_last_error());
  s = ssi_footprint(&r->params, l, n, &r->footprint);
  if (s == SSI_OK) s = ssi_workspace_estimate(&r->params, l, n, &r->ws_need);
  if (s != SSI_OK) return srv_fail(s, "%s", ssi_last_error());
  r->io_need = round_up(sizeof(float) * (size_t)l * (size_t)n) + out_sizes(r->layout).total();
  if (r->footprint > S->budget)
    return srv_fail(SSI_ENOMEM, "ssi_server_submit: request needs %zu bytes, budget is %zu",
                    r->footprint, S->budget);
  r->y.resize((size_t)l * (size_t)n);
  for (int32_t a = 0; a < l; ++a)
    std::memcpy(r->y.data() + (size_t)a * n, y + (size_t)a * ldy, sizeof(float) * n);
  {
    std::lock_guard<std::mutex> lk(S->mu);
    r->ticket = S->next_ticket++;
    r->t_submit = Clock::now();
    S->queue.push_back(r);
    S->all[r->ticket] = r;
    ++S->stats.submitted;
    *ticket = r->ticket;
  }
  S->cv_work.notify_all();
  return SSI_OK;
}

static void fill_info(const ssi_server *S, const Request &r, ssi_request_info *info) {
  if (!info) return;
  info->status = r.status;
  info->slot = r.slot;
  info->t_submit_us = us_since(S, r.t_submit);
  info->t_start_us = r.state != Request::QUEUED ? us_since(S, r.t_start) : -1.0;
  info->t_done_us = r.state == Request::DONE ? us_since(S, r.t_done) : -1.0;
  info->footprint = r.footprint;
}

ssi_status ssi_server_poll(ssi_server *S, uint64_t ticket, ssi_request_info *info) {
  if (!S) return srv_fail(SSI_EINVAL, "ssi_server_poll: NULL server");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->all.find(ticket);
  if (it == S->all.end()) return srv_fail(SSI_EINVAL, "ssi_server_poll: unknown ticket");
  fill_info(S, *it->second, info);
  return it->second->state == Request::DONE ? SSI_OK : SSI_EBUSY;
}

ssi_status ssi_server_wait(ssi_server *S, uint64_t ticket, ssi_request_info *info) {
  if (!S) return srv_fail(SSI_EINVAL, "ssi_server_wait: NULL server");
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->all.find(ticket);
  if (it == S->all.end()) return srv_fail(SSI_EINVAL, "ssi_server_wait: unknown ticket");
  auto r = it->second;
  S->cv_done.wait(lk, [&] { return r->state == Request::DONE; });
  fill_info(S, *r, info);
  return SSI_OK;
}

ssi_status ssi_server_result(ssi_server *S, uint64_t ticket, const ssi_host_result **res) {
  if (!S || !res) return srv_fail(SSI_EINVAL, "ssi_server_result: NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->all.find(ticket);
  if (it == S->all.end()) return srv_fail(SSI_EINVAL, "ssi_server_result: unknown ticket");
  const Request &r = *it->second;
  if (r.state != Request::DONE) return srv_fail(SSI_EBUSY, "ssi_server_result: not finished");
  if (r.status != SSI_OK) return srv_fail(r.status, "%s", r.error.c_str());
  *res = &r.host;
  return SSI_OK;
}

ssi_status ssi_server_release(ssi_server *S, uint64_t ticket) {
  if (!S) return srv_fail(SSI_EINVAL, "ssi_server_release: NULL server");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->all.find(ticket);
  if (it == S->all.end()) return srv_fail(SSI_EINVAL, "ssi_server_release: unknown ticket");
  if (it->second->state != Request::DONE)
    return srv_fail(SSI_EBUSY, "ssi_server_release: not finished");
  S->all.erase(it);
  return SSI_OK;
}

ssi_status ssi_server_get_stats(ssi_server *S, ssi_server_stats *out) {
  if (!S || !out) return srv_fail(SSI_EINVAL, "ssi_server_get_stats: NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  *out = S->stats;
  out->budget = S->budget;
  out->held_bytes = S->used;
  out->queued = (int32_t)S->queue.size();
  out->running = S->running;
  return SSI_OK;
}

const char *ssi_server_last_error(void) { return g_srv_error.c_str(); }

}  // extern "C"
