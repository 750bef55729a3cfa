// Host side of the C ABI declared in include/ssicov.h: argument validation,
// output layout, workspace arena and the stream-ordered stage sequence.
#include "../../include/ssicov.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "kernels.h"

// ------------------------------------------------------------ error state
namespace {

thread_local std::string g_last_error;

ssi_status fail(ssi_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

ssi_status hip_fail(hipError_t e, const char *where) {
  return fail(SSI_EDEVICE, "%s: %s", where, hipGetErrorString(e));
}

#define SSI_HIP(call)                                   \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return hip_fail(e_, #call);   \
  } while (0)

}  // namespace

// ------------------------------------------------------------------ context
constexpr int kMaxLanes = 4;      // concurrent lag streams of one identification
constexpr size_t kMaxGraphs = 8;  // captured identifications kept per context (LRU)

struct ssi_ctx {
  int device = 0;
  hipStream_t stream = nullptr;   // stream work is enqueued on right now
  hipStream_t user_stream = nullptr;   // caller's stream; nullptr = default stream
  int num_cus = 256;
  int *status = nullptr;     // device word: kernels OR in failure bits
  char *ws = nullptr;        // workspace arena
  size_t ws_cap = 0;
  size_t ws_top = 0;
  // stage timing
  bool profiling = false;
  std::vector<hipEvent_t> ev_pool;
  struct Rec { int stage; hipEvent_t a, b; };
  std::vector<Rec> recs;
  double acc_ms[SSI_STAGE_COUNT] = {};
  int32_t acc_calls[SSI_STAGE_COUNT] = {};
  // lag sweep over several streams (fork / join through events)
  int n_lanes = 1;
  hipStream_t lanes[kMaxLanes] = {};
  hipEvent_t fork_ev = nullptr;
  hipEvent_t join_ev[kMaxLanes] = {};
  // identifications captured as HIP graphs, keyed by every argument
  bool graphs = false;
  bool capturing = false;
  hipStream_t cap_stream = nullptr;
  struct Graph {
    std::vector<unsigned char> key;
    hipGraphExec_t exec;
  };
  std::vector<Graph> graph_cache;
  // product autotuning: (kind, trans, M, N, K) -> K slices
  bool autotune = false;
  int tile_rows = 128;            // FP32 x FP64 product tiles when not tuned
  // correlation product arithmetic (ssi_corr_mode)
  int corr_mode = SSI_CORR_F16X3;
  // workgroups of the identification's eigen-analysis launch (0: one per CU)
  int eig_workgroups = 0;
  std::map<std::tuple<int, int, int, int, int>, int> tuned;
  // QR sweep limit of the eigen-analysis: sweeps_per_row * max(10, n) per order
  int sweeps_per_row = 30;
  // workspace allocator (NULL: hipMalloc / hipFree)
  void *(*alloc)(size_t, void *) = nullptr;
  void (*release)(void *, void *) = nullptr;
  void *alloc_user = nullptr;
  // device output buffers of ssi_identify_result
  char *obuf = nullptr;
  size_t obuf_cap = 0;
};

namespace {

// Scoped device selection: restores the caller's current device.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

// Bump allocator over the context workspace.  Run a stage's carving once with
// base == nullptr to measure its size, reserve, then carve for real.
struct Arena {
  char *base = nullptr;
  size_t off = 0;
  template <typename T>
  T *take(size_t count) {
    size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += bytes;
    return p;
  }
};

void drop_graphs(ssi_ctx *c) {
  for (auto &g : c->graph_cache) (void)hipGraphExecDestroy(g.exec);
  c->graph_cache.clear();
}

// Device memory for the context: the caller's allocator when one is set.
hipError_t dev_alloc(ssi_ctx *c, char **p, size_t bytes) {
  if (c->alloc) {
    *p = static_cast<char *>(c->alloc(bytes, c->alloc_user));
    return *p ? hipSuccess : hipErrorOutOfMemory;
  }
  return hipMalloc(reinterpret_cast<void **>(p), bytes);
}
void dev_free(ssi_ctx *c, void *p) {
  if (!p) return;
  if (c->release)
    c->release(p, c->alloc_user);
  else
    (void)hipFree(p);
}

// Waits for everything the context enqueued (its stream and lag streams).
void drain(ssi_ctx *c) {
  (void)hipStreamSynchronize(c->stream);
  for (int s = 0; s < kMaxLanes; ++s)
    if (c->lanes[s]) (void)hipStreamSynchronize(c->lanes[s]);
}

// Reserve `bytes` of workspace for the current call (256-byte aligned).  Call
// ws_reserve once with the call's total before ws_take.
ssi_status ws_reserve(ssi_ctx *c, size_t bytes) {
  c->ws_top = 0;
  if (bytes <= c->ws_cap) return SSI_OK;
  // Work already queued may still read the old arena; captured graphs point
  // into it.
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  for (int s = 0; s < c->n_lanes; ++s)
    if (c->lanes[s]) (void)hipStreamSynchronize(c->lanes[s]);
  drop_graphs(c);
  dev_free(c, c->ws);
  c->ws = nullptr;
  c->ws_cap = 0;
  size_t cap = bytes + (bytes >> 3);
  e = dev_alloc(c, &c->ws, cap);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(SSI_ENOMEM, "workspace of %zu bytes could not be allocated", cap);
  }
  c->ws_cap = cap;
  return SSI_OK;
}

hipEvent_t take_event(ssi_ctx *c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Records an event pair around a stage when profiling is on.
struct StageTimer {
  ssi_ctx *c;
  int stage;
  hipEvent_t a = nullptr;
  StageTimer(ssi_ctx *ctx, int s) : c(ctx), stage(s) {
    if (c && c->profiling) {
      a = take_event(c);
      if (a) (void)hipEventRecord(a, c->stream);
    }
  }
  ~StageTimer() {
    if (!a) return;
    hipEvent_t b = take_event(c);
    if (!b) return;
    (void)hipEventRecord(b, c->stream);
    c->recs.push_back({stage, a, b});
  }
};

template <typename T>
T *ws_take(ssi_ctx *c, size_t count) {
  size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
  T *p = reinterpret_cast<T *>(c->ws + c->ws_top);
  c->ws_top += bytes;
  return p;
}

size_t aligned_bytes(size_t count, size_t elem) { return (count * elem + 255) & ~size_t(255); }

}  // namespace

extern "C" {

const char *ssi_last_error(void) { return g_last_error.c_str(); }

const char *ssi_status_string(ssi_status s) {
  switch (s) {
    case SSI_OK: return "ok";
    case SSI_EINVAL: return "invalid argument";
    case SSI_ENOMEM: return "out of device memory";
    case SSI_EDEVICE: return "device error";
    case SSI_ENOCONV: return "iteration limit reached";
    case SSI_EINTERNAL: return "internal error";
    case SSI_EBUSY: return "request not finished";
  }
  return "unknown status";
}

ssi_status ssi_create(int device, void *hip_stream, ssi_ctx **out) {
  if (!out) return fail(SSI_EINVAL, "ssi_create: out is NULL");
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count <= 0) {
    (void)hipGetLastError();
    return fail(SSI_EDEVICE, "ssi_create: no HIP device available");
  }
  if (device < 0 || device >= count) return fail(SSI_EDEVICE, "ssi_create: device %d absent", device);
  hipDeviceProp_t prop;
  SSI_HIP(hipGetDeviceProperties(&prop, device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(SSI_EDEVICE, "ssi_create: device %d is %s, this library is built for gfx950",
                device, prop.gcnArchName);
  DeviceGuard g(device);
  ssi_ctx *c = new ssi_ctx();
  c->device = device;
  c->num_cus = prop.multiProcessorCount;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->user_stream = c->stream;
  e = hipMalloc(&c->status, 256);
  if (e == hipSuccess) e = hipMemset(c->status, 0, 256);
  if (e != hipSuccess) {
    delete c;
    return hip_fail(e, "status word");
  }
  // device address of the static scratch of ssi_stability_noalloc (once per
  // device, while the device is current)
  uint8_t *scr = nullptr;
  e = ssi::noalloc_scratch(device, &scr);
  if (e != hipSuccess) {
    (void)hipFree(c->status);
    delete c;
    return hip_fail(e, "hipGetSymbolAddress");
  }
  *out = c;
  return SSI_OK;
}

void ssi_destroy(ssi_ctx *c) {
  if (!c) return;
  DeviceGuard g(c->device);
  (void)hipStreamSynchronize(c->stream);
  for (int s = 0; s < kMaxLanes; ++s)
    if (c->lanes[s]) {
      (void)hipStreamSynchronize(c->lanes[s]);
      (void)hipStreamDestroy(c->lanes[s]);
    }
  for (int s = 0; s < kMaxLanes; ++s)
    if (c->join_ev[s]) (void)hipEventDestroy(c->join_ev[s]);
  if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
  drop_graphs(c);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  dev_free(c, c->ws);
  dev_free(c, c->obuf);
  if (c->status) (void)hipFree(c->status);
  for (auto &r : c->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : c->ev_pool) (void)hipEventDestroy(e);
  delete c;
}

ssi_status ssi_synchronize(ssi_ctx *c) {
  if (!c) return fail(SSI_EINVAL, "ssi_synchronize: NULL context");
  DeviceGuard g(c->device);
  SSI_HIP(hipStreamSynchronize(c->stream));
  for (int s = 0; s < c->n_lanes; ++s)
    if (c->lanes[s]) SSI_HIP(hipStreamSynchronize(c->lanes[s]));
  int word = 0;
  SSI_HIP(hipMemcpy(&word, c->status, sizeof(int), hipMemcpyDeviceToHost));
  if (word) {
    SSI_HIP(hipMemset(c->status, 0, sizeof(int)));
    if (word & ssi::kStatusNonFinite)
      return fail(SSI_EINVAL, "the record holds non-finite samples (NaN or Inf): its "
                              "correlations are not finite (status bits 0x%x)", word);
    if (word & ssi::kStatusClaimCap)
      return fail(SSI_EINTERNAL, "the eigen-analysis work loop hit its pass cap "
                                 "(status bits 0x%x)", word);
    if (word & ssi::kStatusEigLimit)
      return fail(SSI_ENOCONV, "the QR iteration of at least one model order hit its sweep "
                               "limit; per-order flags mark which (status bits 0x%x)", word);
    return fail(SSI_ENOCONV, "a factorization broke down (status bits 0x%x): the matrix was "
                             "numerically singular or not finite", word);
  }
  return SSI_OK;
}

size_t ssi_workspace_bytes(const ssi_ctx *c) { return c ? c->ws_cap : 0; }

ssi_status ssi_set_profiling(ssi_ctx *c, int enable) {
  if (!c) return fail(SSI_EINVAL, "ssi_set_profiling: NULL context");
  c->profiling = enable != 0;
  return SSI_OK;
}

ssi_status ssi_set_lag_streams(ssi_ctx *c, int32_t n) {
  if (!c) return fail(SSI_EINVAL, "ssi_set_lag_streams: NULL context");
  if (n < 1 || n > kMaxLanes)
    return fail(SSI_EINVAL, "ssi_set_lag_streams: n = %d must be in [1, %d]", n, kMaxLanes);
  DeviceGuard g(c->device);
  SSI_HIP(hipStreamSynchronize(c->stream));
  if (!c->fork_ev) SSI_HIP(hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming));
  for (int s = 0; s < n; ++s) {
    if (!c->lanes[s]) SSI_HIP(hipStreamCreateWithFlags(&c->lanes[s], hipStreamNonBlocking));
    if (!c->join_ev[s]) SSI_HIP(hipEventCreateWithFlags(&c->join_ev[s], hipEventDisableTiming));
  }
  if (n != c->n_lanes) drop_graphs(c);
  c->n_lanes = n;
  return SSI_OK;
}

ssi_status ssi_set_graphs(ssi_ctx *c, int enable) {
  if (!c) return fail(SSI_EINVAL, "ssi_set_graphs: NULL context");
  DeviceGuard g(c->device);
  if (enable && !c->cap_stream)
    SSI_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  if (!enable) {
    SSI_HIP(hipStreamSynchronize(c->stream));
    drop_graphs(c);
  }
  c->graphs = enable != 0;
  return SSI_OK;
}

ssi_status ssi_set_autotune(ssi_ctx *c, int enable) {
  if (!c) return fail(SSI_EINVAL, "ssi_set_autotune: NULL context");
  c->autotune = enable != 0;
  return SSI_OK;
}

ssi_status ssi_set_product_tile_rows(ssi_ctx *c, int32_t rows) {
  if (!c) return fail(SSI_EINVAL, "ssi_set_product_tile_rows: NULL context");
  if (rows != 0 && rows != 64 && rows != 128)
    return fail(SSI_EINVAL, "ssi_set_product_tile_rows: rows = %d must be 0, 64 or 128", rows);
  const int r = rows == 64 ? 64 : 128;
  if (r != c->tile_rows) {
    DeviceGuard g(c->device);
    drain(c);
    drop_graphs(c);
  }
  c->tile_rows = r;
  return SSI_OK;
}

ssi_status ssi_set_eig_workgroups(ssi_ctx *c, int32_t n) {
  if (!c) return fail(SSI_EINVAL, "ssi_set_eig_workgroups: NULL context");
  if (n < 0) return fail(SSI_EINVAL, "ssi_set_eig_workgroups: n = %d must be >= 0", n);
  if (n != c->eig_workgroups) {
    DeviceGuard g(c->device);
    drain(c);
    drop_graphs(c);
  }
  c->eig_workgroups = n;
  return SSI_OK;
}

ssi_status ssi_set_corr_mode(ssi_ctx *c, int32_t mode) {
  if (!c) return fail(SSI_EINVAL, "ssi_set_corr_mode: NULL context");
  if (mode != SSI_CORR_FP32 && mode != SSI_CORR_BF16X6 && mode != SSI_CORR_F16X3)
    return fail(SSI_EINVAL, "ssi_set_corr_mode: unknown mode %d", mode);
  if (mode != c->corr_mode) {
    DeviceGuard g(c->device);
    (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
  }
  c->corr_mode = mode;
  return SSI_OK;
}

ssi_status ssi_set_eig_max_sweeps(ssi_ctx *c, int32_t sweeps_per_row) {
  if (!c) return fail(SSI_EINVAL, "ssi_set_eig_max_sweeps: NULL context");
  if (sweeps_per_row < 0 || sweeps_per_row > 1000)
    return fail(SSI_EINVAL, "ssi_set_eig_max_sweeps: %d not in [0, 1000]", sweeps_per_row);
  if (sweeps_per_row != c->sweeps_per_row) {
    DeviceGuard g(c->device);
    drain(c);
    drop_graphs(c);
  }
  c->sweeps_per_row = sweeps_per_row;
  return SSI_OK;
}

ssi_status ssi_set_allocator(ssi_ctx *c, void *(*alloc)(size_t, void *),
                             void (*release)(void *, void *), void *user) {
  if (!c) return fail(SSI_EINVAL, "ssi_set_allocator: NULL context");
  if ((alloc == nullptr) != (release == nullptr))
    return fail(SSI_EINVAL, "ssi_set_allocator: give both callbacks or neither");
  DeviceGuard g(c->device);
  // memory from the old allocator goes back to it before the switch
  drain(c);
  drop_graphs(c);
  dev_free(c, c->ws);
  dev_free(c, c->obuf);
  c->ws = nullptr;
  c->ws_cap = 0;
  c->obuf = nullptr;
  c->obuf_cap = 0;
  c->alloc = alloc;
  c->release = release;
  c->alloc_user = user;
  return SSI_OK;
}

int32_t ssi_tuned_splits(const ssi_ctx *c, int32_t kind, int32_t trans, int32_t m, int32_t n,
                         int32_t k) {
  if (!c) return 0;
  auto it = c->tuned.find(std::make_tuple(kind, trans, m, n, k));
  return it == c->tuned.end() ? 0 : it->second;
}

ssi_status ssi_profile_read(ssi_ctx *c, double *ms, int32_t *calls, int32_t n_stages) {
  if (!c || !ms || !calls || n_stages < 0) return fail(SSI_EINVAL, "ssi_profile_read: bad argument");
  DeviceGuard g(c->device);
  SSI_HIP(hipStreamSynchronize(c->stream));
  for (auto &r : c->recs) {
    float t = 0.f;
    SSI_HIP(hipEventElapsedTime(&t, r.a, r.b));
    c->acc_ms[r.stage] += t;
    c->acc_calls[r.stage] += 1;
    c->ev_pool.push_back(r.a);
    c->ev_pool.push_back(r.b);
  }
  c->recs.clear();
  for (int i = 0; i < n_stages; ++i) {
    ms[i] = i < SSI_STAGE_COUNT ? c->acc_ms[i] : 0.0;
    calls[i] = i < SSI_STAGE_COUNT ? c->acc_calls[i] : 0;
  }
  for (int i = 0; i < SSI_STAGE_COUNT; ++i) {
    c->acc_ms[i] = 0.0;
    c->acc_calls[i] = 0;
  }
  return SSI_OK;
}

// ------------------------------------------------------------ host helpers
double ssi_tau(int32_t jb, double fs) { return (2.0 * jb - 1.0) / fs; }

int32_t ssi_lag_rule(double fs, double f0, double factor) {
  if (!(fs > 0) || !(f0 > 0) || !(factor > 0)) return -1;
  return (int32_t)std::ceil(factor * fs / (2.0 * f0) - 1e-9);
}

int32_t ssi_default_rank(int64_t t_size) {
  if (t_size <= 0) return -1;
  const double pct = std::max(30.0 - 0.00156 * (double)t_size, 25.0);
  return (int32_t)std::ceil(pct * (double)t_size / 100.0 - 1e-9);
}

static int32_t n_orders_of(const ssi_params *p) {
  return (p->order_max - p->order_min) / p->order_step + 1;
}

ssi_status ssi_validate(const ssi_params *p, int32_t l, int64_t n) {
  if (!p) return fail(SSI_EINVAL, "params is NULL");
  if (l < 1) return fail(SSI_EINVAL, "l = %d must be >= 1", l);
  if (!(p->fs > 0.0) || !std::isfinite(p->fs)) return fail(SSI_EINVAL, "fs must be finite and > 0");
  if (p->n_lags < 1 || !p->lags) return fail(SSI_EINVAL, "need at least one lag");
  if (p->order_step < 1) return fail(SSI_EINVAL, "order_step must be >= 1");
  if (p->order_min < 1 || p->order_max < p->order_min)
    return fail(SSI_EINVAL, "need 1 <= order_min <= order_max");
  if (p->svd != SSI_SVD_FULL && p->svd != SSI_SVD_RANDOMIZED)
    return fail(SSI_EINVAL, "unknown svd mode %d", p->svd);
  if (p->prec != SSI_PREC_FP32 && p->prec != SSI_PREC_BF16 && p->prec != SSI_PREC_BF16X3 &&
      p->prec != SSI_PREC_BF16X6 && p->prec != SSI_PREC_FP8)
    return fail(SSI_EINVAL, "unknown precision %d", p->prec);
  if (p->prec != SSI_PREC_FP32 && p->svd != SSI_SVD_RANDOMIZED)
    return fail(SSI_EINVAL, "reduced-precision products apply to the randomized SVD only");
  if (p->omega && p->svd != SSI_SVD_RANDOMIZED)
    return fail(SSI_EINVAL, "a caller sketch applies to the randomized SVD only");
  if (p->refine < 0 || (p->refine > 0 && p->svd == SSI_SVD_RANDOMIZED &&
                        p->refine > p->power_iters))
    return fail(SSI_EINVAL, "refine = %d must be in [0, power_iters]", p->refine);
  if (p->omega && p->omega_ld < (int64_t)p->rank + p->oversample)
    return fail(SSI_EINVAL, "omega_ld = %lld must be >= k + p = %d", (long long)p->omega_ld,
                p->rank + p->oversample);
  for (int i = 0; i < p->n_lags; ++i) {
    const int64_t jb = p->lags[i];
    if (jb < 2) return fail(SSI_EINVAL, "lag %d: j_b = %lld must be >= 2", i, (long long)jb);
    if (i > 0 && jb <= p->lags[i - 1]) return fail(SSI_EINVAL, "lags must be strictly increasing");
    if (2 * jb - 1 >= n) return fail(SSI_EINVAL, "lag %d: 2 j_b - 1 = %lld must be < N = %lld", i,
                                     (long long)(2 * jb - 1), (long long)n);
    const int64_t m = jb * l;
    if (m > (int64_t)1 << 30) return fail(SSI_EINVAL, "Toeplitz size %lld too large", (long long)m);
    if ((int64_t)p->order_max > (int64_t)l * (jb - 1))
      return fail(SSI_EINVAL, "order_max %d exceeds l (j_b - 1) = %lld for j_b = %lld",
                  p->order_max, (long long)l * (jb - 1), (long long)jb);
    if (p->svd == SSI_SVD_RANDOMIZED) {
      if (p->rank < p->order_max) return fail(SSI_EINVAL, "rank k = %d must be >= order_max = %d",
                                              p->rank, p->order_max);
      if (p->oversample < 0 || p->power_iters < 0)
        return fail(SSI_EINVAL, "oversample and power_iters must be >= 0");
      if ((int64_t)p->rank + p->oversample > m)
        return fail(SSI_EINVAL, "k + p = %d exceeds the Toeplitz size %lld",
                    p->rank + p->oversample, (long long)m);
      if (p->rank + p->oversample > ssi::dense_max_n())
        return fail(SSI_EINVAL, "k + p = %d exceeds %d", p->rank + p->oversample,
                    ssi::dense_max_n());
    } else {
      if (m > ssi::dense_max_n())
        return fail(SSI_EINVAL, "full SVD supports Toeplitz size <= %d, got %lld",
                    ssi::dense_max_n(), (long long)m);
      if (p->order_max > m) return fail(SSI_EINVAL, "order_max exceeds the Toeplitz size");
    }
  }
  if (p->order_max > ssi::modal_max_order())
    return fail(SSI_EINVAL, "order_max must be <= %d", ssi::modal_max_order());
  return SSI_OK;
}

int32_t ssi_pole_offset(const ssi_params *p, int32_t order_index) {
  if (!p || order_index < 0) return -1;
  int32_t off = 0;
  for (int32_t o = 0; o < order_index; ++o) off += (p->order_min + o * p->order_step) / 2;
  return off;
}

ssi_status ssi_output_layout(const ssi_params *p, int32_t l, int64_t n, ssi_layout *out) {
  ssi_status s = ssi_validate(p, l, n);
  if (s != SSI_OK) return s;
  if (!out) return fail(SSI_EINVAL, "layout output is NULL");
  out->n_lags = p->n_lags;
  out->n_orders = n_orders_of(p);
  out->sigma_per_lag = p->svd == SSI_SVD_RANDOMIZED ? p->rank : p->order_max;
  out->pole_cap = ssi_pole_offset(p, out->n_orders);
  out->l = l;
  out->n_corr = 2 * p->lags[p->n_lags - 1] - 1;
  return SSI_OK;
}

}  // extern "C"

// ------------------------------------------------------ workspace planning
namespace {

bool is_device_ptr(const void *p) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice;
}

// ------------------------------------------------------------ products
// out = op(T) X with T FP32 and X FP64 (FP64 MFMA, split-K partial sums).
// Launch configuration of a range-finder product: its number of K slices
// and, for the FP32 x FP64 kernel, its output-tile height.  With autotuning
// on, the first product of each shape times every candidate configuration on
// the stream (each run computes the full, correct product) and keeps the
// fastest for later calls, which are then also safe to capture in a graph.
// A configuration is encoded as slices + kTuneTile64 for 64-row tiles.
constexpr int kTuneSplits[] = {2, 4, 6, 8, 12, 16};
constexpr int kTuneMaxSplits = 16;
constexpr int kTuneTile64 = 100;

template <typename Launch>
int tuned_splits(ssi_ctx *c, int kind, bool ta, int M, int N, int K, int planned, Launch &&run,
                 hipError_t &err, bool tiles = false) {
  const auto key = std::make_tuple(kind, ta ? 1 : 0, M, N, K);
  auto it = c->tuned.find(key);
  if (it != c->tuned.end()) return it->second;
  if (!c->autotune || c->capturing) return 0;
  hipEvent_t a = take_event(c), b = take_event(c);
  if (!a || !b) return 0;
  int best = 0;
  float best_ms = 0.f;
  int cands[2 * (1 + sizeof(kTuneSplits) / sizeof(int))];
  int nc = 0;
  cands[nc++] = planned;                        // the planner's own choice first
  for (int v : kTuneSplits)
    if (v != planned) cands[nc++] = v;
  if (tiles) {
    const int n1 = nc;
    for (int i = 0; i < n1; ++i) cands[nc++] = cands[i] + kTuneTile64;
  }
  for (int ci = 0; ci < nc; ++ci) {
    const int cand = cands[ci];
    err = run(cand);                            // warm-up
    if (err == hipSuccess) err = hipEventRecord(a, c->stream);
    for (int r = 0; r < 3 && err == hipSuccess; ++r) err = run(cand);
    if (err == hipSuccess) err = hipEventRecord(b, c->stream);
    if (err == hipSuccess) err = hipEventSynchronize(b);
    float ms = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, a, b);
    if (err != hipSuccess) break;
    if (best == 0 || ms < best_ms) {
      best = cand;
      best_ms = ms;
    }
  }
  c->ev_pool.push_back(a);
  c->ev_pool.push_back(b);
  if (err == hipSuccess && best > 0) c->tuned[key] = best;
  return best;
}

hipError_t prod_tf64(ssi_ctx *c, bool ta, const float *T, int64_t ldt, const double *X,
                     int64_t ldx, int M, int N, int K, double *part, double *out, int64_t ldo) {
  auto run = [&](int cfg) {
    const int bm = cfg >= kTuneTile64 ? 64 : 128;
    const ssi::GemmPlan gp = ssi::plan_gemm_tf64(M, N, K, c->num_cus, cfg % kTuneTile64, bm);
    hipError_t e = ssi::launch_gemm_tf64(gp, ta, T, ldt, X, ldx, M, N, K, part, c->stream);
    if (e != hipSuccess) return e;
    return ssi::launch_reduce(gp, part, M, N, 1.0, out, ldo, nullptr, 0, c->stream);
  };
  hipError_t err = hipSuccess;
  const int planned = ssi::plan_gemm_tf64(M, N, K, c->num_cus).splits;
  int cfg = tuned_splits(c, 0, ta, M, N, K, planned, run, err, true);
  if (cfg == 0 && c->tile_rows == 64) cfg = kTuneTile64;   // untuned: planned slices
  if (err != hipSuccess) return err;
  return run(cfg);
}

hipError_t prod_f64(ssi_ctx *c, bool ta, const double *A, int64_t lda, const double *B,
                    int64_t ldb, int M, int N, int K, double *part, double *out, int64_t ldo,
                    float *out32 = nullptr, int64_t ld32 = 0) {
  const ssi::GemmPlan gp = ssi::plan_gemm_f64(M, N, K, c->num_cus);
  hipError_t e = ssi::launch_gemm_f64(gp, ta, A, lda, B, ldb, M, N, K, part, c->stream);
  if (e != hipSuccess) return e;
  return ssi::launch_reduce(gp, part, M, N, 1.0, out, ldo, out32, ld32, c->stream);
}

// out = op(T) X with T and X rounded to BF16, FP32 MFMA accumulation, FP32
// split partials summed in FP64 (the reduced-precision range finder).
hipError_t prod_bf16(ssi_ctx *c, bool ta, const float *T, int64_t ldt, const double *X,
                     int64_t ldx, int M, int N, int K, int nt, uint16_t *xt, float *part,
                     double *out, int64_t ldo) {
  const ssi::BfPlan bp0 = ssi::plan_gemm_tbf16(M, N, K, c->num_cus, 0, nt);
  hipError_t e = ssi::launch_pack_bf16(bp0, X, ldx, K, N, xt, c->stream);
  if (e != hipSuccess) return e;
  auto run = [&](int splits) {
    const ssi::BfPlan bp = ssi::plan_gemm_tbf16(M, N, K, c->num_cus, splits, nt);
    hipError_t e2 = ssi::launch_gemm_tbf16(bp, ta, T, ldt, xt, M, N, K, part, c->stream);
    if (e2 != hipSuccess) return e2;
    return ssi::launch_reduce_f32(bp, part, M, N, out, ldo, c->stream);
  };
  hipError_t err = hipSuccess;
  const int splits = tuned_splits(c, nt, ta, M, N, K, bp0.splits, run, err);
  if (err != hipSuccess) return err;
  return run(splits);
}

// Partial-sum elements of a range-finder product: the planned K slices, or
// the largest autotuning candidate when tuning may run.
size_t part_tf64(int M, int N, int K, int cus, bool tune = false) {
  size_t e = ssi::plan_gemm_tf64(M, N, K, cus).part_elems();
  if (tune) e = std::max(e, ssi::plan_gemm_tf64(M, N, K, cus, kTuneMaxSplits).part_elems());
  return e;
}
size_t part_f64(int M, int N, int K, int cus) { return ssi::plan_gemm_f64(M, N, K, cus).part_elems(); }

// BF16 products per FP32 product of a reduced-precision mode
int bf16_terms(int prec) {
  return prec == SSI_PREC_BF16X6 ? 6 : (prec == SSI_PREC_BF16X3 ? 3 : 1);
}

// ------------------------------------------------------------ randomized SVD
struct RsvdBufs {
  double *om, *ya, *yb, *gm, *rinv, *lws, *evals, *evecs, *dws, *part;
  uint16_t *xt;        // BF16 X^T of the reduced-precision products
  float *part32;       // their FP32 split partials
  // FP8 products: T quantized along rows (q8, s8) and along columns (q8t,
  // s8t), X along columns (x8, xs8)
  uint8_t *q8, *s8, *q8t, *s8t, *x8, *xs8;
  int ell;
  int prec;
};

RsvdBufs carve_rsvd(Arena &a, ssi_ctx *c, int64_t m, int ell, int k, int prec,
                    const int64_t *m_all = nullptr, int n_m = 0) {
  RsvdBufs b{};
  b.ell = ell;
  b.prec = prec;
  const int mi = (int)m, cu = c->num_cus;
  b.om = a.take<double>((size_t)m * ell);
  b.ya = a.take<double>((size_t)m * ell);
  b.yb = a.take<double>((size_t)m * ell);
  b.gm = a.take<double>((size_t)ell * ell);
  b.rinv = a.take<double>((size_t)ell * ell);
  b.lws = a.take<double>((size_t)ell * ell);
  b.evals = a.take<double>(ell);
  b.evecs = a.take<double>((size_t)ell * ell);
  b.dws = a.take<double>(ssi::dense_ws_doubles(ell));
  size_t part = 0;
  for (int i = 0; i < (m_all ? n_m : 1); ++i) {
    const int mm = m_all ? (int)m_all[i] : mi;
    part = std::max({part, part_tf64(mm, ell, mm, cu, c->autotune), part_f64(ell, ell, mm, cu),
                     part_f64(mm, ell, ell, cu), part_f64(mm, k, ell, cu)});
  }
  b.part = a.take<double>(part);
  if (prec == SSI_PREC_FP8) {
    size_t q = 0, sc = 0, xq = 0, xs = 0, p32 = 0;
    for (int i = 0; i < (m_all ? n_m : 1); ++i) {
      const int mm = m_all ? (int)m_all[i] : mi;
      const ssi::Fp8Plan fp = ssi::plan_gemm_fp8(mm, ell, mm, cu);
      q = std::max(q, (size_t)mm * fp.kp);
      sc = std::max(sc, fp.scale_bytes(mm));
      xq = std::max(xq, (size_t)fp.n_pad * fp.kp);
      xs = std::max(xs, fp.scale_bytes(fp.n_pad));
      p32 = std::max(p32, fp.part_elems());
    }
    b.q8 = a.take<uint8_t>(q);
    b.q8t = a.take<uint8_t>(q);
    b.s8 = a.take<uint8_t>(sc);
    b.s8t = a.take<uint8_t>(sc);
    b.x8 = a.take<uint8_t>(xq);
    b.xs8 = a.take<uint8_t>(xs);
    b.part32 = a.take<float>(p32);
  } else if (prec != SSI_PREC_FP32) {
    const int nt = bf16_terms(prec);
    size_t xt = 0, p32 = 0;
    for (int i = 0; i < (m_all ? n_m : 1); ++i) {
      const int mm = m_all ? (int)m_all[i] : mi;
      const ssi::BfPlan bp = ssi::plan_gemm_tbf16(mm, ell, mm, cu, 0, nt);
      xt = std::max(xt, bp.xt_elems());
      p32 = std::max(p32, bp.part_elems());
      if (c->autotune)
        p32 = std::max(p32,
                       ssi::plan_gemm_tbf16(mm, ell, mm, cu, kTuneMaxSplits, nt).part_elems());
    }
    b.xt = a.take<uint16_t>(xt);
    b.part32 = a.take<float>(p32);
  }
  return b;
}

// out = op(T) X on the FP8 operands (T quantized by quant_t8 for this SVD).
hipError_t prod_fp8(ssi_ctx *c, RsvdBufs &b, bool ta, const double *X, int64_t ldx, int M,
                    int N, int K, double *out, int64_t ldo) {
  const ssi::Fp8Plan fp = ssi::plan_gemm_fp8(M, N, K, c->num_cus);
  hipError_t e = ssi::launch_quant_cols_f64(X, ldx, K, N, fp.kp, fp.n_pad, b.x8, b.xs8,
                                            c->stream);
  if (e != hipSuccess) return e;
  e = ssi::launch_gemm_fp8(fp, ta ? b.q8t : b.q8, ta ? b.s8t : b.s8, b.x8, b.xs8, M, N, b.part32,
                           c->stream);
  if (e != hipSuccess) return e;
  ssi::BfPlan rp{};
  rp.splits = fp.splits;
  rp.split_stride = fp.split_stride;
  rp.ldc = fp.ldc;
  return ssi::launch_reduce_f32(rp, b.part32, M, N, out, ldo, c->stream);
}

// T (m x m) quantized to FP8 along its rows and along its columns.
hipError_t quant_t8(ssi_ctx *c, RsvdBufs &b, const float *t, int64_t ldt, int m) {
  const ssi::Fp8Plan fp = ssi::plan_gemm_fp8(m, b.ell, m, c->num_cus);
  hipError_t e = ssi::launch_quant_rows_f32(t, ldt, m, m, fp.kp, b.q8, b.s8, c->stream);
  if (e != hipSuccess) return e;
  return ssi::launch_quant_cols_f32(t, ldt, m, m, fp.kp, m, b.q8t, b.s8t, c->stream);
}

// Basis of the columns of cur (m x ell, FP64) by shifted CholeskyQR: pass 1
// with a diagonal shift that keeps the Cholesky factor defined for
// ill-conditioned input, then plain passes.  passes = 3 (shifted
// CholeskyQR2) gives an orthonormal Q; passes = 1 keeps the span with a
// well-conditioned basis, which is all the power iteration needs between
// products.  Returns the buffer holding Q.
double *orthonormalize(ssi_ctx *c, RsvdBufs &b, double *cur, double *nxt, int64_t m,
                       int passes, hipError_t &err) {
  const int ell = b.ell, mi = (int)m;
  const double shift_rel = 11.0 * ((double)m * ell + (double)ell * (ell + 1)) * 0x1.0p-53;
  for (int pass = 0; pass < passes && err == hipSuccess; ++pass) {
    err = prod_f64(c, true, cur, ell, cur, ell, ell, ell, mi, b.part, b.gm, ell);
    if (err != hipSuccess) break;
    err = ssi::launch_chol_inv(b.gm, ell, ell, pass == 0 ? shift_rel : 0.0, b.rinv, ell, b.lws,
                               b.dws, c->status, c->stream);
    if (err != hipSuccess) break;
    err = prod_f64(c, false, cur, ell, b.rinv, ell, mi, ell, ell, b.part, nxt, ell);
    std::swap(cur, nxt);
  }
  return cur;
}

ssi_status run_rsvd(ssi_ctx *c, RsvdBufs &b, const float *t, int64_t m, int64_t ldt, int k,
                    int p, int q, const float *omega, int64_t ldo, uint64_t seed,
                    uint32_t stream, double *u, double *sigma, int refine = 0) {
  const int ell = k + p, mi = (int)m;
  hipError_t e;
  {
    StageTimer tm(c, SSI_STAGE_SKETCH);
    if (omega)
      e = ssi::launch_convert_f32_f64(omega, ldo, mi, ell, b.om, ell, c->stream);
    else
      e = ssi::launch_sketch(seed, stream, m, ell, b.om, ell, c->stream);
  }
  if (e != hipSuccess) return hip_fail(e, "sketch");
  // Y = T Omega, Q = orth(Y)
  {
    StageTimer tm(c, SSI_STAGE_PRODUCTS);
    if (b.prec == SSI_PREC_FP8) {
      e = quant_t8(c, b, t, ldt, mi);
      if (e == hipSuccess) e = prod_fp8(c, b, false, b.om, ell, mi, ell, mi, b.ya, ell);
    } else if (b.prec != SSI_PREC_FP32)
      e = prod_bf16(c, false, t, ldt, b.om, ell, mi, ell, mi, bf16_terms(b.prec),
                    b.xt, b.part32, b.ya, ell);
    else
      e = prod_tf64(c, false, t, ldt, b.om, ell, mi, ell, mi, b.part, b.ya, ell);
  }
  if (e != hipSuccess) return hip_fail(e, "Y = T Omega");
  double *Q;
  {
    StageTimer tm(c, SSI_STAGE_ORTH);
    Q = orthonormalize(c, b, b.ya, b.yb, m, q == 0 ? 3 : 1, e);
  }
  if (e != hipSuccess) return hip_fail(e, "orthonormalize");
  // power iterations: Q = orth(T^T Q), Q = orth(T Q)
  for (int it = 0; it < q; ++it) {
    for (int side = 0; side < 2; ++side) {
      double *other = (Q == b.ya) ? b.yb : b.ya;
      {
        StageTimer tm(c, SSI_STAGE_PRODUCTS);
        // the last `refine` iterations of a reduced-precision range finder
        // run in full precision
        if (b.prec == SSI_PREC_FP8 && it < q - refine)
          e = prod_fp8(c, b, side == 0, Q, ell, mi, ell, mi, other, ell);
        else if (b.prec != SSI_PREC_FP32 && it < q - refine)
          e = prod_bf16(c, side == 0, t, ldt, Q, ell, mi, ell, mi,
                        bf16_terms(b.prec), b.xt, b.part32, other, ell);
        else
          e = prod_tf64(c, side == 0, t, ldt, Q, ell, mi, ell, mi, b.part, other, ell);
      }
      if (e != hipSuccess) return hip_fail(e, "power iteration product");
      {
        StageTimer tm(c, SSI_STAGE_ORTH);
        const bool final_basis = it == q - 1 && side == 1;
        Q = orthonormalize(c, b, other, Q, m, final_basis ? 3 : 1, e);
      }
      if (e != hipSuccess) return hip_fail(e, "orthonormalize");
    }
  }
  // P^T = T^T Q; G = P P^T; G = U~ S^2 U~^T; U = Q U~[:, :k].  The projection
  // is always taken in full precision (FP32 T, FP64 Q and accumulation): a
  // reduced-precision range finder only perturbs the basis Q, and P = Q^T T
  // of that basis is then exact to FP64 rounding.
  double *pt = (Q == b.ya) ? b.yb : b.ya;
  {
    StageTimer tm(c, SSI_STAGE_PRODUCTS);
    e = prod_tf64(c, true, t, ldt, Q, ell, mi, ell, mi, b.part, pt, ell);
  }
  if (e != hipSuccess) return hip_fail(e, "P^T = T^T Q");
  StageTimer tm_small(c, SSI_STAGE_SMALL_SVD);
  e = prod_f64(c, true, pt, ell, pt, ell, ell, ell, mi, b.part, b.gm, ell);
  if (e != hipSuccess) return hip_fail(e, "P P^T");
  e = ssi::launch_sym_eig(b.gm, ell, ell, k, b.evals, b.evecs, ell, b.dws, c->status,
                          c->stream);
  if (e != hipSuccess) return hip_fail(e, "small eigen-decomposition");
  e = ssi::launch_sqrt_clamp(b.evals, k, sigma, c->stream);
  if (e != hipSuccess) return hip_fail(e, "sigma");
  e = prod_f64(c, false, Q, ell, b.evecs, ell, mi, k, ell, b.part, u, k);
  if (e != hipSuccess) return hip_fail(e, "U = Q U~");
  return SSI_OK;
}

// ------------------------------------------------------------ full SVD
struct FullBufs {
  double *tt, *gm, *evals, *evecs, *dws, *part;
};

FullBufs carve_full(Arena &a, ssi_ctx *c, int m) {
  FullBufs b{};
  b.tt = a.take<double>((size_t)m * m);
  b.gm = a.take<double>((size_t)m * m);
  b.evals = a.take<double>(m);
  b.evecs = a.take<double>((size_t)m * m);
  b.dws = a.take<double>(ssi::dense_ws_doubles(m));
  b.part = a.take<double>(part_f64(m, m, m, c->num_cus));
  return b;
}

// Left singular vectors and singular values of T from the FP64 symmetric
// eigen-decomposition of T T^T.
ssi_status run_svd_full(ssi_ctx *c, FullBufs &b, const float *t, int m, int64_t ldt, int k,
                        double *u, double *sigma) {
  hipError_t e = ssi::launch_transpose_f32_f64(t, ldt, m, m, b.tt, m, c->stream);
  if (e != hipSuccess) return hip_fail(e, "transpose");
  e = prod_f64(c, true, b.tt, m, b.tt, m, m, m, m, b.part, b.gm, m);
  if (e != hipSuccess) return hip_fail(e, "T T^T");
  e = ssi::launch_sym_eig(b.gm, m, m, k, b.evals, b.evecs, m, b.dws, c->status, c->stream);
  if (e != hipSuccess) return hip_fail(e, "eigen-decomposition");
  e = ssi::launch_sqrt_clamp(b.evals, k, sigma, c->stream);
  if (e != hipSuccess) return hip_fail(e, "sigma");
  e = hipMemcpy2DAsync(u, (size_t)k * 8, b.evecs, (size_t)m * 8, (size_t)k * 8, (size_t)m,
                       hipMemcpyDeviceToDevice, c->stream);
  if (e != hipSuccess) return hip_fail(e, "copy U");
  return SSI_OK;
}

// ------------------------------------------------------------ modal stage
// Per-lane buffers of the shift least squares and the order matrices X_n
// (reused by the lags of a lane one after another).
struct ModalLane {
  double *gt, *hm, *rinv, *lws, *w, *dws, *part, *xbuf;
};

// Buffers of the eigen-analysis, one slot per lag of the launch (lag g at g
// times each buffer's per-lag size), plus the per-wave scratch of the launch.
struct ModalShared {
  ssi::ModalSizes sz;
  int n_lags, ldu;
  double *hbuf, *vref, *taus, *evbuf, *gscr;
  double *tf, *txi, *tmu, *tphi, *uhead;
  int *npole, *pidx, *flags_tmp;
  int *queue, *done;
};

ModalLane carve_modal_lane(Arena &a, ssi_ctx *c, int64_t m, int l, const ssi_params *p) {
  ModalLane b{};
  const int kk = p->order_max;               // leading columns used by the orders
  const int cu = c->num_cus;
  const ssi::ModalSizes sz = ssi::modal_sizes(p->order_min, kk, p->order_step, l);
  b.gt = a.take<double>((size_t)kk * kk);
  b.hm = a.take<double>((size_t)kk * kk);
  b.rinv = a.take<double>((size_t)kk * kk);
  b.lws = a.take<double>((size_t)kk * kk);
  b.w = a.take<double>((size_t)kk * kk);
  b.dws = a.take<double>(ssi::dense_ws_doubles(kk));
  b.part = a.take<double>(std::max(part_f64(kk, kk, (int)(m - l), cu), part_f64(kk, kk, kk, cu)));
  b.xbuf = a.take<double>(sz.sq);
  return b;
}

// ldu: columns of U (k); the first l rows of each lag's U are copied,
// transposed, into uhead, so the mode shapes of every lag are read from one
// place.
ModalShared carve_modal_shared(Arena &a, int l, const ssi_params *p, int ldu, int n_lags) {
  ModalShared b{};
  b.sz = ssi::modal_sizes(p->order_min, p->order_max, p->order_step, l);
  b.n_lags = n_lags;
  b.ldu = ldu;
  const size_t g = (size_t)n_lags;
  b.hbuf = a.take<double>(g * b.sz.sq);
  b.vref = a.take<double>(g * b.sz.vref);
  b.taus = a.take<double>(g * b.sz.taus);
  b.evbuf = a.take<double>(g * 2 * b.sz.vec);
  b.gscr = a.take<double>(g * b.sz.n_orders * b.sz.francis_glb);
  b.tf = a.take<double>(g * b.sz.poles);
  b.txi = a.take<double>(g * b.sz.poles);
  b.tmu = a.take<double>(g * 2 * b.sz.poles);
  b.tphi = a.take<double>(g * 2 * b.sz.poles * l);
  b.uhead = a.take<double>(g * l * ldu);
  b.npole = a.take<int>(g * b.sz.n_orders);
  b.pidx = a.take<int>(g * b.sz.vec);
  b.flags_tmp = a.take<int>(g * b.sz.n_orders);
  b.queue = a.take<int>(b.sz.queue_ints);
  b.done = a.take<int>(g * b.sz.n_orders);
  return b;
}

ssi::ModalArgs modal_args(ssi_ctx *c, const ModalShared &sh, int l, const ssi_params *p) {
  ssi::ModalArgs a{};
  a.sizes = sh.sz;
  a.nmin = p->order_min;
  a.step = p->order_step;
  a.n_lags = sh.n_lags;
  a.ldw = p->order_max;
  a.ldu = sh.ldu;
  a.l = l;
  a.fs = p->fs;
  a.u = sh.uhead;
  a.hbuf = sh.hbuf; a.vref = sh.vref; a.taus = sh.taus;
  a.evbuf = sh.evbuf; a.gscr = sh.gscr;
  a.tf = sh.tf; a.txi = sh.txi; a.tmu = sh.tmu; a.tphi = sh.tphi;
  a.npole = sh.npole; a.pidx = sh.pidx; a.flags_tmp = sh.flags_tmp;
  a.queue = sh.queue; a.done = sh.done; a.status = c->status;
  a.sweeps_per_row = c->sweeps_per_row;
  return a;
}

// Shift least squares and Hessenberg forms of every order of one lag into
// lag slot `slot` of sh.  U: m x k (ld k).
ssi_status run_modal_prep(ssi_ctx *c, ModalLane &b, ModalShared &sh, const double *u, int64_t m,
                          int k, int l, const ssi_params *p, int slot) {
  const int kk = p->order_max, mt = (int)(m - l);
  hipError_t e;
  StageTimer tm_ls(c, SSI_STAGE_SHIFT_LS);
  // Gram matrices of the shifted observability blocks (leading kk columns)
  e = prod_f64(c, true, u, k, u, k, kk, kk, mt, b.part, b.gt, kk);
  if (e != hipSuccess) return hip_fail(e, "U_top^T U_top");
  e = prod_f64(c, true, u, k, u + (int64_t)l * k, k, kk, kk, mt, b.part, b.hm, kk);
  if (e != hipSuccess) return hip_fail(e, "U_top^T U_bot");
  e = ssi::launch_chol_inv(b.gt, kk, kk, 0.0, b.rinv, kk, b.lws, b.dws, c->status, c->stream);
  if (e != hipSuccess) return hip_fail(e, "Cholesky of U_top^T U_top");
  e = prod_f64(c, true, b.rinv, kk, b.hm, kk, kk, kk, kk, b.part, b.w, kk);
  if (e != hipSuccess) return hip_fail(e, "W = R^-T H");
  ssi::ModalArgs a = modal_args(c, sh, l, p);
  a.rinv = b.rinv;
  a.w = b.w;
  a.xbuf = b.xbuf;
  e = ssi::launch_modal_prep(a, slot, c->stream);
  if (e != hipSuccess) return hip_fail(e, "Hessenberg reduction");
  // mode shapes use U[0:l, :n], read transposed
  e = ssi::launch_mode_head(u, k, l, sh.uhead + (int64_t)slot * l * sh.ldu, c->stream);
  if (e != hipSuccess) return hip_fail(e, "mode-shape rows");
  return SSI_OK;
}

// Eigen-analysis, poles and sorting of the sh.n_lags prepared lags in one
// launch; slot g goes to lag slot lag0 + g of out.
ssi_status run_modal_eig(ssi_ctx *c, ModalShared &sh, int l, const ssi_params *p, int lag0,
                         const ssi_output *out, int eig_grid) {
  const int no = sh.sz.n_orders;
  const int64_t pole_cap = sh.sz.poles;
  ssi::ModalArgs a = modal_args(c, sh, l, p);
  a.eig_grid = eig_grid;
  a.count = out->count + (int64_t)lag0 * no;
  a.flags = out->flags + (int64_t)lag0 * no;
  a.f = out->f + (int64_t)lag0 * pole_cap;
  a.xi = out->xi + (int64_t)lag0 * pole_cap;
  a.mu = out->mu + 2 * (int64_t)lag0 * pole_cap;
  a.phi = out->phi + 2 * (int64_t)lag0 * pole_cap * l;
  StageTimer tm_eig(c, SSI_STAGE_EIG);
  const hipError_t e = ssi::launch_modal_eig(a, c->stream);
  if (e != hipSuccess) return hip_fail(e, "modal kernels");
  return SSI_OK;
}

// ------------------------------------------------------------ identification
// Buffers of one lag stream ("lane"): the lags i with i % n_lanes == lane run
// on it one after another, so each lane is sized for its largest lag.
struct LaneBufs {
  float *t;
  double *u, *sig;
  RsvdBufs rb;
  FullBufs fb;
  ModalLane mb;
};

struct IdentBufs {
  float *ystage;                      // device copy of a host record (l x n), or NULL
  ssi::CorrPlan cp;
  double *corr_part;
  uint16_t *planes;                   // BF16 parts of the record (BF16x6 correlations)
  float *r;
  int n_lanes;
  LaneBufs lane[kMaxLanes];
  ModalShared ms;                     // every lag's eigen-analysis, one launch
};

int lanes_for(const ssi_ctx *c, const ssi_params *p) { return std::min(c->n_lanes, p->n_lags); }

IdentBufs carve_identify(Arena &a, ssi_ctx *c, int l, int64_t n, const ssi_params *p,
                         bool stage_y = false) {
  IdentBufs b{};
  if (stage_y) b.ystage = a.take<float>((size_t)l * n);
  const int L = 2 * p->lags[p->n_lags - 1] - 1;
  b.cp = ssi::plan_correlate(l, n, L, c->num_cus, c->corr_mode);
  b.corr_part = a.take<double>(b.cp.partial_elems);
  b.planes = a.take<uint16_t>(b.cp.planes_elems);
  b.r = a.take<float>((size_t)L * l * l);
  b.n_lanes = lanes_for(c, p);
  const int kcols = p->svd == SSI_SVD_RANDOMIZED ? p->rank : p->order_max;
  for (int s = 0; s < b.n_lanes; ++s) {
    LaneBufs &lb = b.lane[s];
    std::vector<int64_t> ms;
    for (int i = s; i < p->n_lags; i += b.n_lanes) ms.push_back((int64_t)p->lags[i] * l);
    const int64_t mmax = *std::max_element(ms.begin(), ms.end());
    const int64_t ldt = (mmax + 3) & ~int64_t(3);
    lb.t = a.take<float>((size_t)mmax * ldt);
    lb.u = a.take<double>((size_t)mmax * kcols);
    lb.sig = a.take<double>(kcols);
    if (p->svd == SSI_SVD_RANDOMIZED)
      lb.rb = carve_rsvd(a, c, mmax, p->rank + p->oversample, p->rank, p->prec, ms.data(),
                         (int)ms.size());
    else
      lb.fb = carve_full(a, c, (int)mmax);
    lb.mb = carve_modal_lane(a, c, mmax, l, p);
  }
  b.ms = carve_modal_shared(a, l, p, kcols, p->n_lags);
  return b;
}

// Enqueues one lag (Toeplitz, SVD, shift least squares and Hessenberg forms
// into lag slot i of ms) on c->stream; the eigen-analysis of all lags follows
// in one launch.
ssi_status run_lag(ssi_ctx *c, LaneBufs &b, ModalShared &ms, const float *r, int l,
                   const ssi_params *p, int i, const ssi_output *out) {
  const int jb = p->lags[i];
  const int64_t m = (int64_t)jb * l;
  const int64_t ldt = (m + 3) & ~int64_t(3);
  const int kcols = p->svd == SSI_SVD_RANDOMIZED ? p->rank : p->order_max;
  hipError_t e;
  {
    StageTimer tm(c, SSI_STAGE_TOEPLITZ);
    e = ssi::launch_toeplitz(r, l, jb, b.t, ldt, c->stream);
  }
  if (e != hipSuccess) return hip_fail(e, "Toeplitz");
  ssi_status s;
  if (p->svd == SSI_SVD_RANDOMIZED)
    // a caller sketch gives every lag its leading m rows
    s = run_rsvd(c, b.rb, b.t, m, ldt, p->rank, p->oversample, p->power_iters, p->omega,
                 p->omega_ld, p->seed, (uint32_t)i, b.u, b.sig, p->refine);
  else
    s = run_svd_full(c, b.fb, b.t, (int)m, ldt, kcols, b.u, b.sig);
  if (s != SSI_OK) return s;
  e = hipMemcpyAsync(out->sigma + (int64_t)i * kcols, b.sig, sizeof(double) * kcols,
                     hipMemcpyDeviceToDevice, c->stream);
  if (e != hipSuccess) return hip_fail(e, "sigma copy");
  return run_modal_prep(c, b.mb, ms, b.u, m, kcols, l, p, i);
}

// Points c->stream at another stream for the lifetime of the guard.
struct StreamSwap {
  ssi_ctx *c;
  hipStream_t saved;
  StreamSwap(ssi_ctx *ctx, hipStream_t s) : c(ctx), saved(ctx->stream) { c->stream = s; }
  ~StreamSwap() { c->stream = saved; }
};

ssi_status run_identify(ssi_ctx *c, IdentBufs &b, const float *y, int l, int64_t n,
                        int64_t ldy, const ssi_params *p, const ssi_output *out) {
  const int L = 2 * p->lags[p->n_lags - 1] - 1;
  hipError_t e;
  if (b.cp.mode != SSI_CORR_FP32) {
    StageTimer tm(c, SSI_STAGE_CORR_SPLIT);
    e = ssi::launch_correlate_split(b.cp, y, l, n, ldy, b.planes, c->stream);
    if (e != hipSuccess) return hip_fail(e, "correlation split");
  }
  {
    StageTimer tm(c, SSI_STAGE_CORR_MFMA);
    e = ssi::launch_correlate_mfma(b.cp, y, l, n, ldy, L, b.corr_part, b.planes, c->stream);
  }
  if (e != hipSuccess) return hip_fail(e, "correlations");
  {
    StageTimer tm(c, SSI_STAGE_CORR_REDUCE);
    e = ssi::launch_correlate_reduce(b.cp, l, n, L, b.corr_part, b.planes, b.r, c->status,
                                     c->stream);
  }
  if (e != hipSuccess) return hip_fail(e, "correlation reduction");
  if (b.n_lanes == 1) {
    for (int i = 0; i < p->n_lags; ++i) {
      ssi_status s = run_lag(c, b.lane[0], b.ms, b.r, l, p, i, out);
      if (s != SSI_OK) return s;
    }
  } else {
    // Several lanes: fork after the correlations and join before the
    // eigen-analysis.  Lags of different lanes overlap on the device (the
    // latency-bound factorizations of one lag run beside the products of
    // the next).
    hipStream_t main = c->stream;
    SSI_HIP(hipEventRecord(c->fork_ev, main));
    for (int s = 0; s < b.n_lanes; ++s) SSI_HIP(hipStreamWaitEvent(c->lanes[s], c->fork_ev, 0));
    ssi_status st = SSI_OK;
    for (int i = 0; i < p->n_lags && st == SSI_OK; ++i) {
      const int s = i % b.n_lanes;
      StreamSwap sw(c, c->lanes[s]);
      st = run_lag(c, b.lane[s], b.ms, b.r, l, p, i, out);
    }
    for (int s = 0; s < b.n_lanes; ++s) {
      SSI_HIP(hipEventRecord(c->join_ev[s], c->lanes[s]));
      SSI_HIP(hipStreamWaitEvent(main, c->join_ev[s], 0));
    }
    if (st != SSI_OK) return st;
  }
  // every (lag, order) of the diagram in one persistent launch
  return run_modal_eig(c, b.ms, l, p, 0, out, c->eig_workgroups);
}

}  // namespace

extern "C" {

ssi_status ssi_correlate(ssi_ctx *c, const float *y, int32_t l, int64_t n, int64_t ldy,
                         int32_t n_corr, float *r) {
  if (!c) return fail(SSI_EINVAL, "ssi_correlate: NULL context");
  if (!y || !r) return fail(SSI_EINVAL, "ssi_correlate: NULL buffer");
  if (l < 1 || n < 2 || ldy < n || n_corr < 1 || n_corr >= n)
    return fail(SSI_EINVAL, "ssi_correlate: need l >= 1, ldy >= n, 1 <= n_corr < n");
  if ((int64_t)l * n_corr > (int64_t)1 << 30) return fail(SSI_EINVAL, "ssi_correlate: too many rows");
  DeviceGuard g(c->device);
  if (!is_device_ptr(y) || !is_device_ptr(r))
    return fail(SSI_EINVAL, "ssi_correlate: y and r must be device pointers");
  const ssi::CorrPlan cp = ssi::plan_correlate(l, n, n_corr, c->num_cus, c->corr_mode);
  ssi_status s = ws_reserve(c, aligned_bytes(cp.partial_elems, sizeof(double)) +
                                   aligned_bytes(cp.planes_elems, sizeof(uint16_t)));
  if (s != SSI_OK) return s;
  double *partial = ws_take<double>(c, cp.partial_elems);
  uint16_t *planes = ws_take<uint16_t>(c, cp.planes_elems);
  if (cp.mode != SSI_CORR_FP32) {
    StageTimer tm(c, SSI_STAGE_CORR_SPLIT);
    SSI_HIP(ssi::launch_correlate_split(cp, y, l, n, ldy, planes, c->stream));
  }
  {
    StageTimer tm(c, SSI_STAGE_CORR_MFMA);
    SSI_HIP(ssi::launch_correlate_mfma(cp, y, l, n, ldy, n_corr, partial, planes, c->stream));
  }
  StageTimer tm(c, SSI_STAGE_CORR_REDUCE);
  SSI_HIP(ssi::launch_correlate_reduce(cp, l, n, n_corr, partial, planes, r, c->status,
                                       c->stream));
  return SSI_OK;
}

ssi_status ssi_toeplitz(ssi_ctx *c, const float *r, int32_t l, int32_t jb, float *t,
                        int64_t ldt) {
  if (!c) return fail(SSI_EINVAL, "ssi_toeplitz: NULL context");
  if (!r || !t) return fail(SSI_EINVAL, "ssi_toeplitz: NULL buffer");
  if (l < 1 || jb < 1 || (int64_t)jb * l > (int64_t)1 << 30 || ldt < (int64_t)jb * l)
    return fail(SSI_EINVAL, "ssi_toeplitz: need l, jb >= 1 and ldt >= jb l");
  DeviceGuard g(c->device);
  if (!is_device_ptr(r) || !is_device_ptr(t))
    return fail(SSI_EINVAL, "ssi_toeplitz: r and t must be device pointers");
  StageTimer tm(c, SSI_STAGE_TOEPLITZ);
  SSI_HIP(ssi::launch_toeplitz(r, l, jb, t, ldt, c->stream));
  return SSI_OK;
}

ssi_status ssi_sketch(ssi_ctx *c, uint64_t seed, uint32_t stream, int64_t m, int32_t ell,
                      float *omega, int64_t ldo) {
  if (!c) return fail(SSI_EINVAL, "ssi_sketch: NULL context");
  if (!omega || m < 1 || ell < 1 || ldo < ell)
    return fail(SSI_EINVAL, "ssi_sketch: need m, ell >= 1, ldo >= ell and a buffer");
  DeviceGuard g(c->device);
  if (!is_device_ptr(omega)) return fail(SSI_EINVAL, "ssi_sketch: omega must be a device pointer");
  SSI_HIP(ssi::launch_sketch(seed, stream, m, ell, omega, ldo, c->stream));
  return SSI_OK;
}

ssi_status ssi_workspace_estimate(const ssi_params *p, int32_t l, int64_t n, size_t *bytes) {
  ssi_status s = ssi_validate(p, l, n);
  if (s != SSI_OK) return s;
  if (!bytes) return fail(SSI_EINVAL, "bytes is NULL");
  ssi_ctx probe_ctx;
  Arena a;
  carve_identify(a, &probe_ctx, l, n, p);
  *bytes = a.off;
  return SSI_OK;
}

ssi_status ssi_rsvd(ssi_ctx *c, const float *t, int64_t m, int64_t ldt, int32_t k, int32_t p,
                    int32_t q, int32_t prec, int32_t refine, const float *omega, uint64_t seed,
                    uint32_t stream, double *u, double *sigma) {
  if (!c) return fail(SSI_EINVAL, "ssi_rsvd: NULL context");
  if (!t || !u || !sigma) return fail(SSI_EINVAL, "ssi_rsvd: NULL buffer");
  if (m < 1 || ldt < m || k < 1 || p < 0 || q < 0 || (int64_t)k + p > m)
    return fail(SSI_EINVAL, "ssi_rsvd: need 1 <= k, 0 <= p, 0 <= q, k + p <= m <= ldt");
  if (refine < 0 || refine > q)
    return fail(SSI_EINVAL, "ssi_rsvd: refine = %d must be in [0, q]", refine);
  if (k + p > ssi::dense_max_n())
    return fail(SSI_EINVAL, "ssi_rsvd: k + p = %d exceeds %d", k + p, ssi::dense_max_n());
  if (m > INT32_MAX / 2) return fail(SSI_EINVAL, "ssi_rsvd: m too large");
  if (prec != SSI_PREC_FP32 && prec != SSI_PREC_BF16 && prec != SSI_PREC_BF16X3 &&
      prec != SSI_PREC_BF16X6 && prec != SSI_PREC_FP8)
    return fail(SSI_EINVAL, "ssi_rsvd: unknown precision %d", prec);
  DeviceGuard g(c->device);
  if (!is_device_ptr(t) || !is_device_ptr(u) || !is_device_ptr(sigma) ||
      (omega && !is_device_ptr(omega)))
    return fail(SSI_EINVAL, "ssi_rsvd: buffers must be device pointers");
  Arena probe;
  carve_rsvd(probe, c, m, k + p, k, prec);
  ssi_status s = ws_reserve(c, probe.off);
  if (s != SSI_OK) return s;
  Arena a{c->ws, 0};
  RsvdBufs b = carve_rsvd(a, c, m, k + p, k, prec);
  return run_rsvd(c, b, t, m, ldt, k, p, q, omega, k + p, seed, stream, u, sigma, refine);
}

ssi_status ssi_svd_full(ssi_ctx *c, const float *t, int64_t m, int64_t ldt, int32_t k, double *u,
                        double *sigma) {
  if (!c) return fail(SSI_EINVAL, "ssi_svd_full: NULL context");
  if (!t || !u || !sigma) return fail(SSI_EINVAL, "ssi_svd_full: NULL buffer");
  if (m < 1 || ldt < m || k < 1 || k > m)
    return fail(SSI_EINVAL, "ssi_svd_full: need 1 <= k <= m <= ldt");
  if (m > ssi::dense_max_n())
    return fail(SSI_EINVAL, "ssi_svd_full: m = %lld exceeds %d", (long long)m,
                ssi::dense_max_n());
  DeviceGuard g(c->device);
  if (!is_device_ptr(t) || !is_device_ptr(u) || !is_device_ptr(sigma))
    return fail(SSI_EINVAL, "ssi_svd_full: buffers must be device pointers");
  Arena probe;
  carve_full(probe, c, (int)m);
  ssi_status s = ws_reserve(c, probe.off);
  if (s != SSI_OK) return s;
  Arena a{c->ws, 0};
  FullBufs b = carve_full(a, c, (int)m);
  return run_svd_full(c, b, t, (int)m, ldt, k, u, sigma);
}

ssi_status ssi_modal(ssi_ctx *c, const double *u, const double *sigma, int64_t m, int32_t k,
                     int32_t l, const ssi_params *p, int32_t lag_index, const ssi_output *out) {
  (void)sigma;   // the eigenvalues of A do not depend on S (similarity); kept for the ABI
  if (!c || !u || !p || !out) return fail(SSI_EINVAL, "ssi_modal: NULL argument");
  if (l < 1 || m <= l || k < 1) return fail(SSI_EINVAL, "ssi_modal: need 1 <= l < m, k >= 1");
  if (p->order_step < 1 || p->order_min < 1 || p->order_max < p->order_min ||
      p->order_max > k || p->order_max > m - l || p->order_max > ssi::modal_max_order())
    return fail(SSI_EINVAL, "ssi_modal: need 1 <= order_min <= order_max <= min(k, m - l, %d)",
                ssi::modal_max_order());
  if (!(p->fs > 0.0)) return fail(SSI_EINVAL, "ssi_modal: fs must be > 0");
  if (lag_index < 0 || lag_index >= p->n_lags) return fail(SSI_EINVAL, "ssi_modal: bad lag index");
  DeviceGuard g(c->device);
  Arena probe;
  carve_modal_lane(probe, c, m, l, p);
  carve_modal_shared(probe, l, p, k, 1);
  ssi_status s = ws_reserve(c, probe.off);
  if (s != SSI_OK) return s;
  Arena a{c->ws, 0};
  ModalLane b = carve_modal_lane(a, c, m, l, p);
  ModalShared sh = carve_modal_shared(a, l, p, k, 1);
  s = run_modal_prep(c, b, sh, u, m, k, l, p, 0);
  if (s != SSI_OK) return s;
  return run_modal_eig(c, sh, l, p, lag_index, out, 0);
}

}  // extern "C"

namespace {

// Shared checks and launch of ssi_stability and ssi_stability_noalloc; `hc`
// is the per-slot scratch (slots bytes), from the workspace or the static
// array.  get_hc is called after validation with the slot count.
template <typename GetHc>
ssi_status stability_impl(ssi_ctx *c, const char *name, const ssi_params *p, int32_t l,
                          const ssi_output *out, const ssi_stability_params *sp, double *mpc,
                          double *mpd, uint8_t *flags, GetHc &&get_hc) {
  if (!c || !p || !out || !sp || !mpc || !mpd || !flags)
    return fail(SSI_EINVAL, "%s: NULL argument", name);
  if (!out->count || !out->f || !out->xi || !out->phi)
    return fail(SSI_EINVAL, "%s: NULL output buffer", name);
  if (l < 1 || p->n_lags < 1 || p->order_step < 1 || p->order_min < 1 ||
      p->order_max < p->order_min)
    return fail(SSI_EINVAL, "%s: bad sizes", name);
  if (!(sp->xi_max > 0.0) || !(sp->alpha_f >= 0.0) || !(sp->alpha_xi >= 0.0) ||
      !(sp->alpha_mac >= 0.0))
    return fail(SSI_EINVAL, "%s: thresholds must be non-negative (xi_max > 0)", name);
  DeviceGuard g(c->device);
  const int n_orders = n_orders_of(p);
  const int pole_cap = ssi_pole_offset(p, n_orders);
  const size_t slots = (size_t)p->n_lags * pole_cap;
  uint8_t *hc = nullptr;
  ssi_status s = get_hc(slots, &hc);
  if (s != SSI_OK) return s;
  ssi::StabilityArgs a{};
  a.n_lags = p->n_lags;
  a.n_orders = n_orders;
  a.nmin = p->order_min;
  a.step = p->order_step;
  a.pole_cap = pole_cap;
  a.l = l;
  a.count = out->count;
  a.f = out->f;
  a.xi = out->xi;
  a.phi = out->phi;
  a.xi_max = sp->xi_max;
  a.mpc_min = sp->mpc_min;
  a.mpd_max = sp->mpd_max;
  a.alpha_f = sp->alpha_f;
  a.alpha_xi = sp->alpha_xi;
  a.alpha_mac = sp->alpha_mac;
  a.mpc = mpc;
  a.mpd = mpd;
  a.hc = hc;
  a.flags = flags;
  SSI_HIP(ssi::launch_stability(a, c->stream));
  return SSI_OK;
}

}  // namespace

extern "C" {

ssi_status ssi_stability(ssi_ctx *c, const ssi_params *p, int32_t l, const ssi_output *out,
                         const ssi_stability_params *sp, double *mpc, double *mpd,
                         uint8_t *flags) {
  return stability_impl(c, "ssi_stability", p, l, out, sp, mpc, mpd, flags,
                        [c](size_t slots, uint8_t **hc) {
                          ssi_status s = ws_reserve(c, aligned_bytes(slots, 1));
                          if (s == SSI_OK) *hc = ws_take<uint8_t>(c, slots);
                          return s;
                        });
}

ssi_status ssi_stability_noalloc(ssi_ctx *c, const ssi_params *p, int32_t l,
                                 const ssi_output *out, const ssi_stability_params *sp,
                                 double *mpc, double *mpd, uint8_t *flags) {
  return stability_impl(c, "ssi_stability_noalloc", p, l, out, sp, mpc, mpd, flags,
                        [c](size_t slots, uint8_t **hc) {
                          const size_t cap = ssi::noalloc_stability_slots();
                          if (slots > cap)
                            return fail(SSI_EINVAL,
                                        "ssi_stability_noalloc: %zu pole slots exceed the "
                                        "fixed scratch of %zu",
                                        slots, cap);
                          // every slot of the scratch that the kernels read is
                          // written first by quality_kernel: nothing to clear
                          const hipError_t e = ssi::noalloc_scratch(c->device, hc);
                          if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress");
                          return SSI_OK;
                        });
}

int64_t ssi_stability_noalloc_max_slots(void) { return (int64_t)ssi::noalloc_stability_slots(); }

ssi_status ssi_identify(ssi_ctx *c, const float *y, int32_t l, int64_t n, int64_t ldy,
                        const ssi_params *p, const ssi_output *out) {
  if (!c || !y || !p || !out) return fail(SSI_EINVAL, "ssi_identify: NULL argument");
  ssi_status s = ssi_validate(p, l, n);
  if (s != SSI_OK) return s;
  if (ldy < n) return fail(SSI_EINVAL, "ssi_identify: ldy < n");
  if (!out->sigma || !out->count || !out->f || !out->xi || !out->mu || !out->phi || !out->flags)
    return fail(SSI_EINVAL, "ssi_identify: NULL output buffer");
  DeviceGuard g(c->device);
  if (p->omega && !is_device_ptr(p->omega))
    return fail(SSI_EINVAL, "ssi_identify: omega must be a device pointer");
  // a host record (pinned or pageable) is copied into the workspace first
  const bool host_y = !is_device_ptr(y);
  Arena probe;
  carve_identify(probe, c, l, n, p, host_y);
  s = ws_reserve(c, probe.off);
  if (s != SSI_OK) return s;
  Arena a{c->ws, 0};
  IdentBufs b = carve_identify(a, c, l, n, p, host_y);
  if (host_y) {
    SSI_HIP(hipMemcpy2DAsync(b.ystage, (size_t)n * sizeof(float), y, (size_t)ldy * sizeof(float),
                             (size_t)n * sizeof(float), (size_t)l, hipMemcpyHostToDevice,
                             c->stream));
    y = b.ystage;
    ldy = n;
  }
  // graphs replay device work only: a host record always runs eagerly
  if (!c->graphs || host_y) return run_identify(c, b, y, l, n, ldy, p, out);

  // Graph mode: every argument (pointers included) keys a captured graph of
  // the whole identification.  The first call with a key runs eagerly (any
  // autotuning happens there) and then captures; later calls launch the
  // graph on the caller's stream.
  std::vector<unsigned char> key;
  auto put = [&key](const void *v, size_t nb) {
    const unsigned char *q = static_cast<const unsigned char *>(v);
    key.insert(key.end(), q, q + nb);
  };
  const void *ptrs[] = {y, out->sigma, out->count, out->f, out->xi, out->mu, out->phi,
                        out->flags, c->ws};
  put(ptrs, sizeof ptrs);
  put(&l, sizeof l);
  put(&n, sizeof n);
  put(&ldy, sizeof ldy);
  ssi_params pc = *p;
  pc.lags = nullptr;
  put(&pc, sizeof pc);
  put(p->lags, sizeof(int32_t) * p->n_lags);
  put(&c->n_lanes, sizeof c->n_lanes);
  for (size_t gi = 0; gi < c->graph_cache.size(); ++gi)
    if (c->graph_cache[gi].key == key) {
      // most recently used first
      std::rotate(c->graph_cache.begin(), c->graph_cache.begin() + gi,
                  c->graph_cache.begin() + gi + 1);
      SSI_HIP(hipGraphLaunch(c->graph_cache.front().exec, c->stream));
      return SSI_OK;
    }
  s = run_identify(c, b, y, l, n, ldy, p, out);
  if (s != SSI_OK) return s;
  // the lanes join the capture below; let the eager run drain from them first
  SSI_HIP(hipStreamSynchronize(c->stream));
  for (int ln = 0; ln < c->n_lanes; ++ln)
    if (c->lanes[ln]) SSI_HIP(hipStreamSynchronize(c->lanes[ln]));
  hipGraph_t graph = nullptr;
  {
    StreamSwap sw(c, c->cap_stream);
    const bool prof = c->profiling;
    c->profiling = false;
    c->capturing = true;
    hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) {
      c->profiling = prof;
      c->capturing = false;
      return hip_fail(e, "hipStreamBeginCapture");
    }
    s = run_identify(c, b, y, l, n, ldy, p, out);
    e = hipStreamEndCapture(c->cap_stream, &graph);
    c->profiling = prof;
    c->capturing = false;
    if (s != SSI_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return s;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  }
  hipGraphExec_t exec = nullptr;
  hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  if (c->graph_cache.size() >= kMaxGraphs) {
    // evict the least recently used graph once nothing of it can be in flight
    drain(c);
    (void)hipGraphExecDestroy(c->graph_cache.back().exec);
    c->graph_cache.pop_back();
  }
  c->graph_cache.insert(c->graph_cache.begin(), {std::move(key), exec});
  return SSI_OK;
}

}  // extern "C"

// ------------------------------------------------------------ host results
// Host copy of one identification's outputs (ssi_output layout), owned by the
// library until ssi_result_free.
struct ssi_result {
  ssi_layout lay{};
  int32_t nmin = 0, step = 1;
  std::vector<int32_t> offs;          // pole slot offset of each order within a lag
  std::vector<double> sigma, f, xi, mu;
  std::vector<int32_t> count, flags;
  std::vector<float> phi;
};

namespace {

// Output sizes from the parameters alone (the record length only enters
// validation).
ssi_status layout_of(const ssi_params *p, int32_t l, ssi_layout *lay) {
  if (!p || !p->lags || p->n_lags < 1 || l < 1 || p->order_step < 1 || p->order_min < 1 ||
      p->order_max < p->order_min || (p->svd != SSI_SVD_FULL && p->svd != SSI_SVD_RANDOMIZED))
    return fail(SSI_EINVAL, "invalid parameters for an output layout");
  lay->n_lags = p->n_lags;
  lay->n_orders = n_orders_of(p);
  lay->sigma_per_lag = p->svd == SSI_SVD_RANDOMIZED ? p->rank : p->order_max;
  lay->pole_cap = ssi_pole_offset(p, lay->n_orders);
  lay->l = l;
  lay->n_corr = 2 * p->lags[p->n_lags - 1] - 1;
  return SSI_OK;
}

struct OutSizes {
  size_t sigma, count, poles, phi;
  explicit OutSizes(const ssi_layout &L)
      : sigma((size_t)L.n_lags * L.sigma_per_lag), count((size_t)L.n_lags * L.n_orders),
        poles((size_t)L.n_lags * L.pole_cap), phi((size_t)L.n_lags * L.pole_cap * L.l * 2) {}
};

}  // namespace

extern "C" {

ssi_status ssi_result_fetch(ssi_ctx *c, const ssi_params *p, int32_t l, const ssi_output *out,
                            ssi_result **res) {
  if (!c || !p || !out || !res) return fail(SSI_EINVAL, "ssi_result_fetch: NULL argument");
  if (!out->sigma || !out->count || !out->f || !out->xi || !out->mu || !out->phi || !out->flags)
    return fail(SSI_EINVAL, "ssi_result_fetch: NULL output buffer");
  ssi_layout lay;
  ssi_status s = layout_of(p, l, &lay);
  if (s != SSI_OK) return s;
  DeviceGuard g(c->device);
  // the identification's own status; its result is copied in every case so
  // that per-order flags can be read after SSI_ENOCONV
  const ssi_status run = ssi_synchronize(c);
  const std::string run_msg = run == SSI_OK ? std::string() : g_last_error;
  ssi_result *r = new ssi_result();
  r->lay = lay;
  r->nmin = p->order_min;
  r->step = p->order_step;
  for (int o = 0; o <= lay.n_orders; ++o) r->offs.push_back(ssi_pole_offset(p, o));
  const OutSizes z(lay);
  r->sigma.resize(z.sigma);
  r->count.resize(z.count);
  r->flags.resize(z.count);
  r->f.resize(z.poles);
  r->xi.resize(z.poles);
  r->mu.resize(2 * z.poles);
  r->phi.resize(z.phi);
  struct { void *dst; const void *src; size_t bytes; } cp[] = {
      {r->sigma.data(), out->sigma, z.sigma * sizeof(double)},
      {r->count.data(), out->count, z.count * sizeof(int32_t)},
      {r->flags.data(), out->flags, z.count * sizeof(int32_t)},
      {r->f.data(), out->f, z.poles * sizeof(double)},
      {r->xi.data(), out->xi, z.poles * sizeof(double)},
      {r->mu.data(), out->mu, 2 * z.poles * sizeof(double)},
      {r->phi.data(), out->phi, z.phi * sizeof(float)}};
  for (auto &x : cp) {
    const hipError_t e = hipMemcpy(x.dst, x.src, x.bytes, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      delete r;
      return hip_fail(e, "ssi_result_fetch: copy to host");
    }
  }
  *res = r;
  if (run != SSI_OK) g_last_error = run_msg;
  return run;
}

ssi_status ssi_identify_result(ssi_ctx *c, const float *y, int32_t l, int64_t n, int64_t ldy,
                               const ssi_params *p, ssi_result **res) {
  if (!c || !y || !p || !res) return fail(SSI_EINVAL, "ssi_identify_result: NULL argument");
  ssi_status s = ssi_validate(p, l, n);
  if (s != SSI_OK) return s;
  ssi_layout lay;
  s = layout_of(p, l, &lay);
  if (s != SSI_OK) return s;
  const OutSizes z(lay);
  Arena probe;
  probe.take<double>(z.sigma);
  probe.take<int32_t>(z.count);
  probe.take<int32_t>(z.count);
  probe.take<double>(z.poles);
  probe.take<double>(z.poles);
  probe.take<double>(2 * z.poles);
  probe.take<float>(z.phi);
  DeviceGuard g(c->device);
  if (probe.off > c->obuf_cap) {
    // outputs of earlier calls may still be read by queued work or graphs
    drain(c);
    drop_graphs(c);
    dev_free(c, c->obuf);
    c->obuf = nullptr;
    c->obuf_cap = 0;
    const hipError_t e = dev_alloc(c, &c->obuf, probe.off);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(SSI_ENOMEM, "output buffers of %zu bytes could not be allocated", probe.off);
    }
    c->obuf_cap = probe.off;
  }
  Arena a{c->obuf, 0};
  ssi_output out;
  out.sigma = a.take<double>(z.sigma);
  out.count = a.take<int32_t>(z.count);
  out.flags = a.take<int32_t>(z.count);
  out.f = a.take<double>(z.poles);
  out.xi = a.take<double>(z.poles);
  out.mu = a.take<double>(2 * z.poles);
  out.phi = a.take<float>(z.phi);
  s = ssi_identify(c, y, l, n, ldy, p, &out);
  if (s != SSI_OK) return s;
  return ssi_result_fetch(c, p, l, &out, res);
}

ssi_status ssi_result_dims(const ssi_result *r, int32_t *n_lags, int32_t *n_orders, int32_t *l) {
  if (!r) return fail(SSI_EINVAL, "ssi_result_dims: NULL result");
  if (n_lags) *n_lags = r->lay.n_lags;
  if (n_orders) *n_orders = r->lay.n_orders;
  if (l) *l = r->lay.l;
  return SSI_OK;
}

ssi_status ssi_result_poles(const ssi_result *r, int32_t lag_i, int32_t order_i, int32_t *order,
                            int32_t *n_poles, const double **f_hz, const double **zeta,
                            const double **mu_reim, const float **phi_reim, int32_t *flag) {
  if (!r) return fail(SSI_EINVAL, "ssi_result_poles: NULL result");
  if (lag_i < 0 || lag_i >= r->lay.n_lags || order_i < 0 || order_i >= r->lay.n_orders)
    return fail(SSI_EINVAL, "ssi_result_poles: lag %d / order %d out of range", lag_i, order_i);
  const size_t slot = (size_t)lag_i * r->lay.pole_cap + r->offs[order_i];
  const size_t oi = (size_t)lag_i * r->lay.n_orders + order_i;
  if (order) *order = r->nmin + order_i * r->step;
  if (n_poles) *n_poles = r->count[oi];
  if (f_hz) *f_hz = r->f.data() + slot;
  if (zeta) *zeta = r->xi.data() + slot;
  if (mu_reim) *mu_reim = r->mu.data() + 2 * slot;
  if (phi_reim) *phi_reim = r->phi.data() + slot * r->lay.l * 2;
  if (flag) *flag = r->flags[oi];
  return SSI_OK;
}

ssi_status ssi_result_singular_values(const ssi_result *r, int32_t lag_i, int32_t *n,
                                      const double **sigma) {
  if (!r) return fail(SSI_EINVAL, "ssi_result_singular_values: NULL result");
  if (lag_i < 0 || lag_i >= r->lay.n_lags)
    return fail(SSI_EINVAL, "ssi_result_singular_values: lag %d out of range", lag_i);
  if (n) *n = r->lay.sigma_per_lag;
  if (sigma) *sigma = r->sigma.data() + (size_t)lag_i * r->lay.sigma_per_lag;
  return SSI_OK;
}

void ssi_result_free(ssi_result *r) { delete r; }

}  // extern "C"
