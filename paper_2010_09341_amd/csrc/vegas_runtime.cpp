// vegas_runtime.cpp — handles and the C interface of libvegas.so (declared in
// include/vegas.h). Host code only: argument validation, device memory,
// launch configuration and the inverse-variance combination of iterations;
// every per-event and per-bin step runs in the kernels of vegas_kernels.hip.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "vegas.h"
#include "vegas_common.hpp"
#include "vegas_types.hpp"
#include "vegas_launch.hpp"

using vegas::DevGrid;
using vegas::IntegrandArgs;

namespace vegas {

const char* status_name(int s) {
  switch (s) {
    case VEGAS_OK: return "ok";
    case VEGAS_EINVAL: return "invalid argument";
    case VEGAS_ENOMEM: return "out of memory";
    case VEGAS_EDEVICE: return "device error";
    case VEGAS_ESTATE: return "invalid state";
    case VEGAS_ENONFINITE: return "non-finite weights";
    case VEGAS_EBUSY: return "busy";
    case VEGAS_ECOMPILE: return "integrand source did not compile";
    default: return "unknown status";
  }
}

bool shape_ok(int dim, int nb) {
  return dim >= 1 && dim <= VEGAS_MAX_DIM && nb >= 2 && nb <= VEGAS_MAX_BINS &&
         dim * nb <= VEGAS_MAX_CELLS;
}

Layout layout(int dim, int nb, int max_partials, int ring) {
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  Layout L;
  size_t o = 0;
  L.t = o;
  o += 256;
  L.edges = o;
  o = al(o + sizeof(double) * dim * (nb + 1));
  L.hist = o;
  o = al(o + sizeof(double) * dim * nb);
  L.copies = o;
  o = al(o + sizeof(double) * kHistCopies * dim * nb);
  L.rec64 = o;
  o = al(o + sizeof(Rec64) * dim * nb);
  L.rec32 = o;
  o = al(o + sizeof(Rec32) * dim * nb);
  L.partials = o;
  o = al(o + sizeof(double) * 4 * (size_t)max_partials);
  L.results = o;
  o = al(o + sizeof(double) * 4 * (size_t)ring);
  L.total = o;
  return L;
}

DevGrid bind_grid(void* ws, int dim, int nb, int max_partials, int ring) {
  const Layout L = layout(dim, nb, max_partials, ring);
  char* b = static_cast<char*>(ws);
  DevGrid g;
  g.dim = dim;
  g.nb = nb;
  g.t = reinterpret_cast<uint32_t*>(b + L.t);
  g.edges = reinterpret_cast<double*>(b + L.edges);
  g.hist = reinterpret_cast<double*>(b + L.hist);
  g.copies = reinterpret_cast<double*>(b + L.copies);
  g.rec64 = b + L.rec64;
  g.rec32 = b + L.rec32;
  g.partials = reinterpret_cast<double*>(b + L.partials);
  g.results = reinterpret_cast<double*>(b + L.results);
  g.max_blocks = max_partials;
  g.ring = ring;
  return g;
}

// Derived integrand constants from the user's parameters (the parameter
// conventions are those listed with the VEGAS_F_* identifiers).
int build_integrand_args(int fid, int dim, const double* p, int np, IntegrandArgs* out) {
  IntegrandArgs a;
  std::memset(&a, 0, sizeof(a));
  auto par = [&](int i, double dflt) { return (p && i < np) ? p[i] : dflt; };
  const double pi = 3.14159265358979323846;
  if (np < 0 || np > VEGAS_MAX_PARAMS || (np > 0 && !p)) return VEGAS_EINVAL;
  for (int i = 0; i < np; ++i)
    if (!std::isfinite(p[i])) return VEGAS_EINVAL;
  if (fid >= VEGAS_F_USER) {
    // run-time integrand: the parameters as given, zero-filled
    if (!user_integrand_fits(fid, dim) || np > VEGAS_MAX_USER_PARAMS) return VEGAS_EINVAL;
    for (int i = 0; i < np; ++i) {
      a.c64[i] = p[i];
      a.c32[i] = (float)p[i];
    }
    if (out) *out = a;
    return VEGAS_OK;
  }
  switch (fid) {
    case VEGAS_F_CONST:
    case VEGAS_F_SUM:
      if (np != 0) return VEGAS_EINVAL;
      break;
    case VEGAS_F_GAUSS: {
      if (!(np == 0 || np == 1 || np == 1 + dim)) return VEGAS_EINVAL;
      const double w = par(0, 0.1);
      if (!(w > 0.0)) return VEGAS_EINVAL;
      a.d[0] = 1.0 / (w * w);
      a.d[1] = -dim * std::log(w * std::sqrt(pi));
      a.f[0] = (float)(1.0 / (std::log(2.0) * w * w));
      a.f[1] = (float)(-dim * std::log2(w * std::sqrt(pi)));
      for (int d = 0; d < dim; ++d) {
        const double c = (np == 1 + dim) ? p[1 + d] : 0.5;
        a.c64[d] = c;
        a.c32[d] = (float)c;
      }
      break;
    }
    case VEGAS_F_LO_TOY: {
      if (dim != 4 || np > 4) return VEGAS_EINVAL;
      const double sqrt_s = par(0, 13000.0), m = par(1, 91.19), G = par(2, 2.5),
                   cut = par(3, 20.0);
      if (!(sqrt_s > 0.0) || !(m > 0.0) || !(G > 0.0)) return VEGAS_EINVAL;
      a.d[0] = sqrt_s * sqrt_s;
      a.d[1] = m * m;
      a.d[2] = m * G;
      a.d[3] = (m * G / pi) * 2.0 * (2.0 * pi);
      a.d[4] = cut;
      for (int i = 0; i < 4; ++i) a.f[i] = (float)a.d[i];
      a.f[4] = cut > 0.0 ? (float)(cut * cut) : -1.0f;
      break;
    }
    case VEGAS_F_RAMBO24: {
      if (dim != 16 || np > 3) return VEGAS_EINVAL;
      const double sqrt_s = par(0, 1000.0), cut_frac = par(1, 0.01), mode = par(2, 0.0);
      if (!(sqrt_s > 0.0) || !(mode == 0.0 || mode == 1.0)) return VEGAS_EINVAL;
      const double s = sqrt_s * sqrt_s;
      a.d[0] = sqrt_s;
      a.d[1] = (pi / 2.0) * (pi / 2.0) * (pi / 2.0) * s * s / 12.0;
      a.d[2] = cut_frac * s;
      a.d[3] = 2.0 * pi;
      // the cut and the weight on the invariants of the unscaled momenta
      a.d[4] = a.d[2] / (2.0 * s);
      a.d[5] = a.d[1] / (16.0 * s * s * s * s);
      a.f[0] = (float)a.d[0];
      a.f[1] = (float)a.d[1];
      a.f[2] = (float)a.d[2];
      // neither form applies RAMBO's final scale: the cut and the weight are
      // carried as c/(2s) and W/(16 s^4)
      a.f[3] = (float)a.d[4];
      a.f[4] = (float)a.d[5];
      a.mode = (int)mode;
      break;
    }
    case VEGAS_F_BW_FLAT: {
      if (np > 2) return VEGAS_EINVAL;
      const double m = par(0, 0.5), G = par(1, 0.02);
      if (!(G > 0.0)) return VEGAS_EINVAL;
      a.d[0] = m;
      a.d[1] = G * G / 4.0;
      a.d[2] = G / (2.0 * pi);
      for (int i = 0; i < 3; ++i) a.f[i] = (float)a.d[i];
      break;
    }
    default:
      return VEGAS_EINVAL;
  }
  if (out) *out = a;
  return VEGAS_OK;
}

namespace {

std::mutex g_occ_mu;
int g_cus = 0;
std::map<std::pair<const void*, int>, int> g_occ;  // (kernel, threads and LDS) -> blocks per CU

// Resident workgroups per CU of `kernel` (-1 on a HIP error). Holds g_occ_mu.
int blocks_per_cu_locked(const IterKernel& kernel, int threads, size_t lds) {
  if (g_cus == 0) {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
      return -1;
    g_cus = prop.multiProcessorCount;
  }
  const auto key = std::make_pair(kernel.key(), threads * 65536 + (int)(lds / 256));
  auto it = g_occ.find(key);
  if (it != g_occ.end()) return it->second;
  int n = 0;
  const hipError_t e =
      kernel.fn ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel.fn, threads, lds)
                : hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel.mf, threads, lds);
  if (e != hipSuccess) return -1;
  g_occ[key] = n;
  return n;
}

std::map<const void*, int> g_max_threads;  // kernel -> largest workgroup it was built for

int max_threads_locked(const IterKernel& kernel) {
  auto it = g_max_threads.find(kernel.key());
  if (it != g_max_threads.end()) return it->second;
  int n = 0;
  if (kernel.fn) {
    hipFuncAttributes a;
    if (hipFuncGetAttributes(&a, kernel.fn) != hipSuccess) return -1;
    n = a.maxThreadsPerBlock;
  } else if (hipFuncGetAttribute(&n, HIP_FUNC_ATTRIBUTE_MAX_THREADS_PER_BLOCK, kernel.mf) !=
             hipSuccess) {
    return -1;
  }
  g_max_threads[kernel.key()] = n;
  return n;
}

}  // namespace

int kernel_max_threads(const IterKernel& kernel) {
  std::lock_guard<std::mutex> lk(g_occ_mu);
  return max_threads_locked(kernel);
}

int default_threads(const IterKernel& kernel, size_t lds) {
  std::lock_guard<std::mutex> lk(g_occ_mu);
  const int max_threads = max_threads_locked(kernel);
  if (max_threads < 0) return -1;
  // powers of two only: other multiples of 64 can fill more wave slots (two
  // 640-thread workgroups where a SIMD holds 5 waves), but measured slower
  // (the 8-D binary64 Gaussian: 75 instead of 63 us per 1e7 events)
  int best = 0, best_waves = -1;
  for (int threads : {1024, 512, 256, 128, 64}) {
    if (threads > max_threads) continue;
    const int n = blocks_per_cu_locked(kernel, threads, lds);
    if (n < 0) return -1;
    const int waves = n * threads / 64;
    if (waves > best_waves) {
      best = threads;
      best_waves = waves;
    }
  }
  return best;
}

int default_blocks(const IterKernel& kernel, int threads, size_t lds, int64_t n_events, int cap) {
  int per_cu = 0, cus = 0;
  {
    std::lock_guard<std::mutex> lk(g_occ_mu);
    per_cu = blocks_per_cu_locked(kernel, threads, lds);
    cus = g_cus;
  }
  if (per_cu < 0) return -1;
  int64_t want = (n_events + threads - 1) / threads;
  int64_t fill = (int64_t)std::max(per_cu, 1) * cus;
  int64_t b = std::min<int64_t>(want, fill);
  b = std::min<int64_t>(b, cap);
  return (int)std::max<int64_t>(b, 1);
}

void combine(const std::vector<double>& I_t, const std::vector<double>& s_t, double* I,
             double* sigma, double* chi2) {
  const size_t n = I_t.size();
  for (size_t i = 0; i < n; ++i)
    if (!(s_t[i] > 0.0)) {
      *I = I_t[i];
      *sigma = 0.0;
      *chi2 = 0.0;
      return;
    }
  double sw = 0.0, swi = 0.0;
  for (size_t i = 0; i < n; ++i) {
    const double w = 1.0 / (s_t[i] * s_t[i]);
    sw += w;
    swi += w * I_t[i];
  }
  const double mean = swi / sw;
  double c2 = 0.0;
  for (size_t i = 0; i < n; ++i) {
    const double z = (I_t[i] - mean) / s_t[i];
    c2 += z * z;
  }
  *I = mean;
  *sigma = 1.0 / std::sqrt(sw);
  *chi2 = n > 1 ? c2 / (double)(n - 1) : 0.0;
}

}  // namespace vegas

using namespace vegas;

struct vegas_ctx {
  int device = 0;
  int dim = 0, nb = 0, prec = VEGAS_FP64;
  hipStream_t own_stream = nullptr;
  hipStream_t stream = nullptr;
  void* own_ws = nullptr;
  void* ws = nullptr;
  DevGrid g;
  double* pinned = nullptr;
  size_t pinned_n = 0;
  double* ring_host = nullptr;  // [kRing][4] host mirror of the result ring
  double* ring_dev = nullptr;   // the same memory as the device addresses it
  uint32_t t = 0;
  bool hist_valid = false;
  bool poisoned = false;
  std::vector<double> I_t, s_t;
  int64_t last_bad = 0;
  std::vector<double> params[VEGAS_N_INTEGRANDS];
  std::map<int, std::vector<double>> user_params;  // run-time integrands
  int max_blocks = 0;
  int threads = 0;  // 0: chosen per kernel (default_threads)
  int64_t events_limit = 0;  // events per launch within an iteration (0: all)
  bool timing = false;
  double time_ms = 0.0;
  int64_t n_timed = 0;
  std::vector<hipEvent_t> events;
  double* dump_buf = nullptr;
  size_t dump_n = 0;
  // hipGraph of the last vegas_run configuration
  bool use_graph = true;
  hipGraphExec_t graph = nullptr;
  struct RunKey {
    int fid, prec, n_iter, blocks, threads, timing;
    int64_t n_events, events_limit;
    uint64_t seed;
    double alpha;
    hipStream_t stream;
    std::vector<double> params;
    bool operator==(const RunKey& o) const {
      return fid == o.fid && prec == o.prec && n_iter == o.n_iter && blocks == o.blocks &&
             threads == o.threads && timing == o.timing && n_events == o.n_events &&
             events_limit == o.events_limit &&
             seed == o.seed && alpha == o.alpha && stream == o.stream && params == o.params;
    }
  } graph_key{};
};

namespace {

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess || prev == dev || hipSetDevice(dev) != hipSuccess)
      prev = -1;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

int fail(vegas_h h, hipError_t e) {
  if (e == hipSuccess) return VEGAS_OK;
  if (h) h->poisoned = true;
  return VEGAS_EDEVICE;
}

#define VEGAS_TRY(h, expr)                 \
  do {                                     \
    hipError_t _e = (expr);                \
    if (_e != hipSuccess) return fail(h, _e); \
  } while (0)

int ready(vegas_h h) {
  if (!h) return VEGAS_EINVAL;
  if (h->poisoned) return VEGAS_EDEVICE;
  return VEGAS_OK;
}

const std::vector<double>& params_of(vegas_h h, int fid) {
  static const std::vector<double> none;
  if (fid >= 0 && fid < VEGAS_N_INTEGRANDS) return h->params[fid];
  auto it = h->user_params.find(fid);
  return it == h->user_params.end() ? none : it->second;
}

int integrand_args(vegas_h h, int fid, IntegrandArgs* a) {
  if (!integrand_id_ok(fid)) return VEGAS_EINVAL;
  const std::vector<double>& p = params_of(h, fid);
  int rc = build_integrand_args(fid, h->dim, p.empty() ? nullptr : p.data(), (int)p.size(), a);
  if (rc != VEGAS_OK) return rc;
  // a run-time integrand that exists for this dimension but whose code does
  // not load on this GPU is a device error
  if (!iterate_kernel(fid, h->prec, h->dim, false))
    return fid >= VEGAS_F_USER ? VEGAS_EDEVICE : VEGAS_EINVAL;
  return VEGAS_OK;
}

hipError_t ensure_events(vegas_h h, size_t n) {
  while (h->events.size() < n) {
    hipEvent_t e;
    // timing only (read after the stream is synchronised): no system-scope
    // fence, so recording the event does not write back and invalidate the
    // caches around the kernel it brackets
    hipError_t rc = hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
    if (rc != hipSuccess) return rc;
    h->events.push_back(e);
  }
  return hipSuccess;
}

// Launch shape of the iteration kernel for n_events per launch: the handle's
// thread count (0: the one that keeps the most waves resident) and enough
// workgroups to fill the GPU. VEGAS_EINVAL if the handle's thread count
// exceeds the workgroup the kernel was built for; VEGAS_EDEVICE on a HIP
// error.
struct Shape {
  int blocks = 0, threads = 0;
};

int shape_for(vegas_h h, int fid, int64_t n_events, Shape* s) {
  const IterKernel k = iterate_kernel(fid, h->prec, h->dim, false);
  const size_t lds = iterate_lds_bytes(h->dim, h->nb);
  if (h->threads > 0) {
    const int max_threads = kernel_max_threads(k);
    if (max_threads < 0) return VEGAS_EDEVICE;
    if (h->threads > max_threads) return VEGAS_EINVAL;
    s->threads = h->threads;
  } else {
    s->threads = default_threads(k, lds);
    if (s->threads < 1) return VEGAS_EDEVICE;
  }
  const int cap = h->max_blocks > 0 ? std::min(h->max_blocks, kMaxBlocks) : kMaxBlocks;
  s->blocks = default_blocks(k, s->threads, lds, n_events, cap);
  return s->blocks < 1 ? VEGAS_EDEVICE : VEGAS_OK;
}

// Events per launch of the iteration kernel.
int64_t batch_events(vegas_h h, int64_t n_events) {
  return h->events_limit > 0 && h->events_limit < n_events ? h->events_limit : n_events;
}

// Enqueue iterate + finalize (+ refine) for one iteration; event slots 2i, 2i+1
// bracket the iteration kernel launches when timing is on. With an events
// limit the iteration's events go through several launches of at most that
// many events, each adding to the workgroup partials of the previous ones.
hipError_t enqueue_iteration(vegas_h h, int fid, const IntegrandArgs& P, int64_t n_events,
                             uint64_t seed, const Shape& shape, size_t ev_slot, bool refine,
                             double alpha) {
  const int64_t batch = batch_events(h, n_events);
  IterLaunch L;
  L.fid = fid;
  L.prec = h->prec;
  L.seed = seed;
  L.blocks = shape.blocks;
  L.threads = shape.threads;
  hipError_t e;
  if (h->timing && (e = hipEventRecord(h->events[2 * ev_slot], h->stream)) != hipSuccess) return e;
  for (int64_t first = 0; first < n_events; first += batch) {
    L.first = (uint64_t)first;
    L.n_events = std::min(batch, n_events - first);
    L.accumulate = first > 0;
    if ((e = launch_iterate(h->g, L, P, h->stream)) != hipSuccess) return e;
  }
  if (h->timing && (e = hipEventRecord(h->events[2 * ev_slot + 1], h->stream)) != hipSuccess)
    return e;
  return launch_finalize(h->g, shape.blocks, n_events, refine, alpha, h->stream);
}

hipError_t collect_timing(vegas_h h, size_t n) {
  if (!h->timing) return hipSuccess;
  for (size_t i = 0; i < n; ++i) {
    float ms = 0.f;
    hipError_t e = hipEventElapsedTime(&ms, h->events[2 * i], h->events[2 * i + 1]);
    if (e != hipSuccess) return e;
    h->time_ms += ms;
    h->n_timed += 1;
  }
  return hipSuccess;
}

}  // namespace

// ---- checkpoint: a flat little-endian record -------------------------------
//   u64 magic, u32 version, i32 dim, i32 nb, i32 prec, u32 t, i32 hist_valid,
//   i64 events_limit, u64 n_hist, then per integrand u64 np + np doubles,
//   then n_hist I_t, n_hist sigma_t, dim*(nb+1) edges, dim*nb histogram.
namespace {
constexpr uint64_t kStateMagic = 0x5345544147455653ull;  // "SVEGATES"
constexpr uint32_t kStateVersion = 1;
// most per-iteration results a record may hold (VEGAS_MAX_HISTORY)
constexpr uint64_t kMaxHistory = VEGAS_MAX_HISTORY;

struct Writer {
  unsigned char* p;
  size_t n, o = 0;
  template <class T>
  void put(const T& v) {
    if (p && o + sizeof(T) <= n) std::memcpy(p + o, &v, sizeof(T));
    o += sizeof(T);
  }
  void put_doubles(const double* v, size_t k) {
    if (p && o + 8 * k <= n && k) std::memcpy(p + o, v, 8 * k);
    o += 8 * k;
  }
};

struct Reader {
  const unsigned char* p;
  size_t n, o = 0;
  bool ok = true;
  template <class T>
  T get() {
    T v{};
    if (o + sizeof(T) > n) {
      ok = false;
      return v;
    }
    std::memcpy(&v, p + o, sizeof(T));
    o += sizeof(T);
    return v;
  }
  bool get_doubles(double* v, size_t k) {
    if (o + 8 * k > n) return ok = false;
    if (k) std::memcpy(v, p + o, 8 * k);
    o += 8 * k;
    return true;
  }
};

// Serialise the handle's state; the grid and histogram come from the device.
int save_state(vegas_h h, Writer& w) {
  const size_t ne = (size_t)h->dim * (h->nb + 1), nh = (size_t)h->dim * h->nb;
  std::vector<double> edges(ne), hist(nh);
  if (w.p) {
    int rc = vegas_get_grid(h, edges.data(), ne);
    if (rc) return rc;
    rc = vegas_get_hist(h, hist.data(), nh);
    if (rc) return rc;
  }
  w.put(kStateMagic);
  w.put(kStateVersion);
  w.put((int32_t)h->dim);
  w.put((int32_t)h->nb);
  w.put((int32_t)h->prec);
  w.put((uint32_t)h->t);
  w.put((int32_t)(h->hist_valid ? 1 : 0));
  w.put((int64_t)h->events_limit);
  w.put((uint64_t)h->I_t.size());
  for (int f = 0; f < VEGAS_N_INTEGRANDS; ++f) {
    w.put((uint64_t)h->params[f].size());
    w.put_doubles(h->params[f].data(), h->params[f].size());
  }
  w.put_doubles(h->I_t.data(), h->I_t.size());
  w.put_doubles(h->s_t.data(), h->s_t.size());
  w.put_doubles(edges.data(), ne);
  w.put_doubles(hist.data(), nh);
  return VEGAS_OK;
}
}  // namespace

namespace {
// Host-side allocations (the per-iteration history, checkpoint buffers,
// parameter vectors) may throw; no exception crosses the C interface.
template <class F>
int no_throw(F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return VEGAS_ENOMEM;
  } catch (...) {
    return VEGAS_EINVAL;
  }
}

}  // namespace

extern "C" {

const char* vegas_strerror(int status) { return status_name(status); }

int vegas_workspace_bytes(int dim, int n_bins, size_t* bytes) {
  if (!shape_ok(dim, n_bins) || !bytes) return VEGAS_EINVAL;
  *bytes = layout(dim, n_bins).total;
  return VEGAS_OK;
}

int vegas_create(int dim, int n_bins, vegas_h* out) {
  if (!out || !shape_ok(dim, n_bins)) return VEGAS_EINVAL;
  *out = nullptr;
  vegas_h h = new (std::nothrow) vegas_ctx();
  if (!h) return VEGAS_ENOMEM;
  h->dim = dim;
  h->nb = n_bins;
  int rc = VEGAS_OK;
  hipError_t e = hipGetDevice(&h->device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&h->own_stream, hipStreamNonBlocking);
  if (e == hipSuccess) {
    h->stream = h->own_stream;
    e = hipMalloc(&h->own_ws, layout(dim, n_bins).total);
    if (e == hipErrorOutOfMemory) rc = VEGAS_ENOMEM;
  }
  if (e == hipSuccess) {
    h->ws = h->own_ws;
    h->g = bind_grid(h->ws, dim, n_bins);
    h->pinned_n = (size_t)dim * (n_bins + 1);
    e = hipHostMalloc(reinterpret_cast<void**>(&h->pinned), sizeof(double) * h->pinned_n,
                      hipHostMallocDefault);
  }
  // the result ring's host mirror: pinned, mapped into the device's address
  // space, coherent (the finalize kernel's stores reach host memory)
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void**>(&h->ring_host), sizeof(double) * 4 * kRing,
                      hipHostMallocMapped | hipHostMallocCoherent);
  if (e == hipSuccess)
    e = hipHostGetDevicePointer(reinterpret_cast<void**>(&h->ring_dev), h->ring_host, 0);
  if (e == hipSuccess) h->g.results_host = h->ring_dev;
  if (e == hipSuccess) e = launch_init_grid(h->g, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    vegas_destroy(h);
    return rc != VEGAS_OK ? rc : VEGAS_EDEVICE;
  }
  *out = h;
  return VEGAS_OK;
}

int vegas_destroy(vegas_h h) {
  if (!h) return VEGAS_OK;
  DeviceGuard dg(h->device);
  // teardown: errors are ignored, the handle goes away regardless
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  for (hipEvent_t e : h->events) (void)hipEventDestroy(e);
  if (h->dump_buf) (void)hipFree(h->dump_buf);
  if (h->graph) (void)hipGraphExecDestroy(h->graph);
  if (h->own_ws) (void)hipFree(h->own_ws);
  if (h->pinned) (void)hipHostFree(h->pinned);
  if (h->ring_host) (void)hipHostFree(h->ring_host);
  if (h->own_stream) (void)hipStreamDestroy(h->own_stream);
  delete h;
  return VEGAS_OK;
}

int vegas_reset(vegas_h h) {
  int rc = ready(h);
  if (rc) return rc;
  DeviceGuard dg(h->device);
  // queued on the handle's stream ahead of any later work; not waited for
  VEGAS_TRY(h, launch_init_grid(h->g, h->stream));
  h->t = 0;
  h->hist_valid = false;
  h->I_t.clear();
  h->s_t.clear();
  h->last_bad = 0;
  return VEGAS_OK;
}

static int vegas_set_params_body(vegas_h h, int integrand_id, const double* params, int n_params) {
  int rc = ready(h);
  if (rc) return rc;
  if (!integrand_id_ok(integrand_id)) return VEGAS_EINVAL;
  rc = build_integrand_args(integrand_id, h->dim, params, n_params, nullptr);
  if (rc) return rc;
  if (integrand_id >= VEGAS_F_USER)
    h->user_params[integrand_id].assign(params, params + n_params);
  else
    h->params[integrand_id].assign(params, params + n_params);
  return VEGAS_OK;
}

int vegas_set_precision(vegas_h h, int prec) {
  int rc = ready(h);
  if (rc) return rc;
  if (prec != VEGAS_FP64 && prec != VEGAS_FP32_EVAL) return VEGAS_EINVAL;
  h->prec = prec;
  return VEGAS_OK;
}

int vegas_bind_stream(vegas_h h, void* hip_stream) {
  int rc = ready(h);
  if (rc) return rc;
  DeviceGuard dg(h->device);
  hipStream_t next = hip_stream ? static_cast<hipStream_t>(hip_stream) : h->own_stream;
  if (next != h->stream) {
    // order the new stream after everything queued on the old one
    VEGAS_TRY(h, hipStreamSynchronize(h->stream));
    h->stream = next;
  }
  return VEGAS_OK;
}

int vegas_bind_workspace(vegas_h h, void* dev_ptr, size_t bytes) {
  int rc = ready(h);
  if (rc) return rc;
  const size_t need = layout(h->dim, h->nb).total;
  void* next = dev_ptr ? dev_ptr : h->own_ws;
  if (dev_ptr && (bytes < need || (reinterpret_cast<uintptr_t>(dev_ptr) & 255)))
    return VEGAS_EINVAL;
  DeviceGuard dg(h->device);
  if (!next) {
    VEGAS_TRY(h, hipMalloc(&h->own_ws, need));
    next = h->own_ws;
  }
  if (next != h->ws) {
    VEGAS_TRY(h, hipMemcpyAsync(next, h->ws, need, hipMemcpyDeviceToDevice, h->stream));
    VEGAS_TRY(h, hipStreamSynchronize(h->stream));
    h->ws = next;
    h->g = bind_grid(h->ws, h->dim, h->nb);
    h->g.results_host = h->ring_dev;
    // records hold no pointers, the copy preserved everything; a captured
    // run refers to the old workspace
    if (h->graph) {
      VEGAS_TRY(h, hipGraphExecDestroy(h->graph));
      h->graph = nullptr;
    }
  }
  if (dev_ptr && h->own_ws) {
    VEGAS_TRY(h, hipFree(h->own_ws));
    h->own_ws = nullptr;
  }
  return VEGAS_OK;
}

static int vegas_iterate_body(vegas_h h, int integrand_id, int64_t n_events, uint64_t seed, double* I,
                  double* sigma) {
  int rc = ready(h);
  if (rc) return rc;
  if (n_events < 2 || !I || !sigma) return VEGAS_EINVAL;
  if (h->I_t.size() + 1 > kMaxHistory) return VEGAS_ESTATE;
  // room for this iteration's result first: a failed allocation changes nothing
  h->I_t.reserve(h->I_t.size() + 1);
  h->s_t.reserve(h->s_t.size() + 1);
  IntegrandArgs P;
  DeviceGuard dg(h->device);  // kernels of run-time integrands load per device
  rc = integrand_args(h, integrand_id, &P);
  if (rc) return rc;
  Shape shape;
  rc = shape_for(h, integrand_id, batch_events(h, n_events), &shape);
  if (rc == VEGAS_EDEVICE) return fail(h, hipErrorInvalidValue);
  if (rc) return rc;
  if (h->timing) VEGAS_TRY(h, ensure_events(h, 2));
  VEGAS_TRY(h, enqueue_iteration(h, integrand_id, P, n_events, seed, shape, 0, false, 0.0));
  // finalize writes the result into the host-mapped ring as well
  VEGAS_TRY(h, hipStreamSynchronize(h->stream));
  VEGAS_TRY(h, collect_timing(h, 1));
  const double* r = h->ring_host + 4 * (h->t % kRing);
  *I = r[0];
  *sigma = r[1];
  h->last_bad = (int64_t)r[2];
  h->t += 1;
  h->hist_valid = true;
  h->I_t.push_back(*I);
  h->s_t.push_back(*sigma);
  return h->last_bad > 0 ? VEGAS_ENONFINITE : VEGAS_OK;
}

int vegas_refine(vegas_h h, double alpha) {
  int rc = ready(h);
  if (rc) return rc;
  if (!(alpha >= 0.0 && alpha <= VEGAS_MAX_ALPHA)) return VEGAS_EINVAL;
  if (!h->hist_valid) return VEGAS_ESTATE;
  DeviceGuard dg(h->device);
  VEGAS_TRY(h, launch_refine(h->g, alpha, h->stream));
  VEGAS_TRY(h, hipStreamSynchronize(h->stream));
  h->hist_valid = false;
  return VEGAS_OK;
}

static int vegas_run_body(vegas_h h, int integrand_id, int64_t n_events, uint64_t seed, int n_iter,
              double alpha, double* I_t, double* sigma_t) {
  int rc = ready(h);
  if (rc) return rc;
  if (n_events < 2 || n_iter < 1 || n_iter > VEGAS_MAX_RUN_ITER ||
      !(alpha >= 0.0 && alpha <= VEGAS_MAX_ALPHA))
    return VEGAS_EINVAL;
  if (h->I_t.size() + (size_t)n_iter > kMaxHistory) return VEGAS_ESTATE;
  h->I_t.reserve(h->I_t.size() + n_iter);
  h->s_t.reserve(h->s_t.size() + n_iter);
  IntegrandArgs P;
  DeviceGuard dg(h->device);  // kernels of run-time integrands load per device
  rc = integrand_args(h, integrand_id, &P);
  if (rc) return rc;
  Shape shape;
  rc = shape_for(h, integrand_id, batch_events(h, n_events), &shape);
  if (rc == VEGAS_EDEVICE) return fail(h, hipErrorInvalidValue);
  if (rc) return rc;
  if (h->timing) VEGAS_TRY(h, ensure_events(h, 2 * (size_t)n_iter));
  auto enqueue_all = [&]() -> hipError_t {
    for (int i = 0; i < n_iter; ++i) {
      hipError_t e = enqueue_iteration(h, integrand_id, P, n_events, seed, shape, i,
                                       i + 1 < n_iter, alpha);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  if (h->use_graph && !h->timing) {
    // the iterations read and advance the iteration counter on the device, so
    // one captured sequence serves every run of the same configuration
    vegas_ctx::RunKey key{integrand_id, h->prec, n_iter, shape.blocks, shape.threads, 0,
                          n_events, h->events_limit, seed, alpha, h->stream,
                          params_of(h, integrand_id)};
    if (!h->graph || !(key == h->graph_key)) {
      if (h->graph) {
        VEGAS_TRY(h, hipGraphExecDestroy(h->graph));
        h->graph = nullptr;
      }
      hipGraph_t g = nullptr;
      VEGAS_TRY(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
      const hipError_t ce = enqueue_all();
      const hipError_t ee = hipStreamEndCapture(h->stream, &g);
      if (ce != hipSuccess || ee != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(h, ce != hipSuccess ? ce : ee);
      }
      const hipError_t ie = hipGraphInstantiate(&h->graph, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ie != hipSuccess) {
        h->graph = nullptr;
        return fail(h, ie);
      }
      h->graph_key = key;
    }
    VEGAS_TRY(h, hipGraphLaunch(h->graph, h->stream));
  } else {
    VEGAS_TRY(h, enqueue_all());
  }
  // each finalize wrote its result into the host-mapped ring as well
  VEGAS_TRY(h, hipStreamSynchronize(h->stream));
  VEGAS_TRY(h, collect_timing(h, (size_t)n_iter));
  int64_t bad = 0;
  for (int i = 0; i < n_iter; ++i) {
    const double* r = h->ring_host + 4 * ((h->t + i) % kRing);
    if (I_t) I_t[i] = r[0];
    if (sigma_t) sigma_t[i] = r[1];
    h->I_t.push_back(r[0]);
    h->s_t.push_back(r[1]);
    bad += (int64_t)r[2];
  }
  h->t += (uint32_t)n_iter;
  h->hist_valid = true;
  h->last_bad = bad;
  return bad > 0 ? VEGAS_ENONFINITE : VEGAS_OK;
}

int vegas_result(vegas_h h, double* I, double* sigma, double* chi2_dof) {
  int rc = ready(h);
  if (rc) return rc;
  if (!I || !sigma || !chi2_dof) return VEGAS_EINVAL;
  if (h->I_t.empty()) return VEGAS_ESTATE;
  combine(h->I_t, h->s_t, I, sigma, chi2_dof);
  return VEGAS_OK;
}

int vegas_get_grid(vegas_h h, double* edges, size_t n) {
  int rc = ready(h);
  if (rc) return rc;
  const size_t need = (size_t)h->dim * (h->nb + 1);
  if (!edges || n != need) return VEGAS_EINVAL;
  DeviceGuard dg(h->device);
  VEGAS_TRY(h, hipMemcpyAsync(h->pinned, h->g.edges, need * sizeof(double),
                              hipMemcpyDeviceToHost, h->stream));
  VEGAS_TRY(h, hipStreamSynchronize(h->stream));
  std::memcpy(edges, h->pinned, need * sizeof(double));
  return VEGAS_OK;
}

int vegas_set_grid(vegas_h h, const double* edges, size_t n) {
  int rc = ready(h);
  if (rc) return rc;
  const size_t need = (size_t)h->dim * (h->nb + 1);
  if (!edges || n != need) return VEGAS_EINVAL;
  for (int d = 0; d < h->dim; ++d) {
    const double* e = edges + (size_t)d * (h->nb + 1);
    if (e[0] != 0.0 || e[h->nb] != 1.0) return VEGAS_EINVAL;
    for (int i = 0; i < h->nb; ++i)
      if (!(e[i + 1] > e[i])) return VEGAS_EINVAL;
  }
  DeviceGuard dg(h->device);
  VEGAS_TRY(h, hipStreamSynchronize(h->stream));
  std::memcpy(h->pinned, edges, need * sizeof(double));
  VEGAS_TRY(h, hipMemcpyAsync(h->g.edges, h->pinned, need * sizeof(double),
                              hipMemcpyHostToDevice, h->stream));
  VEGAS_TRY(h, launch_prepare(h->g, h->stream));
  VEGAS_TRY(h, hipStreamSynchronize(h->stream));
  return VEGAS_OK;
}

int vegas_get_hist(vegas_h h, double* hist, size_t n) {
  int rc = ready(h);
  if (rc) return rc;
  const size_t need = (size_t)h->dim * h->nb;
  if (!hist || n != need) return VEGAS_EINVAL;
  DeviceGuard dg(h->device);
  VEGAS_TRY(h, hipMemcpyAsync(h->pinned, h->g.hist, need * sizeof(double),
                              hipMemcpyDeviceToHost, h->stream));
  VEGAS_TRY(h, hipStreamSynchronize(h->stream));
  std::memcpy(hist, h->pinned, need * sizeof(double));
  return VEGAS_OK;
}

int vegas_set_hist(vegas_h h, const double* hist, size_t n) {
  int rc = ready(h);
  if (rc) return rc;
  const size_t need = (size_t)h->dim * h->nb;
  if (!hist || n != need) return VEGAS_EINVAL;
  for (size_t i = 0; i < need; ++i)
    if (!(hist[i] >= 0.0) || !std::isfinite(hist[i])) return VEGAS_EINVAL;
  DeviceGuard dg(h->device);
  VEGAS_TRY(h, hipStreamSynchronize(h->stream));
  std::memcpy(h->pinned, hist, need * sizeof(double));
  VEGAS_TRY(h, hipMemcpyAsync(h->g.hist, h->pinned, need * sizeof(double),
                              hipMemcpyHostToDevice, h->stream));
  VEGAS_TRY(h, hipStreamSynchronize(h->stream));
  h->hist_valid = true;
  return VEGAS_OK;
}

int vegas_get_iteration(vegas_h h, uint32_t* t) {
  int rc = ready(h);
  if (rc) return rc;
  if (!t) return VEGAS_EINVAL;
  *t = h->t;
  return VEGAS_OK;
}

int vegas_set_iteration(vegas_h h, uint32_t t) {
  int rc = ready(h);
  if (rc) return rc;
  DeviceGuard dg(h->device);
  VEGAS_TRY(h, launch_set_t(h->g, t, h->stream));
  VEGAS_TRY(h, hipStreamSynchronize(h->stream));
  h->t = t;
  return VEGAS_OK;
}

int vegas_nonfinite(vegas_h h, int64_t* count) {
  int rc = ready(h);
  if (rc) return rc;
  if (!count) return VEGAS_EINVAL;
  *count = h->last_bad;
  return VEGAS_OK;
}

int vegas_dump_weights(vegas_h h, int integrand_id, uint64_t seed, uint64_t first, int64_t count,
                       double* w_out) {
  int rc = ready(h);
  if (rc) return rc;
  if (count < 0 || count > (int64_t(1) << 26) || (count > 0 && !w_out)) return VEGAS_EINVAL;
  IntegrandArgs P;
  DeviceGuard dg(h->device);  // kernels of run-time integrands load per device
  rc = integrand_args(h, integrand_id, &P);
  if (rc) return rc;
  if (count == 0) return VEGAS_OK;
  if (h->dump_n < (size_t)count) {
    if (h->dump_buf) VEGAS_TRY(h, hipFree(h->dump_buf));
    h->dump_buf = nullptr;
    h->dump_n = 0;
    VEGAS_TRY(h, hipMalloc(reinterpret_cast<void**>(&h->dump_buf), sizeof(double) * count));
    h->dump_n = (size_t)count;
  }
  IterLaunch L;
  L.fid = integrand_id;
  L.prec = h->prec;
  L.seed = seed;
  L.first = first;
  L.count = count;
  L.w_out = h->dump_buf;
  VEGAS_TRY(h, launch_dump(h->g, L, P, h->stream));
  VEGAS_TRY(h, hipMemcpyAsync(w_out, h->dump_buf, sizeof(double) * count, hipMemcpyDeviceToHost,
                              h->stream));
  VEGAS_TRY(h, hipStreamSynchronize(h->stream));
  return VEGAS_OK;
}

int vegas_set_launch(vegas_h h, int max_blocks, int threads) {
  int rc = ready(h);
  if (rc) return rc;
  if (max_blocks < 0 || max_blocks > kMaxBlocks) return VEGAS_EINVAL;
  if (threads < 0 || threads > kIterThreadsMax || threads % 64 != 0) return VEGAS_EINVAL;
  h->max_blocks = max_blocks;
  h->threads = threads;
  return VEGAS_OK;
}

static int vegas_state_bytes_body(vegas_h h, size_t* bytes) {
  int rc = ready(h);
  if (rc) return rc;
  if (!bytes) return VEGAS_EINVAL;
  Writer w{nullptr, 0};
  save_state(h, w);
  *bytes = w.o;
  return VEGAS_OK;
}

static int vegas_save_body(vegas_h h, void* buf, size_t bytes) {
  int rc = ready(h);
  if (rc) return rc;
  size_t need = 0;
  vegas_state_bytes(h, &need);
  if (!buf || bytes < need) return VEGAS_EINVAL;
  Writer w{static_cast<unsigned char*>(buf), bytes};
  return save_state(h, w);
}

static int vegas_load_body(vegas_h h, const void* buf, size_t bytes) {
  int rc = ready(h);
  if (rc) return rc;
  if (!buf) return VEGAS_EINVAL;
  Reader r{static_cast<const unsigned char*>(buf), bytes};
  if (r.get<uint64_t>() != kStateMagic || r.get<uint32_t>() != kStateVersion) return VEGAS_EINVAL;
  const int dim = r.get<int32_t>(), nb = r.get<int32_t>(), prec = r.get<int32_t>();
  const uint32_t t = r.get<uint32_t>();
  const int hist_valid = r.get<int32_t>();
  const int64_t limit = r.get<int64_t>();
  const uint64_t n_hist = r.get<uint64_t>();
  if (!r.ok || dim != h->dim || nb != h->nb || (prec != VEGAS_FP64 && prec != VEGAS_FP32_EVAL) ||
      limit < 0 || n_hist > kMaxHistory)
    return VEGAS_EINVAL;
  // the record must hold the two n_hist-double arrays before anything is
  // sized from n_hist (a truncated or corrupt record allocates nothing)
  if (16 * n_hist > bytes - r.o) return VEGAS_EINVAL;
  std::vector<double> params[VEGAS_N_INTEGRANDS];
  for (int f = 0; f < VEGAS_N_INTEGRANDS; ++f) {
    const uint64_t np = r.get<uint64_t>();
    if (!r.ok || np > VEGAS_MAX_PARAMS) return VEGAS_EINVAL;
    params[f].resize(np);
    if (!r.get_doubles(params[f].data(), np)) return VEGAS_EINVAL;
    if (np && build_integrand_args(f, dim, params[f].data(), (int)np, nullptr) != VEGAS_OK)
      return VEGAS_EINVAL;
  }
  std::vector<double> I_t(n_hist), s_t(n_hist);
  std::vector<double> edges((size_t)dim * (nb + 1)), hist((size_t)dim * nb);
  if (!r.get_doubles(I_t.data(), n_hist) || !r.get_doubles(s_t.data(), n_hist) ||
      !r.get_doubles(edges.data(), edges.size()) || !r.get_doubles(hist.data(), hist.size()))
    return VEGAS_EINVAL;
  // validate the arrays before touching the device, so a bad record changes nothing
  for (int d = 0; d < dim; ++d) {
    const double* e = edges.data() + (size_t)d * (nb + 1);
    if (e[0] != 0.0 || e[nb] != 1.0) return VEGAS_EINVAL;
    for (int i = 0; i < nb; ++i)
      if (!(e[i + 1] > e[i])) return VEGAS_EINVAL;
  }
  for (double v : hist)
    if (!(v >= 0.0) || !std::isfinite(v)) return VEGAS_EINVAL;
  rc = vegas_set_grid(h, edges.data(), edges.size());
  if (rc) return rc;
  rc = vegas_set_hist(h, hist.data(), hist.size());
  if (rc) return rc;
  rc = vegas_set_iteration(h, t);
  if (rc) return rc;
  for (int f = 0; f < VEGAS_N_INTEGRANDS; ++f) h->params[f] = params[f];
  h->prec = prec;
  h->events_limit = limit;
  h->hist_valid = hist_valid != 0;
  h->I_t = I_t;
  h->s_t = s_t;
  return VEGAS_OK;
}

int vegas_set_events_limit(vegas_h h, int64_t limit) {
  int rc = ready(h);
  if (rc) return rc;
  if (limit < 0) return VEGAS_EINVAL;
  h->events_limit = limit;
  return VEGAS_OK;
}

int vegas_set_graph(vegas_h h, int enable) {
  int rc = ready(h);
  if (rc) return rc;
  h->use_graph = enable != 0;
  return VEGAS_OK;
}

int vegas_timing(vegas_h h, int enable, int reset, double* iterate_ms, int64_t* n_launches) {
  int rc = ready(h);
  if (rc) return rc;
  if (iterate_ms) *iterate_ms = h->time_ms;
  if (n_launches) *n_launches = h->n_timed;
  if (reset || (enable != 0) != h->timing) {
    h->time_ms = 0.0;
    h->n_timed = 0;
  }
  h->timing = enable != 0;
  return VEGAS_OK;
}

int vegas_set_params(vegas_h h, int integrand_id, const double* params, int n_params) {
  return no_throw([&] { return vegas_set_params_body(h, integrand_id, params, n_params); });
}

int vegas_iterate(vegas_h h, int integrand_id, int64_t n_events, uint64_t seed, double* I,
                  double* sigma) {
  return no_throw([&] { return vegas_iterate_body(h, integrand_id, n_events, seed, I, sigma); });
}

int vegas_run(vegas_h h, int integrand_id, int64_t n_events, uint64_t seed, int n_iter,
              double alpha, double* I_t, double* sigma_t) {
  return no_throw([&] {
    return vegas_run_body(h, integrand_id, n_events, seed, n_iter, alpha, I_t, sigma_t);
  });
}

int vegas_state_bytes(vegas_h h, size_t* bytes) {
  return no_throw([&] { return vegas_state_bytes_body(h, bytes); });
}

int vegas_save(vegas_h h, void* buf, size_t bytes) {
  return no_throw([&] { return vegas_save_body(h, buf, bytes); });
}

int vegas_load(vegas_h h, const void* buf, size_t bytes) {
  return no_throw([&] { return vegas_load_body(h, buf, bytes); });
}

}  // extern "C"
