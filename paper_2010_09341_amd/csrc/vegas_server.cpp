// vegas_server.cpp — the serving loop behind vegas_server_* (include/vegas.h).
//
// A scheduler thread owns a device arena (the memory budget) and a few HIP
// streams (lanes). Requests are admitted first-in first-out when a slot and
// arena bytes are free; every admitted integral keeps its grid, histogram
// and partial sums resident in its arena range, and is assigned to a lane:
// an idle one if there is one (so it starts at once, its work overlapping
// whatever the other lanes run), else the lane holding the fewest integrals.
// A lane advances its integrals one iteration per tick, and runs the ticks
// up to the next completion of one of them as one chain, enqueued back to
// back with no host round trip between them; the scheduler polls the lanes'
// streams and collects a chain's results when it has drained. A tick:
//   1. newly admitted integrals get their uniform grid (k_serve_init);
//   2. one launch per (precision, dimension class) runs every event chunk of
//      every integral's current iteration (k_serve_iterate), so small
//      integrals share the GPU; an integral of at least 2^20 events per
//      iteration instead gets one launch of the single-integral iteration
//      kernel (exact dimension count, up to 1024-thread workgroups), whose
//      workgroups take the place of its chunks;
//   3. one launch closes all those iterations: moments, histogram reduction
//      and refinement (k_serve_finalize);
//   4. the per-integral (I_t, sigma_t) come back through mapped host memory,
//      32 bytes per integral and tick, which the closing kernel writes;
//      finished integrals free their slot and arena range for waiting
//      requests.
// The inputs of a chain (new slot descriptors, work lists) are packed into
// one pinned buffer mapped into the device's address space, from which a
// small kernel (k_serve_stage) moves them into device memory.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "vegas.h"
#include "vegas_common.hpp"
#include "vegas_sched.hpp"
#include "vegas_serve.hpp"

using namespace vegas;

namespace {

using Clock = std::chrono::steady_clock;

struct Req {
  uint64_t ticket = 0;
  vegas_request r{};
  std::vector<double> params;
  IntegrandArgs P{};
  int64_t chunk = 0;
  uint32_t n_chunks = 0;
  // A large request runs each iteration as one launch of the single-integral
  // iteration kernel (its workgroups take the place of chunks).
  bool big = false;
  int big_threads = 0;
  DevGrid g{};
  Layout L{};
  int slot = -1;
  size_t off = 0;
  bool fresh = false;
  int iters = 0;
  std::vector<double> I_t, s_t;
  int64_t bad = 0;
  Clock::time_point t_submit, t_done;
  bool done = false;
  int status = VEGAS_OK;
  double I = 0, sigma = 0, chi2 = 0;
};

// Requests of at least this many events per iteration run as single-integral
// iteration-kernel launches rather than as chunks of the batched kernel.
constexpr int64_t kServeBigEvents = int64_t(1) << 20;
// Upper end of each lane's input buffers reserved when a server is created.
constexpr size_t kServeReserveBytes = size_t(4) << 20;
// Longest chain of ticks enqueued before the host synchronises, and the most
// events a chain may carry (about 2 ms of device work at full rate, so that a
// request arriving during a chain of large integrals does not wait longer).
constexpr int kChainMax = 32;
constexpr int64_t kChainEvents = int64_t(300) << 20;
// Streams (lanes) whose chains run concurrently: by default 4, the hardware
// queues a process gets by default; at most 8.
constexpr int kDefaultLanes = 4;
constexpr int kMaxLanes = 8;

struct DeviceGuardSrv {
  int prev = -1;
  explicit DeviceGuardSrv(int dev) {
    if (hipGetDevice(&prev) != hipSuccess || prev == dev || hipSetDevice(dev) != hipSuccess)
      prev = -1;
  }
  ~DeviceGuardSrv() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

Layout slot_layout(int dim, int nb, uint32_t n_chunks, int ring) {
  return layout(dim, nb, (int)n_chunks, ring);
}

size_t slot_bytes(const Req* q) { return q->L.total; }

template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  hipError_t reserve(size_t want) {
    if (want <= n) return hipSuccess;
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
    size_t cap = want + want / 2 + 64;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&p), cap * sizeof(T));
    if (e == hipSuccess) n = cap;
    return e;
  }
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

// Pinned host memory mapped into the device's address space (coherent): a
// tick's packed inputs, which the host writes and a kernel reads, and its
// results, which a kernel writes and the host reads after synchronising.
template <class T>
struct Mapped {
  T* host = nullptr;
  T* dev = nullptr;
  size_t n = 0;
  hipError_t reserve(size_t want) {
    if (want <= n) return hipSuccess;
    if (host) (void)hipHostFree(host);
    host = dev = nullptr;
    n = 0;
    const size_t cap = want + want / 2 + 64;
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&host), cap * sizeof(T),
                                 hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void**>(&dev), host, 0);
    if (e == hipSuccess) n = cap;
    return e;
  }
  ~Mapped() {
    if (host) (void)hipHostFree(host);
  }
};

// One stream of the server and the chain of ticks it runs: the integrals
// assigned to a lane advance together, and the lanes run concurrently on
// their own streams, so that a request arriving while other integrals are on
// the GPU starts at once on an idle lane instead of waiting for their chain.
struct Lane {
  hipStream_t stream = nullptr;
  Mapped<unsigned char> in_pin;  // a chain's inputs, staged into in_dev by a kernel
  DevBuf<unsigned char> in_dev;
  Mapped<double> out;            // per-tick results, written by the finalize kernel
  // tick lists, kept between chains to reuse their storage: the closing
  // items of every tick of a chain but the last (every integral refines) and
  // of its last tick (the integrals at their last iteration do not)
  std::vector<FinItem> init_items, fin_items, fin_last;
  std::vector<WorkItem> work[2][2];  // [prec][dim class 16 / 32]
  std::vector<Req*> fresh, big;
  // A chain whose inputs equal the previous chain's (same integrals, same
  // chunks, none new) repeats its device work without staging its inputs
  // again; with graph replay on, such a tick is captured once it has
  // repeated kGraphRepeats times and replayed until the inputs change.
  std::vector<unsigned char> last_in;
  int repeats = 0;
  hipGraphExec_t graph = nullptr;
  const void* graph_bufs[3] = {nullptr, nullptr, nullptr};
  // the integrals of this lane, and the chain in flight
  std::vector<Req*> members, act;
  int K = 0;
  bool busy = false;

  void drop_graph() {
    if (graph) (void)hipGraphExecDestroy(graph);
    graph = nullptr;
  }
  hipError_t create(size_t in_bytes, size_t out_doubles) {
    hipError_t e = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = in_pin.reserve(in_bytes);
    if (e == hipSuccess) e = in_dev.reserve(in_bytes);
    if (e == hipSuccess) e = out.reserve(out_doubles);
    return e;
  }
  ~Lane() {
    if (stream) (void)hipStreamSynchronize(stream);
    drop_graph();
    if (stream) (void)hipStreamDestroy(stream);
  }
};

}  // namespace

struct vegas_srv {
  int device = 0;
  void* arena_dev = nullptr;
  Arena arena;
  int max_slots = 0;
  int64_t chunk_fixed = 0;
  SlotDev* slots_dev = nullptr;
  SlotDev* slots_pin = nullptr;  // per-slot staging of descriptors
  size_t lane_in_bytes = 0;
  std::vector<std::unique_ptr<Lane>> lanes;
  int n_lanes = 0;

  std::thread worker;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  int error = VEGAS_OK;
  std::unique_ptr<Admission<Req*>> adm;
  std::map<uint64_t, std::unique_ptr<Req>> reqs;
  uint64_t next_ticket = 1;
  std::vector<Req*> active;  // by slot
  int n_active = 0;
  // submissions so far, read by the worker while it waits for a chain
  std::atomic<uint64_t> submitted{0};
  // statistics
  int64_t completed = 0, events = 0, work_items = 0, peak_active = 0;
  std::atomic<int64_t> ticks{0}, graph_ticks{0}, chains{0};
  static constexpr int kGraphRepeats = 8;
  std::atomic<bool> use_graph{false};
  // longest chain of ticks (1: one tick per chain)
  std::atomic<int> chain_max{kChainMax};

  void run();
  hipError_t chain(Lane& L, int K);
  void collect(Lane& L);
  void fail_all();
  hipError_t add_lanes(int n);
};

hipError_t vegas_srv::add_lanes(int n) {
  while ((int)lanes.size() < n) {
    auto L = std::make_unique<Lane>();
    const hipError_t e = L->create(lane_in_bytes, 4 * (size_t)max_slots * kChainMax);
    if (e != hipSuccess) return e;
    lanes.push_back(std::move(L));
  }
  return hipSuccess;
}

// Enqueue K ticks in a row over the lane's integrals (none finishes before
// the last of them) on the lane's stream; the results of tick j land at
// L.out.host[4 (j L.act.size() + i)] once the stream has drained.
hipError_t vegas_srv::chain(Lane& L, int K) {
  std::vector<Req*>& act = L.act;
  // ---- host-side tick lists (member vectors: no allocation per chain) --------
  for (auto& a : L.work)
    for (auto& v : a) v.clear();
  L.init_items.clear();
  L.fin_items.clear();
  L.fin_last.clear();
  L.fresh.clear();
  L.big.clear();
  int max_lds[2][2] = {{0, 0}, {0, 0}};
  int max_nb = 2;
  for (size_t i = 0; i < act.size(); ++i) {
    Req* q = act[i];
    const int dim = q->r.dim, nb = q->r.n_bins;
    max_nb = std::max(max_nb, nb);
    if (q->fresh) {
      for (int d = 0; d < dim; ++d)
        L.init_items.push_back(FinItem{(uint32_t)q->slot, d, (uint32_t)L.fresh.size(), 0});
      L.fresh.push_back(q);
    }
    if (q->big) {
      L.big.push_back(q);
    } else {
      const int pc = q->r.prec == VEGAS_FP64 ? 0 : 1;
      const int dc = dim <= 16 ? 0 : 1;
      for (uint32_t c = 0; c < q->n_chunks; ++c)
        L.work[pc][dc].push_back(WorkItem{(uint32_t)q->slot, c});
      const LdsLayout ll = lds_layout(dim, nb, kServeCopies, kServeLdsBudget);
      max_lds[pc][dc] = std::max(max_lds[pc][dc], (int)lds_bytes(ll));
    }
    // no refinement after an integral's last iteration
    const uint32_t refine_last = q->iters + K < q->r.n_iter ? 1u : 0u;
    L.fin_items.push_back(FinItem{(uint32_t)q->slot, -1, (uint32_t)i, 0});
    L.fin_last.push_back(FinItem{(uint32_t)q->slot, -1, (uint32_t)i, 0});
    for (int d = 0; d < dim; ++d) {
      L.fin_items.push_back(FinItem{(uint32_t)q->slot, d, (uint32_t)i, 1u});
      L.fin_last.push_back(FinItem{(uint32_t)q->slot, d, (uint32_t)i, refine_last});
    }
  }
  // ---- pack the inputs into one pinned buffer ------------------------------
  // [closing items][closing items of the last tick][work items by class] —
  // the part that repeats from chain to chain — then, for new integrals only,
  // [descriptors][init items].
  size_t core = (L.fin_items.size() + L.fin_last.size()) * sizeof(FinItem);
  for (auto& a : L.work)
    for (auto& v : a) core += v.size() * sizeof(WorkItem);
  const size_t o_desc = (core + 15) / 16 * 16;
  const size_t o_init = o_desc + L.fresh.size() * sizeof(SlotDev);
  const size_t bytes = L.fresh.empty() ? core : o_init + L.init_items.size() * sizeof(FinItem);
  hipError_t e;
  // the staging kernel moves whole 16-byte words
  const size_t staged = (bytes + 15) / 16 * 16;
  if ((e = L.in_pin.reserve(staged)) != hipSuccess) return e;
  if ((e = L.in_dev.reserve(staged)) != hipSuccess) return e;
  if ((e = L.out.reserve(4 * act.size() * (size_t)K)) != hipSuccess) return e;
  size_t o = 0;
  auto put = [&](const void* src, size_t n) {
    const size_t at = o;
    if (n) std::memcpy(L.in_pin.host + o, src, n);
    o += n;
    return at;
  };
  const size_t o_fin = put(L.fin_items.data(), L.fin_items.size() * sizeof(FinItem));
  const size_t o_fin_last = put(L.fin_last.data(), L.fin_last.size() * sizeof(FinItem));
  size_t o_work[2][2];
  for (int p = 0; p < 2; ++p)
    for (int c = 0; c < 2; ++c)
      o_work[p][c] = put(L.work[p][c].data(), L.work[p][c].size() * sizeof(WorkItem));
  if (!L.fresh.empty()) {
    o = o_desc;
    for (Req* q : L.fresh) put(slots_pin + q->slot, sizeof(SlotDev));
    put(L.init_items.data(), L.init_items.size() * sizeof(FinItem));
  }
  // ---- device work ------------------------------------------------------------
  hipStream_t stream = L.stream;
  auto fin_at = [&](size_t off) { return reinterpret_cast<const FinItem*>(L.in_dev.p + off); };
  auto work_at = [&](size_t off) { return reinterpret_cast<const WorkItem*>(L.in_dev.p + off); };
  // one tick after the inputs are staged: grids of new integrals (first tick
  // of the chain only), the chunks of every integral's iteration, closing the
  // iterations (the finalize kernel writes their results into mapped host
  // memory, row `row` of the chain's results)
  auto enqueue_tick = [&](bool init, bool last, size_t row) -> hipError_t {
    hipError_t e2;
    if (init && !L.fresh.empty() &&
        (e2 = launch_serve_init(slots_dev, fin_at(o_init), (int)L.init_items.size(), max_nb,
                                reinterpret_cast<const SlotDev*>(L.in_dev.p + o_desc),
                                stream)) != hipSuccess)
      return e2;
    for (Req* q : L.big) {
      IterLaunch it;
      it.fid = q->r.integrand_id;
      it.prec = q->r.prec;
      it.n_events = q->r.n_events;
      it.seed = q->r.seed;
      it.blocks = (int)q->n_chunks;
      it.threads = q->big_threads;
      if ((e2 = launch_iterate(q->g, it, q->P, stream)) != hipSuccess) return e2;
    }
    for (int p = 0; p < 2; ++p)
      for (int c = 0; c < 2; ++c) {
        if (L.work[p][c].empty()) continue;
        if ((e2 = launch_serve_iterate(c == 0 ? 16 : 32, p == 0 ? VEGAS_FP64 : VEGAS_FP32_EVAL,
                                       slots_dev, work_at(o_work[p][c]),
                                       (int)L.work[p][c].size(), max_lds[p][c], stream)) !=
            hipSuccess)
          return e2;
      }
    return launch_serve_finalize(slots_dev, fin_at(last ? o_fin_last : o_fin),
                                 (int)L.fin_items.size(), max_nb,
                                 L.out.dev + 4 * act.size() * row, stream);
  };
  ticks += K;
  ++chains;
  // the inputs already on the device (the same integrals and chunks as the
  // lane's last chain, none new): no staging
  const bool same = L.fresh.empty() && core > 0 && core == L.last_in.size() &&
                    std::memcmp(L.in_pin.host, L.last_in.data(), core) == 0;
  if (same) {
    ++L.repeats;
    // graph replay runs one tick per chain (a captured tick writes a fixed
    // results row)
    const void* bufs[3] = {L.in_dev.p, L.out.dev, nullptr};
    if (L.graph &&
        (std::memcmp(bufs, L.graph_bufs, sizeof(bufs)) != 0 || !use_graph || K != 1))
      L.drop_graph();
    if (use_graph && K == 1 && !L.graph && L.repeats >= kGraphRepeats) {
      if ((e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return e;
      const hipError_t ew = enqueue_tick(false, true, 0);
      hipGraph_t g = nullptr;
      const hipError_t ec = hipStreamEndCapture(stream, &g);
      if (ew == hipSuccess && ec == hipSuccess)
        e = hipGraphInstantiate(&L.graph, g, nullptr, nullptr, 0);
      if (g) (void)hipGraphDestroy(g);
      if (ew != hipSuccess) return ew;
      if (ec != hipSuccess) return ec;
      if (e != hipSuccess) {
        L.graph = nullptr;
        return e;
      }
      std::memcpy(L.graph_bufs, bufs, sizeof(bufs));
    }
    if (L.graph && K == 1) {
      ++graph_ticks;
      return hipGraphLaunch(L.graph, stream);
    }
    for (int j = 0; j < K; ++j)
      if ((e = enqueue_tick(false, j == K - 1, (size_t)j)) != hipSuccess) return e;
    return hipSuccess;
  }
  L.drop_graph();
  L.repeats = 0;
  L.last_in.assign(L.in_pin.host, L.in_pin.host + core);
  for (Req* q : L.fresh) q->fresh = false;
  // the inputs reach device memory through a kernel that reads the mapped
  // host buffer, not through a copy engine: a host-to-device copy of a few
  // KB now and then took milliseconds to enqueue, holding up every integral
  // in flight
  if ((e = launch_serve_stage(L.in_pin.dev, L.in_dev.p, bytes, stream)) != hipSuccess) return e;
  for (int j = 0; j < K; ++j)
    if ((e = enqueue_tick(j == 0, j == K - 1, (size_t)j)) != hipSuccess) return e;
  return hipSuccess;
}

// The results of a lane's drained chain: every integral advances by K
// iterations; finished integrals free their slot and arena range. Holds mu.
void vegas_srv::collect(Lane& L) {
  const std::vector<Req*>& act = L.act;
  for (size_t i = 0; i < act.size(); ++i) {
    Req* q = act[i];
    for (int j = 0; j < L.K; ++j) {
      const double* r = L.out.host + 4 * (act.size() * (size_t)j + i);
      q->I_t.push_back(r[0]);
      q->s_t.push_back(r[1]);
      q->bad += (int64_t)r[2];
    }
    work_items += (int64_t)q->n_chunks * L.K;
    q->iters += L.K;
    events += q->r.n_events * L.K;
    if (q->iters == q->r.n_iter) {
      q->t_done = Clock::now();
      combine(q->I_t, q->s_t, &q->I, &q->sigma, &q->chi2);
      q->status = q->bad > 0 ? VEGAS_ENONFINITE : VEGAS_OK;
      q->done = true;
      active[q->slot] = nullptr;
      --n_active;
      adm->finish(q->slot, q->off);
      ++completed;
      const auto it = std::find(L.members.begin(), L.members.end(), q);
      if (it != L.members.end()) L.members.erase(it);
    }
  }
  L.busy = false;
  cv_done.notify_all();
}

// A device error: every request not yet finished fails with VEGAS_EDEVICE.
// Holds mu.
void vegas_srv::fail_all() {
  error = VEGAS_EDEVICE;
  for (auto& kv : reqs)
    if (!kv.second->done) {
      kv.second->done = true;
      kv.second->status = VEGAS_EDEVICE;
      kv.second->t_done = Clock::now();
    }
  cv_done.notify_all();
}

void vegas_srv::run() {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  uint64_t seen = 0;  // submissions the loop has looked at
  for (;;) {
    if (error == VEGAS_OK) {
      seen = submitted.load();
      auto admitted = adm->admit(slot_bytes);
      for (auto& a : admitted) {
        Req* q = std::get<0>(a);
        q->slot = std::get<1>(a);
        q->off = std::get<2>(a);
        q->fresh = true;
        active[q->slot] = q;
        ++n_active;
        DevGrid g = bind_grid(static_cast<char*>(arena_dev) + q->off, q->r.dim, q->r.n_bins,
                              (int)q->n_chunks, q->r.n_iter);
        q->g = g;
        SlotDev S{};
        S.t = g.t;
        S.edges = g.edges;
        S.hist = g.hist;
        S.copies = g.copies;
        S.rec64 = static_cast<Rec64*>(g.rec64);
        S.rec32 = static_cast<Rec32*>(g.rec32);
        S.partials = g.partials;
        S.results = g.results;
        S.n_events = (uint64_t)q->r.n_events;
        S.chunk_events = (uint64_t)q->chunk;
        S.n_chunks = q->n_chunks;
        S.seed_lo = (uint32_t)q->r.seed;
        S.seed_hi = (uint32_t)(q->r.seed >> 32);
        S.dim = q->r.dim;
        S.nb = (uint32_t)q->r.n_bins;
        S.fid = q->r.integrand_id;
        S.prec = q->r.prec;
        S.ring = q->r.n_iter;
        S.alpha = q->r.alpha;
        S.P = q->P;
        slots_pin[q->slot] = S;
        bool busy[kMaxLanes];
        size_t members[kMaxLanes];
        for (int i = 0; i < n_lanes; ++i) {
          busy[i] = lanes[i]->busy;
          members[i] = lanes[i]->members.size();
        }
        lanes[pick_lane(n_lanes, busy, members)]->members.push_back(q);
      }
      peak_active = std::max<int64_t>(peak_active, n_active);
    }
    // start a chain on every idle lane that has integrals: the ticks until
    // the first of them finishes, within the chain bounds
    for (int i = 0; i < n_lanes && error == VEGAS_OK; ++i) {
      Lane& L = *lanes[i];
      if (L.busy || L.members.empty()) continue;
      std::vector<int> remaining(L.members.size());
      std::vector<int64_t> ev(L.members.size());
      for (size_t m = 0; m < L.members.size(); ++m) {
        remaining[m] = L.members[m]->r.n_iter - L.members[m]->iters;
        ev[m] = L.members[m]->r.n_events;
      }
      L.K = chain_ticks((int)L.members.size(), remaining.data(), ev.data(),
                        use_graph ? 1 : chain_max.load(), kChainEvents);
      L.act = L.members;
      L.busy = true;
      lk.unlock();
      const hipError_t e = chain(L, L.K);
      lk.lock();
      if (e != hipSuccess) fail_all();
    }
    bool any_busy = false;
    for (int i = 0; i < n_lanes; ++i) any_busy = any_busy || lanes[i]->busy;
    if (!any_busy || error != VEGAS_OK) {
      if (error != VEGAS_OK) {
        // drain what was enqueued before the error, then stop taking work
        lk.unlock();
        for (int i = 0; i < n_lanes; ++i) (void)hipStreamSynchronize(lanes[i]->stream);
        lk.lock();
        for (int i = 0; i < n_lanes; ++i) lanes[i]->busy = false;
      }
      if (stop && (adm->pending() == 0 || error != VEGAS_OK)) break;
      cv_work.wait(lk);
      continue;
    }
    // Wait until a lane's chain drains, or a submission arrives while a lane
    // is idle (it can start at once there). Polling: a spin for the first
    // millisecond (a chain of small integrals drains within a few hundred
    // microseconds), then 20-microsecond sleeps.
    bool idle_lane = false;
    for (int i = 0; i < n_lanes; ++i) idle_lane = idle_lane || !lanes[i]->busy;
    lk.unlock();
    Lane* drained = nullptr;
    hipError_t e = hipSuccess;
    const auto spin_until = Clock::now() + std::chrono::milliseconds(1);
    for (;;) {
      for (int i = 0; i < n_lanes && !drained; ++i) {
        Lane& L = *lanes[i];
        if (!L.busy) continue;
        const hipError_t q = hipStreamQuery(L.stream);
        if (q == hipSuccess) {
          drained = &L;
        } else if (q != hipErrorNotReady) {
          drained = &L;
          e = q;
        }
      }
      if (drained || (idle_lane && submitted.load() != seen)) break;
      if (Clock::now() < spin_until)
        std::this_thread::yield();
      else
        std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    lk.lock();
    if (e != hipSuccess) {
      fail_all();
      continue;
    }
    if (drained) collect(*drained);
  }
}

extern "C" {

int vegas_server_create(size_t mem_budget_bytes, int max_slots, int64_t chunk_events,
                        vegas_server* out) {
  if (!out || max_slots < 1 || max_slots > 4096 || chunk_events < 0 || mem_budget_bytes < 4096)
    return VEGAS_EINVAL;
  *out = nullptr;
  auto s = std::make_unique<vegas_srv>();
  s->max_slots = max_slots;
  s->chunk_fixed = chunk_events;
  if (hipGetDevice(&s->device) != hipSuccess) return VEGAS_EDEVICE;
  hipError_t e = hipMalloc(&s->arena_dev, mem_budget_bytes);
  if (e == hipSuccess)
    e = hipMalloc(reinterpret_cast<void**>(&s->slots_dev), sizeof(SlotDev) * max_slots);
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void**>(&s->slots_pin), sizeof(SlotDev) * max_slots,
                      hipHostMallocDefault);
  if (e != hipSuccess) {
    const int rc = e == hipErrorOutOfMemory ? VEGAS_ENOMEM : VEGAS_EDEVICE;
    if (s->slots_pin) (void)hipHostFree(s->slots_pin);
    if (s->slots_dev) (void)hipFree(s->slots_dev);
    if (s->arena_dev) (void)hipFree(s->arena_dev);
    return rc;
  }
  // The per-lane input and result buffers, sized up front for every slot
  // busy with default chunking (an integral below kServeBigEvents events has
  // at most kServeBigEvents / 512 chunks, and a chain two lists of closing
  // items), up to kServeReserveBytes: growing them inside a chain means a
  // pinned allocation and a synchronising free, milliseconds during which
  // every integral of the lane waits.
  const size_t per_slot = sizeof(SlotDev) + 2 * (kMaxDim + 1) * sizeof(FinItem) +
                          (size_t)(kServeBigEvents / 512) * sizeof(WorkItem) + 16;
  s->lane_in_bytes = std::min(per_slot * (size_t)max_slots, kServeReserveBytes);
  e = s->add_lanes(kDefaultLanes);
  if (e != hipSuccess) {
    const int rc = e == hipErrorOutOfMemory ? VEGAS_ENOMEM : VEGAS_EDEVICE;
    s->lanes.clear();
    (void)hipHostFree(s->slots_pin);
    (void)hipFree(s->slots_dev);
    (void)hipFree(s->arena_dev);
    return rc;
  }
  s->n_lanes = kDefaultLanes;
  s->arena = Arena(mem_budget_bytes);
  s->adm = std::make_unique<Admission<Req*>>(max_slots, &s->arena);
  s->active.assign(max_slots, nullptr);
  vegas_srv* raw = s.release();
  raw->worker = std::thread([raw] { raw->run(); });
  *out = raw;
  return VEGAS_OK;
}

int vegas_server_submit(vegas_server s, const vegas_request* r, uint64_t* ticket) {
  if (!s || !r || !ticket) return VEGAS_EINVAL;
  if (!shape_ok(r->dim, r->n_bins) || r->n_events < 2 || r->n_iter < 1 ||
      r->n_iter > VEGAS_MAX_RUN_ITER || !(r->alpha >= 0.0 && r->alpha <= VEGAS_MAX_ALPHA) ||
      (r->prec != VEGAS_FP64 && r->prec != VEGAS_FP32_EVAL) || r->n_params < 0 ||
      // the serving kernels are compiled with the built-in integrands only
      r->integrand_id < 0 || r->integrand_id >= VEGAS_N_INTEGRANDS ||
      r->n_params > VEGAS_MAX_PARAMS || (r->n_params > 0 && !r->params))
    return VEGAS_EINVAL;
  auto q = std::make_unique<Req>();
  q->r = *r;
  q->params.assign(r->params, r->params + r->n_params);
  q->r.params = nullptr;
  if (build_integrand_args(r->integrand_id, r->dim, q->params.data(), r->n_params, &q->P) !=
      VEGAS_OK)
    return VEGAS_EINVAL;
  if (s->chunk_fixed == 0 && r->n_events >= kServeBigEvents) {
    // one launch of the iteration kernel per iteration, its launch shape a
    // function of the request alone (so its estimate does not depend on the
    // mix); its workgroup partials take the chunks' place
    DeviceGuardSrv dg(s->device);
    const IterKernel k = iterate_kernel(r->integrand_id, r->prec, r->dim, false);
    const size_t lds = iterate_lds_bytes(r->dim, r->n_bins);
    const int threads = k ? default_threads(k, lds) : -1;
    const int blocks = threads > 0 ? default_blocks(k, threads, lds, r->n_events, kMaxBlocks) : -1;
    if (blocks < 1) return VEGAS_EDEVICE;
    q->big = true;
    q->big_threads = threads;
    q->chunk = 0;
    q->n_chunks = (uint32_t)blocks;
  } else {
    q->chunk = chunk_events(r->n_events, s->chunk_fixed);
    const int64_t nc = (r->n_events + q->chunk - 1) / q->chunk;
    if (nc > (int64_t)UINT32_MAX / 2) return VEGAS_EINVAL;
    q->n_chunks = (uint32_t)nc;
  }
  q->L = slot_layout(r->dim, r->n_bins, q->n_chunks, r->n_iter);
  if (q->L.total > s->arena.size()) return VEGAS_ENOMEM;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->error != VEGAS_OK) return s->error;
  if (s->stop) return VEGAS_ESTATE;
  q->ticket = s->next_ticket++;
  q->t_submit = Clock::now();
  *ticket = q->ticket;
  s->adm->push(q.get());
  s->reqs[q->ticket] = std::move(q);
  ++s->submitted;
  s->cv_work.notify_one();
  return VEGAS_OK;
}

int vegas_server_wait(vegas_server s, uint64_t ticket, double timeout_s, double* I, double* sigma,
                      double* chi2_dof, double* latency_s) {
  if (!s) return VEGAS_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->reqs.find(ticket) == s->reqs.end()) return VEGAS_EINVAL;
  // The ticket is looked up again at every wake-up: another thread may have
  // released it (and freed its record) once it finished, before this one
  // reacquired the lock.
  Req* q = nullptr;
  auto ready = [&] {
    const auto it = s->reqs.find(ticket);
    q = it == s->reqs.end() ? nullptr : it->second.get();
    return !q || q->done;
  };
  if (timeout_s < 0) {
    s->cv_done.wait(lk, ready);
  } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready)) {
    return VEGAS_EBUSY;
  }
  if (!q) return VEGAS_EINVAL;  // released by another thread meanwhile
  if (q->status == VEGAS_EDEVICE) return VEGAS_EDEVICE;
  if (I) *I = q->I;
  if (sigma) *sigma = q->sigma;
  if (chi2_dof) *chi2_dof = q->chi2;
  if (latency_s) *latency_s = std::chrono::duration<double>(q->t_done - q->t_submit).count();
  return q->status;
}

int vegas_server_iterations(vegas_server s, uint64_t ticket, double* I_t, double* sigma_t) {
  if (!s) return VEGAS_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return VEGAS_EINVAL;
  Req* q = it->second.get();
  if (!q->done) return VEGAS_EBUSY;
  if (q->status == VEGAS_EDEVICE) return VEGAS_EDEVICE;
  for (size_t i = 0; i < q->I_t.size(); ++i) {
    if (I_t) I_t[i] = q->I_t[i];
    if (sigma_t) sigma_t[i] = q->s_t[i];
  }
  return VEGAS_OK;
}

int vegas_server_release(vegas_server s, uint64_t ticket) {
  if (!s) return VEGAS_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return VEGAS_EINVAL;
  // a finished request is referenced by nothing else: collect() removed it
  // from its slot, its lane and the admission queue, and after a device
  // error the worker touches no request again
  if (!it->second->done) return VEGAS_EBUSY;
  s->reqs.erase(it);
  return VEGAS_OK;
}

int vegas_server_stats(vegas_server s, int64_t* completed, int64_t* events, int64_t* work_items,
                       int64_t* peak_active) {
  if (!s) return VEGAS_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (completed) *completed = s->completed;
  if (events) *events = s->events;
  if (work_items) *work_items = s->work_items;
  if (peak_active) *peak_active = s->peak_active;
  return VEGAS_OK;
}

int vegas_server_set_graph(vegas_server s, int enable) {
  if (!s) return VEGAS_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  s->use_graph = enable != 0;
  return VEGAS_OK;
}

int vegas_server_set_chain(vegas_server s, int max_ticks) {
  if (!s || max_ticks < 1 || max_ticks > kChainMax) return VEGAS_EINVAL;
  s->chain_max = max_ticks;
  return VEGAS_OK;
}

int vegas_server_set_lanes(vegas_server s, int lanes) {
  if (!s || lanes < 1 || lanes > kMaxLanes) return VEGAS_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->n_active > 0 || s->adm->pending() > 0) return VEGAS_ESTATE;
  DeviceGuardSrv dg(s->device);
  const hipError_t e = s->add_lanes(lanes);
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? VEGAS_ENOMEM : VEGAS_EDEVICE;
  s->n_lanes = lanes;
  return VEGAS_OK;
}

int vegas_server_chains(vegas_server s, int64_t* chains) {
  if (!s) return VEGAS_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (chains) *chains = s->chains;
  return VEGAS_OK;
}

int vegas_server_ticks(vegas_server s, int64_t* ticks, int64_t* graph_ticks) {
  if (!s) return VEGAS_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (ticks) *ticks = s->ticks;
  if (graph_ticks) *graph_ticks = s->graph_ticks;
  return VEGAS_OK;
}

int vegas_server_destroy(vegas_server s) {
  if (!s) return VEGAS_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  const int rc = s->error;
  {
    DeviceGuardSrv dg(s->device);
    s->lanes.clear();  // each lane drains its stream first
    if (s->slots_pin) (void)hipHostFree(s->slots_pin);
    if (s->slots_dev) (void)hipFree(s->slots_dev);
    if (s->arena_dev) (void)hipFree(s->arena_dev);
  }
  delete s;
  return rc;
}

}  // extern "C"
