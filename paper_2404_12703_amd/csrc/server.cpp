// server.cpp -- continuous batching of many independent DGSEM solves on one GPU.
//
// Requests are queued with their parameters, mesh and initial state.  A
// preparation thread builds the host set-up (geometry, metrics, the CFL step)
// of each request once it has arrived, reusing the set-up of an identical mesh
// seen before.  Each call of the loop (dg_server_run) repeats: admit prepared
// requests in arrival
// order while the memory budget and the slot table allow (strict FIFO: the
// head of the queue is never overtaken); run one RK stage for every active
// request -- one launch per kernel for every group of requests sharing
// (N, precision, shock capturing), each workgroup finding its request through
// block prefix sums and a device array of per-request views; retire requests
// whose last stage has run: copy the state out and release the memory once
// the copy has completed.  A request's arithmetic does not depend on what
// else is in the batch, so each result equals the same solve run alone.
//
// The paper overlaps one solve's kernels on prioritised streams (Sec. 3.2);
// the serving loop instead fills the GPU with the stages of many solves.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "dg_internal.h"
#include "solver_impl.h"

using namespace dg;

namespace {

constexpr int kDescSlots = 64;  // ring of descriptor uploads in flight
// Streams the groups of a tick run on, in turn: groups hold disjoint requests,
// so small batches of different degrees overlap instead of queueing behind
// each other's tails.  Each tick forks from the server's stream and joins it.
constexpr int kGroupStreams = 3;
constexpr int kPrepAhead = 16;  // requests at the head of the queue prepared ahead of admission
// pinned host memory the preparation thread stages initial states in, so
// admission uploads them asynchronously (a state that does not fit goes from
// pageable memory at admission)
constexpr size_t kUpStageBytes = size_t(512) << 20;
constexpr size_t kGeoCacheBytes = size_t(4) << 30;  // host memory of the geometry cache
enum { PREP_WAITING = 0, PREP_RUNNING = 1, PREP_READY = 2, PREP_FAILED = 3 };

struct Request {
  int64_t id = 0;
  dg_params p{};
  int64_t E = 0;
  int n_geo = 1;
  std::vector<double> x_geo;
  std::vector<int64_t> nbr_elem;
  std::vector<int8_t> nbr_face, nbr_orient;
  std::vector<double> U0;
  int32_t n_steps = 0;
  double dt = 0.0;
  double t_arrival = 0.0, t_admit = -1.0, t_done = -1.0;
  int32_t state = DG_REQ_QUEUED;
  // while active: the request's own block (state and temporaries) and the
  // shared geometry block of its mesh
  size_t off = 0, bytes = 0;
  Layout L{};   // LAYOUT_STATE
  Layout Lg{};  // LAYOUT_GEOMETRY
  const HostSetup *geo_key = nullptr;
  View<double> vd{};
  View<float> vf{};
  int step = 0, stage = 0, cur = 0, bpar = 0;  // bpar: alternates over surface sweeps
  double t = 0.0;
  bool traces_valid = false;
  // host set-up, made by the preparation thread once the request has arrived;
  // kept until its upload has landed
  std::shared_ptr<const HostSetup> host;
  size_t up_off = SIZE_MAX;  // the initial state's place in the pinned staging area, if staged
  std::atomic<int> prep{PREP_WAITING};
  std::string prep_err;
  hipEvent_t ready = nullptr;  // set-up copies done
  // retirement: the state leaves through the server's pinned staging slots
  std::vector<double> result;
  bool retiring = false, bad = false;
  size_t issued = 0, copied = 0;  // bytes of the state sent to / landed in result
};

// Pinned host staging for retirement, allocated once at server creation:
// finished states are copied out in chunks through these slots, so the
// serving loop never allocates or frees pinned memory.
constexpr size_t kStageChunk = size_t(16) << 20;
constexpr int kStageSlots = 16;
struct StageSlot {
  char *host = nullptr;  // kStageChunk bytes + one int for the finiteness flag
  hipEvent_t ev = nullptr;
  int64_t req = 0;
  size_t off = 0, bytes = 0;
  bool busy = false, flag = false;
};

// Set-ups of meshes seen before, kept by the preparation thread (the only
// user).  A hit needs the same parameters that shape the set-up and a mesh
// equal byte for byte to the stored copy; least recently used entries go
// beyond kGeoCacheBytes.
struct GeoCache {
  struct Entry {
    std::shared_ptr<const HostSetup> hs;
    dg_params p{};
    int n_geo = 0;
    std::vector<double> x_geo;
    std::vector<int64_t> nbr_elem;
    std::vector<int8_t> nbr_face, nbr_orient;
    size_t bytes = 0;
    uint64_t used = 0;
  };
  std::multimap<uint64_t, Entry> map;  // content hash -> entries
  size_t bytes = 0;
  uint64_t clock = 0;

  static uint64_t mix(uint64_t h, const void *data, size_t n) {
    const unsigned char *c = (const unsigned char *)data;
    size_t i = 0;
    for (; i + 8 <= n; i += 8) {
      uint64_t w;
      std::memcpy(&w, c + i, 8);
      h = (h ^ w) * 0x100000001b3ULL;
      h ^= h >> 29;
    }
    for (; i < n; ++i) h = (h ^ c[i]) * 0x100000001b3ULL;
    return h;
  }
  static uint64_t key(const Request &r) {
    uint64_t h = 0xcbf29ce484222325ULL;
    const int32_t shape[6] = {r.p.N, r.p.nodes, r.p.precision, r.p.source, r.n_geo, 0};
    h = mix(h, shape, sizeof shape);
    h = mix(h, &r.E, sizeof r.E);
    h = mix(h, r.x_geo.data(), r.x_geo.size() * 8);
    h = mix(h, r.nbr_elem.data(), r.nbr_elem.size() * 8);
    h = mix(h, r.nbr_face.data(), r.nbr_face.size());
    return mix(h, r.nbr_orient.data(), r.nbr_orient.size());
  }
  static bool same(const Entry &en, const Request &r) {
    return en.p.N == r.p.N && en.p.nodes == r.p.nodes && en.p.precision == r.p.precision &&
           en.p.source == r.p.source && en.n_geo == r.n_geo && en.x_geo == r.x_geo && en.nbr_elem == r.nbr_elem &&
           en.nbr_face == r.nbr_face && en.nbr_orient == r.nbr_orient;
  }
  std::shared_ptr<const HostSetup> find(uint64_t k, const Request &r) {
    auto range = map.equal_range(k);
    for (auto it = range.first; it != range.second; ++it)
      if (same(it->second, r)) {
        it->second.used = ++clock;
        return it->second.hs;
      }
    return nullptr;
  }
  void insert(uint64_t k, const Request &r, std::shared_ptr<const HostSetup> hs) {
    Entry en;
    en.hs = std::move(hs);
    en.p = r.p;
    en.n_geo = r.n_geo;
    en.x_geo = r.x_geo;
    en.nbr_elem = r.nbr_elem;
    en.nbr_face = r.nbr_face;
    en.nbr_orient = r.nbr_orient;
    en.bytes = en.hs->bytes() + 8 * (en.x_geo.size() + en.nbr_elem.size()) + 2 * en.nbr_face.size();
    if (en.bytes > kGeoCacheBytes) return;
    while (bytes + en.bytes > kGeoCacheBytes && !map.empty()) {
      auto lru = map.begin();
      for (auto it = map.begin(); it != map.end(); ++it)
        if (it->second.used < lru->second.used) lru = it;
      bytes -= lru->second.bytes;
      map.erase(lru);
    }
    en.used = ++clock;
    bytes += en.bytes;
    map.emplace(k, std::move(en));
  }
};

// first-fit allocator over [0, budget) of the arena, 256-byte granules
struct Arena {
  size_t budget = 0;
  std::map<size_t, size_t> free_;  // offset -> size
  void init(size_t base, size_t size) {
    free_.clear();
    budget = size;
    free_[base] = size;
  }
  bool alloc(size_t bytes, size_t &off) {
    bytes = (bytes + 255) & ~size_t(255);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        off = it->first;
        size_t rest = it->second - bytes;
        free_.erase(it);
        if (rest) free_[off + bytes] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

}  // namespace

struct dg_server {
  char *arena = nullptr;
  size_t arena_bytes = 0, budget = 0;
  int max_active = 0;
  hipStream_t st = nullptr, cst = nullptr;
  Arena alloc;
  // descriptor ring: device region at the arena head, pinned host mirrors
  size_t desc_stride = 0;
  char *desc_host[kDescSlots] = {};
  hipEvent_t desc_ev[kDescSlots] = {};
  int desc_next = 0;
  hipStream_t gst[kGroupStreams] = {};
  hipEvent_t fork_ev = nullptr, join_ev[kGroupStreams] = {};
  StageSlot slots[kStageSlots];
  // geometry blocks resident in the arena, one per distinct set-up (mesh,
  // degree, node type, precision), shared by the requests that use it; kept
  // after their last request retires and evicted least recently used when
  // memory is needed
  struct DevGeo {
    std::shared_ptr<const HostSetup> hs;  // holds the key's identity while the block lives
    size_t off = 0, bytes = 0;
    int refs = 0;
    uint64_t used = 0;
  };
  std::map<const HostSetup *, DevGeo> dgeo;
  uint64_t dgeo_clock = 0;
  int64_t st_geo_hits = 0, st_geo_uploads = 0;
  std::vector<hipEvent_t> ev_free;  // events of admitted requests, reused
  char *up_host = nullptr;          // kUpStageBytes of pinned memory
  Arena up_alloc;                   // its allocator, shared by the preparation thread and the loop
  std::mutex up_mu;
  // reqs and queue are shared with the preparation thread: changed under prep_mu
  std::map<int64_t, std::unique_ptr<Request>> reqs;
  std::deque<int64_t> queue;
  std::mutex prep_mu;
  std::condition_variable prep_cv;
  bool prep_stop = false;
  std::thread prep_thread;
  GeoCache geo;  // the preparation thread's
  std::vector<int64_t> active;
  int64_t next_id = 1;
  // the server clock starts at the first dg_server_run call (0 before it)
  std::chrono::steady_clock::time_point t0;
  std::atomic<bool> started{false};
  bool broken = false;
  // loop statistics (dg_server_stats)
  int64_t st_ticks = 0, st_active_sum = 0;
  double st_admit = 0.0, st_tick = 0.0, st_retire = 0.0, st_gpu_wait = 0.0, st_idle = 0.0, st_upload_bytes = 0.0;
  double now() const {
    if (!started.load(std::memory_order_acquire)) return 0.0;
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

size_t view_bytes() { return std::max(sizeof(View<double>), sizeof(View<float>)); }

dg_status server_fail(dg_server *sv, hipError_t e, const char *what) {
  sv->broken = true;
  return fail(DG_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// The preparation thread: host set-up (geometry, metrics, the CFL step) of
// the requests near the head of the queue that have arrived, in queue order,
// while the serving loop keeps the GPU busy.
void prep_loop(dg_server *sv) {
  std::unique_lock<std::mutex> lk(sv->prep_mu);
  while (!sv->prep_stop) {
    Request *next = nullptr;
    double wake = 1e300;
    int pos = 0;
    for (int64_t id : sv->queue) {
      if (pos++ >= kPrepAhead) break;
      Request &r = *sv->reqs[id];
      if (r.prep.load(std::memory_order_acquire) != PREP_WAITING) continue;
      if (r.t_arrival <= sv->now()) {
        next = &r;
        break;
      }
      wake = std::min(wake, r.t_arrival);
    }
    if (!next) {
      if (wake < 1e300)
        sv->prep_cv.wait_for(lk, std::chrono::duration<double>(std::max(0.0, wake - sv->now())));
      else
        sv->prep_cv.wait(lk);
      continue;
    }
    next->prep.store(PREP_RUNNING, std::memory_order_relaxed);
    lk.unlock();
    const uint64_t k = GeoCache::key(*next);
    std::shared_ptr<const HostSetup> hs = sv->geo.find(k, *next);
    dg_status rc = DG_OK;
    std::string err;
    if (!hs) {
      std::shared_ptr<HostSetup> fresh(new HostSetup());
      dg_mesh m{next->E, next->n_geo, 0, next->x_geo.data(), next->nbr_elem.data(), next->nbr_face.data(),
                next->nbr_orient.data()};
      rc = setup_host(next->p, m, *fresh, err);
      if (rc == DG_OK) {
        sv->geo.insert(k, *next, fresh);
        hs = std::move(fresh);
      }
    }
    double dt = next->dt;
    if (rc == DG_OK && dt < 0.0) dt = host_stable_dt(next->p, next->E, *hs, next->U0.data(), -dt);
    size_t up = SIZE_MAX;
    if (rc == DG_OK && sv->up_host) {
      const size_t bytes = next->U0.size() * 8;
      bool got;
      {
        std::lock_guard<std::mutex> ul(sv->up_mu);
        got = sv->up_alloc.alloc(bytes, up);
      }
      if (got) std::memcpy(sv->up_host + up, next->U0.data(), bytes);
      else up = SIZE_MAX;
    }
    lk.lock();
    next->up_off = up;
    if (rc == DG_OK) {
      next->dt = dt;
      next->host = std::move(hs);
      next->prep.store(PREP_READY, std::memory_order_release);
    } else {
      next->prep_err = err;
      next->prep.store(PREP_FAILED, std::memory_order_release);
    }
  }
}

// take arena memory, evicting resident geometry blocks that no active
// request uses (least recently used first) until it fits
bool alloc_evicting(dg_server *sv, size_t bytes, size_t &off) {
  for (;;) {
    if (sv->alloc.alloc(bytes, off)) return true;
    auto lru = sv->dgeo.end();
    for (auto it = sv->dgeo.begin(); it != sv->dgeo.end(); ++it)
      if (it->second.refs == 0 && (lru == sv->dgeo.end() || it->second.used < lru->second.used)) lru = it;
    if (lru == sv->dgeo.end()) return false;
    sv->alloc.release(lru->second.off, lru->second.bytes);
    sv->dgeo.erase(lru);
  }
}

// admit the head of the queue while it fits
dg_status admit(dg_server *sv) {
  const double now = sv->now();
  while ((int)sv->active.size() < sv->max_active) {
    Request *rp;
    {
      std::lock_guard<std::mutex> lk(sv->prep_mu);
      if (sv->queue.empty()) break;
      rp = sv->reqs.at(sv->queue.front()).get();
    }
    Request &r = *rp;
    if (r.t_arrival > now) break;
    const int ps = r.prep.load(std::memory_order_acquire);
    if (ps == PREP_WAITING || ps == PREP_RUNNING) break;  // its set-up is still being made
    if (ps == PREP_FAILED) {  // the mesh passed the checks at submit but not the geometric ones
      {
        std::lock_guard<std::mutex> lk(sv->prep_mu);
        sv->queue.pop_front();
      }
      sv->prep_cv.notify_one();
      std::vector<double>().swap(r.U0);
      r.state = DG_REQ_FAILED;
      r.t_done = now;
      continue;
    }
    // the geometry block of its set-up: resident already, or uploaded now
    auto git = sv->dgeo.find(r.host.get());
    const bool geo_new = git == sv->dgeo.end();
    size_t goff = 0;
    if (geo_new && !alloc_evicting(sv, r.Lg.total, goff)) break;  // wait for memory to free up
    size_t off;
    if (!alloc_evicting(sv, r.L.total, off)) {
      if (geo_new) sv->alloc.release(goff, r.Lg.total);
      break;
    }
    {
      std::lock_guard<std::mutex> lk(sv->prep_mu);
      sv->queue.pop_front();
    }
    sv->prep_cv.notify_one();  // the next request in line may be prepared now
    hipError_t e = hipSuccess;
    if (geo_new) {
      dg_server::DevGeo g;
      g.hs = r.host;
      g.off = goff;
      g.bytes = r.Lg.total;
      e = upload_geometry(r.p, *r.host, sv->arena + goff, r.Lg, sv->cst);
      sv->st_upload_bytes += (double)r.host->bytes();
      ++sv->st_geo_uploads;
      git = sv->dgeo.emplace(r.host.get(), std::move(g)).first;
    } else {
      ++sv->st_geo_hits;
    }
    git->second.refs += 1;
    git->second.used = ++sv->dgeo_clock;
    r.geo_key = r.host.get();
    r.off = off;
    r.bytes = r.L.total;
    void *base = sv->arena + off;
    fill_view(r.vd, base, r.L, r.p, r.E);
    fill_view(r.vf, base, r.L, r.p, r.E);
    attach_geometry(r.vd, sv->arena + git->second.off, r.Lg);
    attach_geometry(r.vf, sv->arena + git->second.off, r.Lg);
    if (e == hipSuccess) e = hipMemsetAsync(base, 0, r.L.total, sv->cst);
    if (e == hipSuccess) {
      const void *src = r.up_off != SIZE_MAX ? (const void *)(sv->up_host + r.up_off) : (const void *)r.U0.data();
      e = hipMemcpyAsync((char *)base + r.L.U, src, r.U0.size() * 8, hipMemcpyHostToDevice, sv->cst);
    }
    sv->st_upload_bytes += (double)(r.U0.size() * 8);
    if (e == hipSuccess) {
      if (!sv->ev_free.empty()) {
        r.ready = sv->ev_free.back();
        sv->ev_free.pop_back();
      } else {
        e = hipEventCreateWithFlags(&r.ready, hipEventDisableTiming);
      }
    }
    if (e == hipSuccess) e = hipEventRecord(r.ready, sv->cst);
    if (e == hipSuccess) e = hipStreamWaitEvent(sv->st, r.ready, 0);
    if (e != hipSuccess) return server_fail(sv, e, "admission upload");
    r.state = DG_REQ_RUNNING;
    r.t_admit = sv->now();
    r.t = 0.0;
    r.step = r.stage = r.cur = r.bpar = 0;
    r.traces_valid = false;
    sv->active.push_back(r.id);
    if (r.n_steps == 0) r.step = r.n_steps;
  }
  return DG_OK;
}

template <typename real>
View<real> &view_of(Request &r);
template <>
View<double> &view_of<double>(Request &r) {
  return r.vd;
}
template <>
View<float> &view_of<float>(Request &r) {
  return r.vf;
}

// a view with its pointers turned into byte offsets from the arena (the form
// the batched kernels read; null stays null)
template <typename real>
View<real> as_offsets(View<real> v, const char *arena) {
  auto off = [arena](auto p) { return p ? (decltype(p))(intptr_t)((const char *)p - arena) : p; };
  v.U = off(v.U);
  v.dU = off(v.dU);
  v.R = off(v.R);
  v.Ja = off(v.Ja);
  v.invJ = off(v.invJ);
  v.NS = off(v.NS);
  v.Utr0 = off(v.Utr0);
  v.Utr1 = off(v.Utr1);
  v.Hv = off(v.Hv);
  v.Vol = off(v.Vol);
  v.conn = off(v.conn);
  v.Xs = off(v.Xs);
  v.basis = off(v.basis);
  v.alpha = off(v.alpha);
  v.alpha_raw = off(v.alpha_raw);
  v.alpha_in = off(v.alpha_in);
  v.bcnt = off(v.bcnt);
  v.blist = off(v.blist);
  return v;
}

// one batched launch of kernel k over the group; descriptors go through the ring
template <typename real>
dg_status launch_group(dg_server *sv, Kernel k, int N, const std::vector<Request *> &grp, hipStream_t st) {
  if (grp.empty()) return DG_OK;
  const int slot = sv->desc_next;
  sv->desc_next = (sv->desc_next + 1) % kDescSlots;
  // the kernel that last read this slot is done, so its host mirror and device
  // copy may be rewritten (that kernel may have run on another stream)
  const auto w0 = std::chrono::steady_clock::now();
  hipError_t e = hipEventSynchronize(sv->desc_ev[slot]);
  sv->st_gpu_wait += std::chrono::duration<double>(std::chrono::steady_clock::now() - w0).count();
  if (e != hipSuccess) return server_fail(sv, e, "descriptor ring");
  char *h = sv->desc_host[slot];
  View<real> *views = (View<real> *)h;
  int *blk = (int *)(h + sv->max_active * view_bytes());
  int total = 0;
  size_t gbytes = 0;
  for (size_t r = 0; r < grp.size(); ++r) {
    Request &q = *grp[r];
    View<real> v = view_of<real>(q);
    const double *A, *B, *C;
    rk_scheme(q.p.time_scheme, &A, &B, &C);
    v.t = q.t + C[q.stage] * q.dt;
    v.dt = q.dt;
    v.rkA = A[q.stage];
    v.rkB = B[q.stage];
    v.cur = q.cur;
    v.bpar = q.bpar;
    v.R = nullptr;
    views[r] = as_offsets(v, sv->arena);
    blk[r] = total;
    total += blocks_per_elements(N, q.E);
    gbytes += q.L.total;
  }
  blk[grp.size()] = total;
  char *d = sv->arena + slot * sv->desc_stride;
  e = hipMemcpyAsync(d, h, sv->desc_stride, hipMemcpyHostToDevice, st);
  // the argument view: the group's settings (shock capturing, viscosity) and the arena
  View<real> v0 = view_of<real>(*grp[0]);
  v0.base = sv->arena;
  v0.nt = gbytes >= kStreamBytes;  // the group's working set decides, as for a single solve
  if (e == hipSuccess)
    e = launch<real>(k, N, 0, (const View<real> *)d, (const int *)(d + sv->max_active * view_bytes()), (int)grp.size(),
                     total, v0, st);
  if (e == hipSuccess) e = hipEventRecord(sv->desc_ev[slot], st);
  if (e != hipSuccess) return server_fail(sv, e, "batched launch");
  return DG_OK;
}

// one RK stage for every active request
dg_status tick(dg_server *sv) {
  // one group per kernel set: degree, precision, shock capturing, viscosity,
  // volume form and nodes
  std::map<std::tuple<int, int, int, int, int>, std::vector<Request *>> groups;
  for (int64_t id : sv->active) {
    Request &r = *sv->reqs[id];
    if (r.retiring || r.step >= r.n_steps) continue;
    groups[{r.p.N, r.p.precision, r.p.shock_capturing, r.p.viscous, 2 * r.p.volume_flux + r.p.nodes}].push_back(&r);
  }
  if (groups.empty()) return DG_OK;
  hipError_t e = hipEventRecord(sv->fork_ev, sv->st);
  const int nst = std::min((int)groups.size(), kGroupStreams);
  for (int i = 0; i < nst && e == hipSuccess; ++i) e = hipStreamWaitEvent(sv->gst[i], sv->fork_ev, 0);
  if (e != hipSuccess) return server_fail(sv, e, "tick fork");
  int gi = 0;
  for (auto &kv : groups) {
    const int N = std::get<0>(kv.first);
    const bool mixed = std::get<1>(kv.first) == 1;
    hipStream_t gs = sv->gst[gi++ % kGroupStreams];
    std::vector<Request *> fresh, visc;
    for (Request *r : kv.second) {
      if (!r->traces_valid) fresh.push_back(r);
      if (r->p.viscous || r->p.shock_capturing || r->p.volume_flux) visc.push_back(r);
    }
    dg_status rc;
    rc = mixed ? launch_group<float>(sv, K_TRACE, N, fresh, gs) : launch_group<double>(sv, K_TRACE, N, fresh, gs);
    if (rc) return rc;
    rc = mixed ? launch_group<float>(sv, K_LIFT, N, visc, gs) : launch_group<double>(sv, K_LIFT, N, visc, gs);
    if (rc) return rc;
    rc = mixed ? launch_group<float>(sv, K_RHS, N, kv.second, gs) : launch_group<double>(sv, K_RHS, N, kv.second, gs);
    if (rc) return rc;
    for (Request *r : kv.second) {
      r->traces_valid = true;
      r->cur ^= 1;
      r->bpar ^= 1;
      const double *A, *B, *C;
      if (++r->stage == rk_scheme(r->p.time_scheme, &A, &B, &C)) {
        r->stage = 0;
        ++r->step;
        r->t = r->step * r->dt;
      }
    }
  }
  // join: retirement and the next tick's work follow every group's launches
  for (int i = 0; i < nst && e == hipSuccess; ++i) {
    e = hipEventRecord(sv->join_ev[i], sv->gst[i]);
    if (e == hipSuccess) e = hipStreamWaitEvent(sv->st, sv->join_ev[i], 0);
  }
  if (e != hipSuccess) return server_fail(sv, e, "tick join");
  return DG_OK;
}

// give a staged initial state's pinned memory back (its upload has landed)
void release_upload(dg_server *sv, Request &r) {
  if (r.up_off == SIZE_MAX) return;
  std::lock_guard<std::mutex> ul(sv->up_mu);
  sv->up_alloc.release(r.up_off, r.U0.size() * 8);
  r.up_off = SIZE_MAX;
}

// Copy finished requests out through the staging slots; release a request's
// memory once its whole state has landed on the host.
dg_status retire(dg_server *sv) {
  // staging copies that have completed: into the requests' results
  for (StageSlot &sl : sv->slots) {
    if (!sl.busy) continue;
    hipError_t q = hipEventQuery(sl.ev);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess) return server_fail(sv, q, "retirement copy");
    Request &r = *sv->reqs[sl.req];
    std::memcpy((char *)r.result.data() + sl.off, sl.host, sl.bytes);
    if (sl.flag) r.bad = *(const int *)(sl.host + kStageChunk) != 0;
    r.copied += sl.bytes;
    sl.busy = false;
  }
  std::vector<int64_t> keep;
  for (int64_t id : sv->active) {
    Request &r = *sv->reqs[id];
    const size_t total = (size_t)5 * r.E * (r.p.N + 1) * (r.p.N + 1) * (r.p.N + 1) * 8;
    int *flag = (int *)(sv->arena + r.off + r.L.scratch);
    const double *U = (const double *)(sv->arena + r.off + r.L.U);
    if (!r.retiring && r.step >= r.n_steps) {
      // the finiteness check runs after the last stage, before the copies
      hipError_t e = launch_zero_int(flag, 1, sv->st);
      if (e == hipSuccess) e = launch_finite(U, (int64_t)(total / 8), flag, sv->st);
      if (e != hipSuccess) return server_fail(sv, e, "retirement check");
      r.result.resize(total / 8);
      r.retiring = true;
      r.issued = r.copied = 0;
      r.bad = false;
    }
    if (r.retiring) {
      for (StageSlot &sl : sv->slots) {
        if (r.issued >= total) break;
        if (sl.busy) continue;
        sl.req = id;
        sl.off = r.issued;
        sl.bytes = std::min(kStageChunk, total - r.issued);
        sl.flag = r.issued + sl.bytes == total;
        hipError_t e = hipMemcpyAsync(sl.host, (const char *)U + sl.off, sl.bytes, hipMemcpyDeviceToHost, sv->st);
        if (e == hipSuccess && sl.flag)
          e = hipMemcpyAsync(sl.host + kStageChunk, flag, sizeof(int), hipMemcpyDeviceToHost, sv->st);
        if (e == hipSuccess) e = hipEventRecord(sl.ev, sv->st);
        if (e != hipSuccess) return server_fail(sv, e, "retirement copy");
        sl.busy = true;
        r.issued += sl.bytes;
      }
      if (r.copied < total) {
        keep.push_back(id);
        continue;
      }
      if (r.ready) sv->ev_free.push_back(r.ready);
      r.ready = nullptr;
      r.host.reset();
      release_upload(sv, r);  // its upload has landed: the copy-out followed it on the stream
      sv->alloc.release(r.off, r.bytes);
      sv->dgeo.at(r.geo_key).refs -= 1;  // the block stays resident for the next request of this mesh
      r.geo_key = nullptr;
      r.state = r.bad ? DG_REQ_FAILED : DG_REQ_DONE;
      r.t_done = sv->now();
      continue;
    }
    // the host set-up and initial state can go once their uploads have landed
    if (r.host && r.ready && hipEventQuery(r.ready) == hipSuccess) {
      r.host.reset();
      release_upload(sv, r);
      std::vector<double>().swap(r.U0);
    }
    keep.push_back(id);
  }
  sv->active.swap(keep);
  return DG_OK;
}

}  // namespace

extern "C" {

dg_status dg_server_create(void *d_arena, size_t arena_bytes, size_t hbm_budget, int32_t max_active, void *hip_stream,
                           void *hip_copy_stream, dg_server **out) {
  if (!out) return fail(DG_EINVAL, "out is NULL");
  *out = nullptr;
  if (!d_arena || (uintptr_t)d_arena % 256) return fail(DG_EINVAL, "arena must be non-NULL and 256-byte aligned");
  if (max_active < 1 || max_active > 4096) return fail(DG_EINVAL, "max_active must be in 1..4096");
  std::unique_ptr<dg_server> sv(new dg_server());
  sv->arena = (char *)d_arena;
  sv->arena_bytes = arena_bytes;
  sv->max_active = max_active;
  sv->st = (hipStream_t)hip_stream;
  sv->cst = hip_copy_stream ? (hipStream_t)hip_copy_stream : sv->st;
  sv->desc_stride = ((max_active * view_bytes() + (max_active + 1) * sizeof(int)) + 255) & ~size_t(255);
  const size_t head = kDescSlots * sv->desc_stride;
  if (arena_bytes <= head) return fail(DG_ENOMEM, "arena smaller than the descriptor ring");
  sv->budget = std::min(hbm_budget, arena_bytes - head);
  sv->alloc.init(head, sv->budget);
  for (int s = 0; s < kDescSlots; ++s) {
    hipError_t e = hipHostMalloc((void **)&sv->desc_host[s], sv->desc_stride, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sv->desc_ev[s], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(sv->desc_ev[s], sv->st);
    if (e != hipSuccess) return fail(DG_EDEVICE, std::string("server set-up: ") + hipGetErrorString(e));
  }
  if (hipHostMalloc((void **)&sv->up_host, kUpStageBytes, hipHostMallocDefault) == hipSuccess)
    sv->up_alloc.init(0, kUpStageBytes);
  else
    sv->up_host = nullptr;  // no staging area: initial states go from pageable memory
  for (StageSlot &sl : sv->slots) {
    hipError_t e = hipHostMalloc((void **)&sl.host, kStageChunk + 256, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming);
    if (e != hipSuccess) {
      for (StageSlot &t : sv->slots) {
        if (t.host) (void)hipHostFree(t.host);
        if (t.ev) (void)hipEventDestroy(t.ev);
      }
      for (int q = 0; q < kDescSlots; ++q) {
        if (sv->desc_host[q]) (void)hipHostFree(sv->desc_host[q]);
        if (sv->desc_ev[q]) (void)hipEventDestroy(sv->desc_ev[q]);
      }
      if (sv->up_host) (void)hipHostFree(sv->up_host);
      return fail(DG_EDEVICE, std::string("server staging: ") + hipGetErrorString(e));
    }
  }
  {
    hipError_t e = hipEventCreateWithFlags(&sv->fork_ev, hipEventDisableTiming);
    for (int i = 0; i < kGroupStreams && e == hipSuccess; ++i) {
      e = hipStreamCreateWithFlags(&sv->gst[i], hipStreamNonBlocking);  // default priority
      if (e == hipSuccess) e = hipEventCreateWithFlags(&sv->join_ev[i], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
      for (int i = 0; i < kGroupStreams; ++i) {
        if (sv->gst[i]) (void)hipStreamDestroy(sv->gst[i]);
        if (sv->join_ev[i]) (void)hipEventDestroy(sv->join_ev[i]);
      }
      if (sv->fork_ev) (void)hipEventDestroy(sv->fork_ev);
      for (int s = 0; s < kDescSlots; ++s) {
        if (sv->desc_host[s]) (void)hipHostFree(sv->desc_host[s]);
        if (sv->desc_ev[s]) (void)hipEventDestroy(sv->desc_ev[s]);
      }
      for (StageSlot &t : sv->slots) {
        (void)hipHostFree(t.host);
        (void)hipEventDestroy(t.ev);
      }
      if (sv->up_host) (void)hipHostFree(sv->up_host);
      return fail(DG_EDEVICE, std::string("server streams: ") + hipGetErrorString(e));
    }
  }
  sv->prep_thread = std::thread(prep_loop, sv.get());
  *out = sv.release();
  return DG_OK;
}

dg_status dg_server_submit(dg_server *sv, const dg_params *p, const dg_mesh *m, const double *U0_host, int32_t n_steps,
                           double dt, double t_arrival, int64_t *req_id) {
  if (!sv) return fail(DG_EINVAL, "server is NULL");
  if (sv->broken) return fail(DG_ESTATE, "server unusable after a device error");
  dg_status rc = check_params(p);
  if (rc) return rc;
  if (!m || !m->x_geo || !m->nbr_elem || !m->nbr_face || !m->nbr_orient || !U0_host || !req_id)
    return fail(DG_EINVAL, "missing mesh, state or id pointer");
  if (!elems_in_range(p->N, m->n_elems) || m->n_geo < 1 || m->n_geo > p->N)
    return fail(DG_EINVAL, "bad mesh sizes");
  if (n_steps < 0 || !std::isfinite(dt) || dt == 0.0) return fail(DG_EINVAL, "need n_steps >= 0 and dt != 0");
  if (!std::isfinite(t_arrival) || t_arrival < 0.0) return fail(DG_EINVAL, "t_arrival must be finite and >= 0");
  std::unique_ptr<Request> r(new Request());
  r->id = sv->next_id++;
  r->p = *p;
  r->E = m->n_elems;
  r->n_geo = m->n_geo;
  r->L = make_layout(*p, r->E, LAYOUT_STATE);
  r->Lg = make_layout(*p, r->E, LAYOUT_GEOMETRY);
  if (r->L.total + r->Lg.total > sv->budget) return fail(DG_EBUSY, "request can never fit the memory budget");
  const int ng = m->n_geo + 1, n = p->N + 1;
  r->x_geo.assign(m->x_geo, m->x_geo + (size_t)r->E * 3 * ng * ng * ng);
  r->nbr_elem.assign(m->nbr_elem, m->nbr_elem + r->E * 6);
  r->nbr_face.assign(m->nbr_face, m->nbr_face + r->E * 6);
  r->nbr_orient.assign(m->nbr_orient, m->nbr_orient + r->E * 6);
  r->U0.assign(U0_host, U0_host + (size_t)5 * r->E * n * n * n);
  r->n_steps = n_steps;
  r->dt = dt;
  r->t_arrival = t_arrival;
  *req_id = r->id;
  {
    std::lock_guard<std::mutex> lk(sv->prep_mu);
    sv->queue.push_back(r->id);
    sv->reqs[r->id] = std::move(r);
  }
  sv->prep_cv.notify_one();
  return DG_OK;
}

dg_status dg_server_run(dg_server *sv, int32_t max_ticks) {
  if (!sv) return fail(DG_EINVAL, "server is NULL");
  if (sv->broken) return fail(DG_ESTATE, "server unusable after a device error");
  if (!sv->started.load(std::memory_order_relaxed)) {
    {
      std::lock_guard<std::mutex> lk(sv->prep_mu);
      sv->t0 = std::chrono::steady_clock::now();
      sv->started.store(true, std::memory_order_release);
    }
    sv->prep_cv.notify_all();  // arrival times are on the clock that starts now
  }
  int ticks = 0;
  using clk = std::chrono::steady_clock;
  auto secs = [](clk::time_point a) { return std::chrono::duration<double>(clk::now() - a).count(); };
  for (;;) {
    auto c0 = clk::now();
    dg_status rc = admit(sv);
    sv->st_admit += secs(c0);
    if (rc) return rc;
    if (sv->active.empty()) {
      double head_arrival;
      {
        std::lock_guard<std::mutex> lk(sv->prep_mu);
        if (sv->queue.empty()) break;
        head_arrival = sv->reqs.at(sv->queue.front())->t_arrival;
      }
      // nothing runs: wait for the next arrival, or for its set-up
      const double wait = std::max(head_arrival - sv->now(), 0.0005);
      c0 = clk::now();
      std::this_thread::sleep_for(std::chrono::duration<double>(std::min(wait, 0.01)));
      sv->st_idle += secs(c0);
      if (max_ticks > 0 && ++ticks >= max_ticks) break;
      continue;
    }
    c0 = clk::now();
    sv->st_active_sum += (int64_t)sv->active.size();
    ++sv->st_ticks;
    rc = tick(sv);
    sv->st_tick += secs(c0);
    if (rc) return rc;
    c0 = clk::now();
    rc = retire(sv);
    sv->st_retire += secs(c0);
    if (rc) return rc;
    if (max_ticks > 0 && ++ticks >= max_ticks) break;
  }
  return DG_OK;
}

dg_status dg_server_poll(dg_server *sv, int64_t req_id, int32_t *state) {
  if (!sv || !state) return fail(DG_EINVAL, "NULL argument");
  auto it = sv->reqs.find(req_id);
  if (it == sv->reqs.end()) return fail(DG_EINVAL, "unknown request");
  *state = it->second->state;
  return DG_OK;
}

dg_status dg_server_fetch(dg_server *sv, int64_t req_id, double *U_host, dg_timing *timing) {
  if (!sv) return fail(DG_EINVAL, "server is NULL");
  auto it = sv->reqs.find(req_id);
  if (it == sv->reqs.end()) return fail(DG_EINVAL, "unknown request");
  Request &r = *it->second;
  if (timing) {
    timing->t_arrival = r.t_arrival;
    timing->t_admit = r.t_admit;
    timing->t_done = r.t_done;
    timing->state = r.state;
    timing->reserved = 0;
  }
  if (r.state != DG_REQ_DONE && r.state != DG_REQ_FAILED) return fail(DG_ESTATE, "request not finished");
  if (U_host && !r.result.empty()) std::memcpy(U_host, r.result.data(), r.result.size() * 8);
  return r.state == DG_REQ_DONE ? DG_OK : fail(DG_ENONFINITE, "request failed: state not finite");
}

dg_status dg_server_stats(dg_server *sv, double out[10]) {
  if (!sv || !out) return fail(DG_EINVAL, "NULL argument");
  out[8] = (double)sv->st_geo_uploads;
  out[9] = (double)sv->st_geo_hits;
  out[0] = (double)sv->st_ticks;
  out[1] = sv->st_ticks ? (double)sv->st_active_sum / (double)sv->st_ticks : 0.0;
  out[2] = sv->st_admit;
  out[3] = sv->st_tick;
  out[4] = sv->st_retire;
  out[5] = sv->st_gpu_wait;
  out[6] = sv->st_idle;
  out[7] = sv->st_upload_bytes;
  return DG_OK;
}

void dg_server_destroy(dg_server *sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->prep_mu);
    sv->prep_stop = true;
  }
  sv->prep_cv.notify_all();
  if (sv->prep_thread.joinable()) sv->prep_thread.join();
  (void)hipStreamSynchronize(sv->st);
  if (sv->cst != sv->st) (void)hipStreamSynchronize(sv->cst);
  for (auto &kv : sv->reqs) {
    Request &r = *kv.second;
    if (r.ready) (void)hipEventDestroy(r.ready);
  }
  for (hipEvent_t ev : sv->ev_free) (void)hipEventDestroy(ev);
  for (StageSlot &sl : sv->slots) {
    if (sl.host) (void)hipHostFree(sl.host);
    if (sl.ev) (void)hipEventDestroy(sl.ev);
  }
  if (sv->up_host) (void)hipHostFree(sv->up_host);
  for (int i = 0; i < kGroupStreams; ++i) {
    if (sv->gst[i]) {
      (void)hipStreamSynchronize(sv->gst[i]);
      (void)hipStreamDestroy(sv->gst[i]);
    }
    if (sv->join_ev[i]) (void)hipEventDestroy(sv->join_ev[i]);
  }
  if (sv->fork_ev) (void)hipEventDestroy(sv->fork_ev);
  for (int s = 0; s < kDescSlots; ++s) {
    if (sv->desc_host[s]) (void)hipHostFree(sv->desc_host[s]);
    if (sv->desc_ev[s]) (void)hipEventDestroy(sv->desc_ev[s]);
  }
  delete sv;
}

}  // extern "C"
