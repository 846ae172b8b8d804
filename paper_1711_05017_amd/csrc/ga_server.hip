// ga_server.hip -- serving loop of libga.so: resident pair data, queued
// pose queries, continuous batching per grid size (see include/ga.h).
//
// Host side: one mutex guards pairs, queues, tickets and byte accounting; a
// scheduler thread owns the launch groups. Per grid size there are up to two
// launch groups sharing the size's stream, each with its own scratch; a group
// takes up to max_slots queued queries as soon as it is free, so new arrivals
// are admitted while the other group (and the groups of other sizes) run.
// While groups are in flight the scheduler sleeps on its condition variable
// for at most 20 us at a time (woken early by submissions) and then looks at
// their completion events: no spinning core, and no host callback (whose
// wake-up measured ~80 us at the median). With nothing in flight it sleeps
// until a submission arrives.
// Device side per group, spectral mode: k_bin_items (placement of every
// query's rotated samples), the fused single-translation pass
// (k_plane_single: splat, z and y transforms of the 4 channels and each
// plane's share of the 7 sums against the pair's resident AX), the sum over
// planes, one copy of the results to pinned host memory. Local mode:
// k_local_query and the sum over sample blocks.
// Test executor (ga_server_cfg.mock_fn): the same scheduling with no device
// memory and no launches; a group's results come from the callback at
// launch and its completion is reported mock_launch_us later.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>

#include <sys/prctl.h>
#include <vector>

#include "ga.h"
#include "ga_launch.hpp"

using namespace ga;
using namespace ga_detail;

namespace {

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Pair {
  uint32_t id = 0;
  int n = 0;
  float sigma = 0.f;
  float cB[3] = {0, 0, 0};
  float* d_xyzr = nullptr;  // moving part's samples (device copy)
  float* d_w = nullptr;
  int64_t n_pts = 0;
  float2* d_AX = nullptr;  // spectral mode: AX and DX of the stationary part (ga_pose_prepare)
  float* d_FA = nullptr;   // local mode: (u_A, grad u_A) per voxel
  size_t bytes = 0;
  int inflight = 0;  // queued or running queries
  bool released = false;
};

struct Pending {
  uint64_t ticket;
  uint32_t pair;
  float R[9];
  int t[3];
  uint64_t t_submit;
};

struct Group {
  hipStream_t stream = nullptr;  // the size class's stream
  hipEvent_t done = nullptr;
  QueryItem* h_items = nullptr;  // pinned
  QueryItem* d_items = nullptr;
  float* h_out = nullptr;  // pinned, slots x 7
  float* d_out = nullptr;
  Placed* rec = nullptr;
  int* off = nullptr;
  float* rmax = nullptr;
  int4* cand = nullptr;
  double* part = nullptr;
  std::vector<Pending> batch;
  uint64_t t_start = 0;
  bool busy = false;
  // test executor: results computed at launch, reported at ready_ns
  bool mock = false;
  std::vector<float> mock_out;
  uint64_t ready_ns = 0;
  bool mock_failed = false;
};

struct SizeClass {
  int n = 0;
  float sigma = 0.f;
  ga_plan* plan = nullptr;
  int slots = 0;
  int64_t max_pts = 0;  // record capacity per query
  int ngroups = 0;
  hipStream_t stream = nullptr;  // shared by the class's groups
  Group groups[2];
  std::deque<Pending> queue;
  size_t bytes = 0;
  bool paused = false;  // set while the scratch is being resized
};

struct Ticket {
  bool done = false;
  ga_result r{};
};

size_t group_bytes(uint32_t mode, int n, int slots, int64_t max_pts) {
  const size_t common = (size_t)slots * (7 * sizeof(float) + sizeof(QueryItem));
  if (mode == GA_SERVE_LOCAL) return common + (size_t)slots * nlocal_of(max_pts) * 7 * sizeof(double);
  const size_t nblk = (size_t)single_blocks_of(n);
  return common + (size_t)slots * ((size_t)max_pts * sizeof(Placed) + (size_t)(n + 1) * sizeof(int) + sizeof(float) +
                                   (size_t)n * sizeof(int4) + nblk * 7 * sizeof(double));
}

void free_group(Group& g) {
  if (g.mock) {
    g = Group{};
    return;
  }
  if (g.stream) (void)hipStreamSynchronize(g.stream);
  if (g.h_items) (void)hipHostFree(g.h_items);
  if (g.h_out) (void)hipHostFree(g.h_out);
  for (void* p : {(void*)g.d_items, (void*)g.d_out, (void*)g.rec, (void*)g.off, (void*)g.rmax, (void*)g.cand,
                  (void*)g.part})
    if (p) (void)hipFree(p);
  if (g.done) (void)hipEventDestroy(g.done);
  g = Group{};
}

bool alloc_group(Group& g, hipStream_t stream, uint32_t mode, int n, int slots, int64_t max_pts, bool mock) {
  if (mock) {
    g.mock = true;
    g.mock_out.assign((size_t)slots * 7, 0.f);
    return true;
  }
  g.stream = stream;
  bool ok = hipEventCreateWithFlags(&g.done, hipEventDisableTiming) == hipSuccess &&
            hipHostMalloc((void**)&g.h_items, sizeof(QueryItem) * slots, hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc((void**)&g.h_out, sizeof(float) * 7 * slots, hipHostMallocDefault) == hipSuccess &&
            hipMalloc(&g.d_items, sizeof(QueryItem) * slots) == hipSuccess &&
            hipMalloc(&g.d_out, sizeof(float) * 7 * slots) == hipSuccess;
  if (ok && mode == GA_SERVE_LOCAL) {
    ok = hipMalloc(&g.part, sizeof(double) * (size_t)nlocal_of(max_pts) * 7 * slots) == hipSuccess;
  } else if (ok) {
    const size_t nblk = (size_t)single_blocks_of(n);
    ok = hipMalloc(&g.rec, sizeof(Placed) * (size_t)max_pts * slots) == hipSuccess &&
         hipMalloc(&g.off, sizeof(int) * (size_t)(n + 1) * slots) == hipSuccess &&
         hipMalloc(&g.rmax, sizeof(float) * slots) == hipSuccess &&
         hipMalloc(&g.cand, sizeof(int4) * (size_t)n * slots) == hipSuccess &&
         hipMalloc(&g.part, sizeof(double) * nblk * 7 * slots) == hipSuccess;
  }
  if (!ok) free_group(g);
  return ok;
}

bool host_part_ok(const ga_part* p, int n, bool allow_empty) {
  if (!p || p->n_pts < 0 || (p->n_pts > 0 && (!p->xyzr || !p->w)) || (!allow_empty && p->n_pts == 0)) return false;
  for (int64_t i = 0; i < p->n_pts; ++i) {
    const float* q = p->xyzr + 4 * i;
    if (!(std::isfinite(q[0]) && std::isfinite(q[1]) && std::isfinite(q[2]) && std::isfinite(q[3]) &&
          std::isfinite(p->w[i])))
      return false;
    if (!(std::fmax(q[3], 1.0f) < 0.5f * n)) return false;
  }
  return true;
}

}  // namespace

struct ga_server {
  int device = 0;
  uint32_t mode = GA_SERVE_LOCAL;
  uint64_t budget = 0;
  int max_slots = 0;
  int queue_depth = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::unordered_map<uint32_t, Pair> pairs;
  uint32_t next_pair = 1;
  std::vector<std::unique_ptr<SizeClass>> classes;
  std::unordered_map<uint64_t, Ticket> tickets;
  uint64_t next_ticket = 1;
  size_t bytes = 0;
  int queued = 0;
  int busy_groups = 0;
  ga_server_stats stats{};
  bool stop = false;
  ga_status sticky = GA_OK;
  std::thread worker;
  // test executor (ga_server_cfg.mock_fn)
  ga_mock_query_fn mock_fn = nullptr;
  void* mock_user = nullptr;
  uint32_t mock_launch_us = 0;
  bool mock() const { return mock_fn != nullptr; }

  SizeClass* find_class(int n, float sigma) {
    for (auto& c : classes)
      if (c->n == n && c->sigma == sigma) return c.get();
    return nullptr;
  }
  void free_pair_locked(Pair& p) {
    for (void* q : {(void*)p.d_xyzr, (void*)p.d_w, (void*)p.d_AX, (void*)p.d_FA})
      if (q) (void)hipFree(q);  // all null under the test executor
    bytes -= p.bytes;
  }
  // After a sticky error nothing is launched any more: every queued query
  // is dropped (its ticket then polls as the sticky error), so that the
  // scheduler can drain and ga_server_destroy return (caller holds mu).
  void fail_queued_locked() {
    for (auto& cp : classes) {
      for (const Pending& q : cp->queue) {
        auto pit = pairs.find(q.pair);
        if (pit != pairs.end() && --pit->second.inflight == 0 && pit->second.released) {
          free_pair_locked(pit->second);
          pairs.erase(pit);
        }
      }
      queued -= (int)cp->queue.size();
      cp->queue.clear();
    }
    stats.pairs = (int32_t)pairs.size();
  }
  void run();
  void launch(SizeClass& c, Group& g);
  void launch_mock(SizeClass& c, Group& g);
  void harvest_locked(Group& g, bool ok, uint64_t t_done);
};

// Fills the pinned descriptors of a group from its batch (caller holds mu).
static void fill_items(ga_server* s, SizeClass& c, Group& g) {
  for (size_t i = 0; i < g.batch.size(); ++i) {
    const Pending& q = g.batch[i];
    const Pair& p = s->pairs.at(q.pair);
    QueryItem it{};
    it.xyzr = reinterpret_cast<const float4*>(p.d_xyzr);
    it.w = p.d_w;
    it.n_pts = p.n_pts;
    it.AX = p.d_AX;
    it.FA = reinterpret_cast<const float4*>(p.d_FA);
    std::memcpy(it.R, q.R, sizeof(it.R));
    std::memcpy(it.c, p.cB, sizeof(it.c));
    std::memcpy(it.t, q.t, sizeof(it.t));
    g.h_items[i] = it;
  }
  (void)c;
}

void ga_server::launch(SizeClass& c, Group& g) {
  const int k = (int)g.batch.size();
  const int n = c.n;
  (void)hipMemcpyAsync(g.d_items, g.h_items, sizeof(QueryItem) * k, hipMemcpyHostToDevice, g.stream);
  SplatParams base = make_splat(nullptr, nullptr, 0, nullptr, nullptr, nullptr, c.sigma);
  const float2* tw = c.plan->d_tw;
  int nblk = 0;
  double scale = 1.0;
  if (mode == GA_SERVE_LOCAL) {
    nblk = nlocal_of(c.max_pts);
    dispatch(n, [&]<int N>() {
      hipLaunchKernelGGL(k_local_query<N>, dim3(nblk, k), dim3(256), 0, g.stream, (const QueryItem*)g.d_items, g.part,
                         base.sig_c, base.e0, base.inv1me0);
    });
  } else {
    nblk = single_blocks_of(n);
    scale = 1.0 / ((double)n * n * n);
    dispatch(n, [&]<int N>() {
      hipLaunchKernelGGL(k_bin_items<N>, dim3(k), dim3(1024), 0, g.stream, g.d_items, base, (long long)c.max_pts, g.rec,
                         g.off, g.rmax, g.cand);
      SplatParams sp = base;
      sp.rec = g.rec;
      sp.off = g.off;
      sp.rmax = g.rmax;
      sp.cand = g.cand;
      sp.n_pts = c.max_pts;
      Launch<N>::plane_single(sp, g.d_items, g.part, k, tw, g.stream);
    });
  }
  hipLaunchKernelGGL(k_reduce_partials, dim3(k), dim3(64), 0, g.stream, (const double*)g.part, nblk, g.d_out, scale,
                     (const QueryItem*)nullptr);  // translations were checked by ga_submit
  (void)hipMemcpyAsync(g.h_out, g.d_out, sizeof(float) * 7 * k, hipMemcpyDeviceToHost, g.stream);
  (void)hipEventRecord(g.done, g.stream);
}

// Test executor: the group's results from mock_fn now (scheduler thread,
// server lock not held), its completion mock_launch_us later.
void ga_server::launch_mock(SizeClass& c, Group& g) {
  g.mock_failed = false;
  for (size_t i = 0; i < g.batch.size(); ++i) {
    const Pending& q = g.batch[i];
    if (mock_fn(mock_user, q.pair, c.n, q.R, q.t, g.mock_out.data() + 7 * i) != 0) g.mock_failed = true;
  }
  g.ready_ns = g.t_start + (uint64_t)mock_launch_us * 1000u;
}

// Results of a finished group to its tickets; frees released pairs whose
// last query this was (caller holds mu).
void ga_server::harvest_locked(Group& g, bool ok, uint64_t t_done) {
  for (size_t i = 0; i < g.batch.size(); ++i) {
    const Pending& q = g.batch[i];
    auto it = tickets.find(q.ticket);
    if (it != tickets.end() && ok) {
      ga_result& r = it->second.r;
      const float* o = (g.mock ? g.mock_out.data() : g.h_out) + 7 * i;
      r.E = o[0];
      r.F[0] = o[1];
      r.F[1] = o[2];
      r.F[2] = o[3];
      r.tau[0] = o[4];
      r.tau[1] = o[5];
      r.tau[2] = o[6];
      r.t_submit_ns = q.t_submit;
      r.t_start_ns = g.t_start;
      r.t_done_ns = t_done;
      it->second.done = true;
    }
    auto pit = pairs.find(q.pair);
    if (pit != pairs.end() && --pit->second.inflight == 0 && pit->second.released) {
      free_pair_locked(pit->second);
      pairs.erase(pit);
    }
  }
  stats.completed += g.batch.size();
  g.batch.clear();
  g.busy = false;
  --busy_groups;
}

void ga_server::run() {
  if (!mock()) (void)hipSetDevice(device);
  (void)prctl(PR_SET_TIMERSLACK, 1000UL);  // 1 us: the short waits below stay short
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    if (sticky != GA_OK && queued > 0) fail_queued_locked();
    // retire finished groups (an event query does not block)
    bool progress = false;
    for (auto& cp : classes)
      for (int gi = 0; gi < cp->ngroups; ++gi) {
        Group& g = cp->groups[gi];
        if (!g.busy) continue;
        if (g.mock) {
          const uint64_t t = now_ns();
          if (t < g.ready_ns) continue;
          if (g.mock_failed) sticky = GA_EDEVICE;
          harvest_locked(g, !g.mock_failed, t);
          progress = true;
          continue;
        }
        const hipError_t e = hipEventQuery(g.done);
        if (e == hipErrorNotReady) continue;
        if (e != hipSuccess) sticky = GA_EDEVICE;
        harvest_locked(g, e == hipSuccess, now_ns());
        progress = true;
      }
    // fill free groups with queued queries (continuous batching)
    std::vector<std::pair<SizeClass*, Group*>> to_launch;
    for (auto& cp : classes) {
      SizeClass& c = *cp;
      for (int gi = 0; gi < c.ngroups; ++gi) {
        Group& g = c.groups[gi];
        if (g.busy || c.paused || c.queue.empty() || sticky != GA_OK) continue;
        const int k = (int)std::min<size_t>(c.queue.size(), (size_t)c.slots);
        g.batch.assign(c.queue.begin(), c.queue.begin() + k);
        c.queue.erase(c.queue.begin(), c.queue.begin() + k);
        queued -= k;
        if (!g.mock) fill_items(this, c, g);
        g.busy = true;
        g.t_start = now_ns();
        ++busy_groups;
        stats.launches += 1;
        to_launch.push_back({&c, &g});
      }
    }
    if (!to_launch.empty()) {
      lk.unlock();
      for (auto& [c, g] : to_launch) {
        if (g->mock) launch_mock(*c, *g);
        else launch(*c, *g);
      }
      lk.lock();
      continue;
    }
    if (progress) continue;
    if (stop && queued == 0 && busy_groups == 0) break;
    // sleep: briefly while groups run (their events are looked at again),
    // else until a submission or stop
    if (busy_groups > 0) cv.wait_for(lk, std::chrono::microseconds(20));
    else cv.wait_for(lk, std::chrono::milliseconds(50));
  }
}

extern "C" {

ga_status ga_server_create(ga_server** server, const ga_server_cfg* cfg) {
  if (!server || !cfg) return GA_EINVAL;
  *server = nullptr;
  if (cfg->max_slots < 1 || cfg->max_slots > 256 || cfg->queue_depth < 1 || cfg->hbm_budget_bytes == 0 ||
      (cfg->mode != GA_SERVE_LOCAL && cfg->mode != GA_SERVE_SPECTRAL))
    return GA_EINVAL;
  if (!cfg->mock_fn) {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || cfg->device < 0 || cfg->device >= ndev) return GA_EINVAL;
  }
  ga_server* s = new (std::nothrow) ga_server();
  if (!s) return GA_ENOMEM;
  s->mock_fn = cfg->mock_fn;
  s->mock_user = cfg->mock_user;
  s->mock_launch_us = cfg->mock_launch_us;
  s->device = cfg->device;
  s->mode = cfg->mode;
  s->budget = cfg->hbm_budget_bytes;
  s->max_slots = cfg->max_slots;
  s->queue_depth = cfg->queue_depth;
  s->worker = std::thread([s] { s->run(); });
  *server = s;
  return GA_OK;
}

ga_status ga_server_destroy(ga_server* s) {
  if (!s) return GA_EINVAL;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  s->worker.join();
  if (!s->mock()) (void)hipSetDevice(s->device);
  for (auto& cp : s->classes) {
    for (int gi = 0; gi < cp->ngroups; ++gi) free_group(cp->groups[gi]);
    if (cp->stream) (void)hipStreamDestroy(cp->stream);
    if (cp->plan) ga_plan_destroy(cp->plan);
  }
  for (auto& kv : s->pairs) s->free_pair_locked(kv.second);
  delete s;
  return GA_OK;
}

ga_status ga_pair_register(ga_server* s, const ga_part* A, const ga_part* B, const float cB[3], int32_t n, float sigma,
                           uint32_t* pair_id) {
  if (!s || !pair_id || !cB || !valid_sigma(sigma)) return GA_EINVAL;
  if (!plane_edge(n)) return GA_EUNSUPPORTED;  // served sizes use the plane path
  if (!host_part_ok(A, n, true) || !host_part_ok(B, n, false)) return GA_EINVAL;
  if (!(std::isfinite(cB[0]) && std::isfinite(cB[1]) && std::isfinite(cB[2]))) return GA_EINVAL;
  const bool mock = s->mock();
  if (!mock && hipSetDevice(s->device) != hipSuccess) return GA_EDEVICE;
  const size_t spec_bytes = spectrum_elems(n) * sizeof(float2);
  const size_t n3 = (size_t)n * n * n;
  const size_t pair_bytes = (size_t)B->n_pts * 5 * sizeof(float) + (s->mode == GA_SERVE_LOCAL ? 16 * n3 : 2 * spec_bytes);
  SizeClass* c = nullptr;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->sticky != GA_OK) return s->sticky;
    c = s->find_class(n, sigma);
    if (!c) {
      // new size class: two launch groups of max_slots, fewer if the budget is short
      auto nc = std::make_unique<SizeClass>();
      nc->n = n;
      nc->sigma = sigma;
      nc->max_pts = B->n_pts;
      int slots = s->max_slots, ngroups = 2;
      while (s->bytes + pair_bytes + (size_t)ngroups * group_bytes(s->mode, n, slots, nc->max_pts) > s->budget) {
        if (slots > 1) slots = (slots + 1) / 2;
        else if (ngroups > 1) ngroups = 1;
        else return GA_ENOMEM;
      }
      if (!mock) {
        if (ga_plan_create(&nc->plan, n, slots, 0) != GA_OK) return GA_EDEVICE;
        if (hipStreamCreateWithFlags(&nc->stream, hipStreamNonBlocking) != hipSuccess) {
          ga_plan_destroy(nc->plan);
          return GA_EDEVICE;
        }
      }
      for (int gi = 0; gi < ngroups; ++gi)
        if (!alloc_group(nc->groups[gi], nc->stream, s->mode, n, slots, nc->max_pts, mock)) {
          for (int gj = 0; gj < gi; ++gj) free_group(nc->groups[gj]);
          if (nc->stream) (void)hipStreamDestroy(nc->stream);
          if (nc->plan) ga_plan_destroy(nc->plan);
          return GA_ENOMEM;
        }
      nc->slots = slots;
      nc->ngroups = ngroups;
      nc->bytes = (size_t)ngroups * group_bytes(s->mode, n, slots, nc->max_pts);
      s->bytes += nc->bytes;
      c = nc.get();
      s->classes.push_back(std::move(nc));
    } else if (B->n_pts > c->max_pts) {
      // grow the record scratch: stop launching this size, wait for its groups
      const size_t grown = (size_t)c->ngroups * group_bytes(s->mode, n, c->slots, B->n_pts);
      if (s->bytes - c->bytes + grown + pair_bytes > s->budget) return GA_ENOMEM;
      c->paused = true;
      for (;;) {
        bool busy = false;
        for (int gi = 0; gi < c->ngroups; ++gi) busy |= c->groups[gi].busy;
        if (!busy) break;
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(100));
        lk.lock();
      }
      // GA_TEST_FAIL_REGROW=1 makes this reallocation report failure
      // without allocating (a host-side test of the sticky-error path)
      const char* fail = std::getenv("GA_TEST_FAIL_REGROW");
      bool ok = !(fail && fail[0] == '1');
      for (int gi = 0; gi < c->ngroups; ++gi) {
        free_group(c->groups[gi]);
        ok = ok && alloc_group(c->groups[gi], c->stream, s->mode, n, c->slots, B->n_pts, mock);
      }
      if (!ok) {
        s->sticky = GA_ENOMEM;
        c->paused = false;
        return GA_ENOMEM;
      }
      s->bytes = s->bytes - c->bytes + grown;
      c->bytes = grown;
      c->max_pts = B->n_pts;
      c->paused = false;
    }
    if (s->bytes + pair_bytes > s->budget) return GA_ENOMEM;
    s->bytes += pair_bytes;  // reserved; released below on failure
  }
  // stationary spectrum and device copies of the samples (outside the lock)
  Pair p;
  p.n = n;
  p.sigma = sigma;
  std::memcpy(p.cB, cB, sizeof(p.cB));
  p.n_pts = B->n_pts;
  p.bytes = pair_bytes;
  if (mock) {  // nothing resident: the test executor computes from the pair id
    std::lock_guard<std::mutex> lk(s->mu);
    p.id = s->next_pair++;
    s->pairs[p.id] = p;
    s->stats.pairs = (int32_t)s->pairs.size();
    *pair_id = p.id;
    return GA_OK;
  }
  float* dA = nullptr;
  float* dAw = nullptr;
  hipStream_t st = nullptr;
  bool ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess &&
            hipMalloc(&p.d_xyzr, sizeof(float) * 4 * B->n_pts) == hipSuccess &&
            hipMalloc(&p.d_w, sizeof(float) * B->n_pts) == hipSuccess &&

            hipMemcpy(p.d_xyzr, B->xyzr, sizeof(float) * 4 * B->n_pts, hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(p.d_w, B->w, sizeof(float) * B->n_pts, hipMemcpyHostToDevice) == hipSuccess;
  float* dgrid = nullptr;
  void* dwork = nullptr;
  float2* dAhat = nullptr;  // the stationary spectrum, needed only to derive the resident data
  if (ok) {
    ok = hipMalloc(&dgrid, sizeof(float) * n3) == hipSuccess && hipMalloc(&dAhat, spec_bytes) == hipSuccess;
    if (ok && A->n_pts > 0) {
      ok = hipMalloc(&dA, sizeof(float) * 4 * A->n_pts) == hipSuccess &&
           hipMalloc(&dAw, sizeof(float) * A->n_pts) == hipSuccess &&
           hipMemcpy(dA, A->xyzr, sizeof(float) * 4 * A->n_pts, hipMemcpyHostToDevice) == hipSuccess &&
           hipMemcpy(dAw, A->w, sizeof(float) * A->n_pts, hipMemcpyHostToDevice) == hipSuccess;
    }
    ok = ok && ga_splat(c->plan, dA, dAw, A->n_pts, nullptr, nullptr, sigma, 1, dgrid, st) == GA_OK &&
         ga_fft3d(c->plan, GA_R2C, dgrid, dAhat, 1, nullptr, 0, st) == GA_OK;
    if (ok && s->mode == GA_SERVE_LOCAL) {
      const size_t wb = ga_workspace_size(c->plan, GA_OP_FIELD_GRAD, 1, 0);
      ok = hipMalloc(&p.d_FA, 16 * n3) == hipSuccess && hipMalloc(&dwork, wb) == hipSuccess &&
           ga_field_grad(c->plan, dgrid, reinterpret_cast<const float*>(dAhat), p.d_FA, dwork, wb, st) == GA_OK;
    } else if (ok) {
      ok = hipMalloc(&p.d_AX, 2 * spec_bytes) == hipSuccess &&
           ga_pose_prepare(c->plan, reinterpret_cast<const float*>(dAhat), reinterpret_cast<float*>(p.d_AX), st) ==
               GA_OK;
    }
    ok = ok && hipStreamSynchronize(st) == hipSuccess;
  }
  for (void* q : {(void*)dA, (void*)dAw, (void*)dgrid, dwork, (void*)dAhat})
    if (q) (void)hipFree(q);
  if (st) (void)hipStreamDestroy(st);
  std::lock_guard<std::mutex> lk(s->mu);
  if (!ok) {
    for (void* q : {(void*)p.d_xyzr, (void*)p.d_w, (void*)p.d_AX, (void*)p.d_FA})
      if (q) (void)hipFree(q);
    s->bytes -= pair_bytes;
    return GA_EDEVICE;
  }
  p.id = s->next_pair++;
  s->pairs[p.id] = p;
  s->stats.pairs = (int32_t)s->pairs.size();
  *pair_id = p.id;
  return GA_OK;
}

ga_status ga_pair_release(ga_server* s, uint32_t pair_id) {
  if (!s) return GA_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->pairs.find(pair_id);
  if (it == s->pairs.end() || it->second.released) return GA_ENOTFOUND;
  it->second.released = true;
  if (it->second.inflight == 0) {
    s->free_pair_locked(it->second);
    s->pairs.erase(it);
  }
  s->stats.pairs = (int32_t)s->pairs.size();
  return GA_OK;
}

ga_status ga_submit(ga_server* s, uint32_t pair_id, const float R[9], const float t[3], uint64_t* ticket) {
  if (!s || !R || !t || !ticket) return GA_EINVAL;
  if (!rotation_ok(R)) return GA_EINVAL;
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(t[a]) || std::fabs(t[a]) > 1.0e9f) return GA_EINVAL;
  Pending q;
  std::memcpy(q.R, R, sizeof(q.R));
  q.pair = pair_id;
  q.t_submit = now_ns();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->sticky != GA_OK) return s->sticky;
    auto it = s->pairs.find(pair_id);
    if (it == s->pairs.end() || it->second.released) return GA_ENOTFOUND;
    if (s->queued >= s->queue_depth) {
      s->stats.rejected_full += 1;
      return GA_EAGAIN;
    }
    const int n = it->second.n;
    for (int a = 0; a < 3; ++a) {
      long long v = std::lround(t[a]) % n;  // nearest lattice point, ties away from zero
      q.t[a] = (int)(v < 0 ? v + n : v);
    }
    SizeClass* c = s->find_class(n, it->second.sigma);
    q.ticket = s->next_ticket++;
    c->queue.push_back(q);
    it->second.inflight += 1;
    s->tickets[q.ticket] = Ticket{};
    s->queued += 1;
    s->stats.submitted += 1;
    *ticket = q.ticket;
  }
  s->cv.notify_one();
  return GA_OK;
}

ga_status ga_poll(ga_server* s, uint64_t ticket, ga_result* out) {
  if (!s || !out) return GA_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return GA_ENOTFOUND;
  if (!it->second.done) return s->sticky != GA_OK ? s->sticky : GA_PENDING;
  *out = it->second.r;
  s->tickets.erase(it);
  return GA_OK;
}

ga_status ga_server_get_stats(ga_server* s, ga_server_stats* out) {
  if (!s || !out) return GA_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  out->bytes_in_use = s->bytes;
  out->pairs = (int32_t)s->pairs.size();
  return GA_OK;
}

}  // extern "C"
