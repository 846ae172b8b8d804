// ga_batch.hip -- heterogeneous batches of energy-field calls recorded into
// one HIP graph (see include/ga.h). Each item is captured on its own stream
// forked from a capture stream, so items of different grid edges become
// parallel branches of the graph; one graph launch replays them all.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <vector>

#include "ga.h"
#include "ga_launch.hpp"

using namespace ga_detail;

struct ga_batch {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int device = 0;
  int n_items = 0;
};

namespace {

void free_batch(ga_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  delete b;
}

}  // namespace

extern "C" {

ga_status ga_batch_create(ga_batch** out, const ga_batch_item* items, int32_t n_items) {
  if (!out) return GA_EINVAL;
  *out = nullptr;
  if (!items || n_items < 1) return GA_EINVAL;
  for (int i = 0; i < n_items; ++i) {
    const ga_batch_item& it = items[i];
    if (!valid_stream_call(it.plan) || !it.d_E || !it.d_work || it.batch < 1) return GA_EINVAL;
    if (it.work_bytes < ga_workspace_size(it.plan, GA_OP_ENERGY, it.batch, it.n_pts)) return GA_ENOMEM;
    const size_t ei = (size_t)it.batch * it.plan->n * it.plan->n * it.plan->n * sizeof(float);
    for (int j = 0; j < i; ++j) {
      const ga_batch_item& jt = items[j];
      const size_t ej = (size_t)jt.batch * jt.plan->n * jt.plan->n * jt.plan->n * sizeof(float);
      if (overlaps(it.d_E, ei, jt.d_E, ej) || overlaps(it.d_work, it.work_bytes, jt.d_work, jt.work_bytes) ||
          overlaps(it.d_E, ei, jt.d_work, jt.work_bytes) || overlaps(it.d_work, it.work_bytes, jt.d_E, ej))
        return GA_EINVAL;
    }
  }
  // An item whose plan asks for overlapped execution (ga_plan_set_overlap)
  // is recorded as that many parts of its batch on parallel branches, each
  // with its own slice of the item's workspace (when the slices fit).
  struct Part {
    const ga_batch_item* it;
    int c0, nb;
    char* work;
    size_t work_bytes;
  };
  std::vector<Part> parts;
  for (int i = 0; i < n_items; ++i) {
    const ga_batch_item& it = items[i];
    const int k = it.plan->tune_k ? it.plan->tune_k : 4;
    const int chunks = std::min(it.plan->chunks, (int)it.batch);
    const int per = ((it.batch + chunks - 1) / chunks + k - 1) / k * k;
    auto slice = [&](int nb) {  // 256-byte aligned slices
      return (ga_workspace_size(it.plan, GA_OP_ENERGY, nb, it.n_pts) + 255) / 256 * 256;
    };
    size_t need = 0;
    for (int c0 = 0; c0 < it.batch; c0 += per) need += slice(std::min(per, it.batch - c0));
    if (chunks <= 1 || need > it.work_bytes || axis_mode(it.plan)) {
      parts.push_back({&it, 0, it.batch, static_cast<char*>(it.d_work), it.work_bytes});
      continue;
    }
    char* w = static_cast<char*>(it.d_work);
    for (int c0 = 0; c0 < it.batch; c0 += per) {
      const int nb = std::min(per, it.batch - c0);
      const size_t wb = slice(nb);
      parts.push_back({&it, c0, nb, w, wb});
      w += wb;
    }
  }
  const int n_parts = (int)parts.size();
  ga_batch* b = new (std::nothrow) ga_batch{};
  if (!b) return GA_ENOMEM;
  b->n_items = n_items;
  (void)hipGetDevice(&b->device);
  hipStream_t cap = nullptr;
  hipEvent_t fork = nullptr;
  std::vector<hipStream_t> br(n_parts, nullptr);
  std::vector<hipEvent_t> joins(n_parts, nullptr);
  bool ok = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&fork, hipEventDisableTiming) == hipSuccess;
  for (int i = 0; ok && i < n_parts; ++i)
    ok = hipStreamCreateWithFlags(&br[i], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&joins[i], hipEventDisableTiming) == hipSuccess;
  ga_status st = GA_OK;
  bool capturing = false;
  if (ok) {
    ok = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
    capturing = ok;
  }
  ok = ok && hipEventRecord(fork, cap) == hipSuccess;
  for (int i = 0; ok && i < n_parts; ++i) {
    const Part& pt = parts[i];
    const ga_batch_item& it = *pt.it;
    const size_t n3 = (size_t)it.plan->n * it.plan->n * it.plan->n;
    ok = hipStreamWaitEvent(br[i], fork, 0) == hipSuccess;
    if (!ok) break;
    st = ga_energy_fields(it.plan, it.d_Ahat, it.d_xyzr, it.d_w, it.n_pts, it.d_R + (size_t)9 * pt.c0, it.c, it.sigma,
                          pt.nb, it.d_E + (size_t)pt.c0 * n3, pt.work, pt.work_bytes, br[i]);
    ok = (st == GA_OK) && hipEventRecord(joins[i], br[i]) == hipSuccess &&
         hipStreamWaitEvent(cap, joins[i], 0) == hipSuccess;
  }
  if (capturing) {
    hipGraph_t g = nullptr;
    const bool ended = hipStreamEndCapture(cap, &g) == hipSuccess;
    if (ended) b->graph = g;
    ok = ok && ended && g != nullptr;
  }
  ok = ok && hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) == hipSuccess;
  for (int i = 0; i < n_parts; ++i) {
    if (joins[i]) (void)hipEventDestroy(joins[i]);
    if (br[i]) (void)hipStreamDestroy(br[i]);
  }
  if (fork) (void)hipEventDestroy(fork);
  if (cap) (void)hipStreamDestroy(cap);
  if (!ok) {
    free_batch(b);
    (void)hipGetLastError();
    return (st != GA_OK) ? st : GA_EDEVICE;
  }
  *out = b;
  return GA_OK;
}

ga_status ga_batch_launch(const ga_batch* b, hipStream_t stream) {
  if (!b || !b->exec) return GA_EINVAL;
  return hipGraphLaunch(b->exec, stream) == hipSuccess ? GA_OK : GA_EDEVICE;
}

ga_status ga_batch_destroy(ga_batch* b) {
  if (!b) return GA_EINVAL;
  free_batch(b);
  return GA_OK;
}

}  // extern "C"
