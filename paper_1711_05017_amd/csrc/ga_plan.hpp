// ga_plan.hpp -- the plan object behind ga_plan*: grid edge, device, twiddle
// table, tuning choices, profiling state and the stream of the overlapped
// execution.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "ga.h"

struct ga_prof_entry {
  int kind;
  hipEvent_t start, stop;
};

struct ga_plan {
  int n;
  int max_batch;
  uint32_t flags;
  int device;
  float2* d_tw;  // exp(-2 pi i k / n), k < n, float64-accurate values rounded to float32
  // device address of the library's static scratch array on `device`
  // (ga_force_torque_noalloc), resolved when the plan is created
  void* scratch = nullptr;
  // per-kernel timing (ga_profile_*); mutable because compute calls take a const plan
  mutable bool prof = false;
  mutable std::vector<ga_prof_entry> prof_pending;
  mutable double prof_ms[GA_K_COUNT] = {};
  mutable long long prof_count[GA_K_COUNT] = {};
  // fused x pass of ga_energy_fields: strip width in transform groups (4 or
  // 8), batch members per workgroup (1, 2, 4, 8) and the XCD-aware grid
  // (1 on, 2 off); 0 = default (4, 4, off)
  int tune_groups = 0;
  int tune_k = 0;
  int tune_xcd = 0;
  // x transforms of the fused pass on the default radix schedule (0) or its
  // alternative (1, where the edge has one)
  int tune_radix = 0;
  // overlapped ga_energy_fields (ga_plan_set_overlap): the batch in `chunks`
  // parts, pass 1 on the caller's stream, the x pass and pass 3 on `aux`,
  // ordered by events ev[0 .. chunks) and joined back by ev[kMaxChunks]
  static constexpr int kMaxChunks = 4;
  int chunks = 1;
  hipStream_t aux = nullptr;
  hipEvent_t ev[kMaxChunks + 1] = {};
};
