// ga_lib.hip -- C ABI of libga.so: plans, argument checks and kernel launches.
// The operations, layouts and error behaviour are documented in include/ga.h.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <mutex>
#include <new>
#include <vector>

#include "ga.h"
#include "ga_launch.hpp"
#include "ga_rotate.hpp"
#include "ga_tune_cache.hpp"

using namespace ga;
using namespace ga_detail;

// Scratch of ga_force_torque_noalloc: one array per device, in the code
// object's static device memory (no allocation at call time). Its name is a
// host-side stand-in; kernels get the device address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) double scratch[GA_NOALLOC_SCRATCH_BYTES / sizeof(double)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on `dev`, which must be the current device;
// resolved once per device and kept for the life of the process.
ga_status scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return GA_EDEVICE;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return GA_EDEVICE;
    g_scratch_addr[dev] = ptr;
  }
  *out = g_scratch_addr[dev];
  return GA_OK;
}

// GA_SINGLE readout: per-strip partial sums into `part`, then their sum per pose.
void launch_single(const ga_plan* plan, const float2* A, const float2* B4, const float* d_t, int n_poses,
                   double* part, float* d_out7, hipStream_t stream) {
  const int n = plan->n;
  ProfScope ps(plan, GA_K_READOUT, stream);
  dispatch_axis(n, [&]<int N>() { Launch<N>::single(A, B4, d_t, n_poses, part, plan->d_tw, stream); });
  const double scale = 1.0 / ((double)n * n * n);
  hipLaunchKernelGGL(k_reduce_partials, dim3(n_poses), dim3(64), 0, stream, (const double*)part, nsingle_of(n), d_out7,
                     scale, (const QueryItem*)nullptr);
}

// Whether edge n has an alternative radix schedule for the fused x pass.
bool has_alt_radix(int n) {
  bool alt = false;
  if (n <= 192 && n >= 16) dispatch_axis(n, [&]<int N>() { alt = Launch<N>::kAltRadix; });
  return alt;
}

// Launch of the rotation kernels for a source (PlanarSrc or PackedSrc).
template <template <int> class SrcT, class MakeSrc>
void launch_rotate(int n, MakeSrc make_src, const float* d_R, int32_t batch, float* d_out, hipStream_t stream) {
  dispatch_axis(n, [&]<int N>() {
    const dim3 block(256);
    const auto out = reinterpret_cast<float2*>(d_out);
    const unsigned nb = (unsigned)std::min(batch, 65535);
    const SrcT<N> src = make_src.template operator()<N>();
    if constexpr ((N / 2) % 8 == 0) {
      constexpr int tiles = (N / 8) * (N / 8) * ((N / 2 + 1 + 7) / 8);  // 8 x 8 x 8 outputs per workgroup
      hipLaunchKernelGGL((k_spectral_rotate<N, SrcT<N>>), dim3(tiles, nb), dim3(SrcT<N>::THREADS), 0, stream, src, d_R,
                         (int)batch, out);
    } else {
      constexpr int tiles = (N / 2) * (N / 8) * ((N / 2 + 1 + 15) / 16);  // 2 x 8 x 16 outputs per workgroup
      hipLaunchKernelGGL((k_spectral_rotate_gather<N, SrcT<N>>), dim3(tiles, nb), block, 0, stream, src, d_R,
                         (int)batch, out);
    }
  });
}

}  // namespace

extern "C" {

const char* ga_status_str(ga_status s) {
  switch (s) {
    case GA_OK: return "ok";
    case GA_PENDING: return "pending";
    case GA_EINVAL: return "invalid argument";
    case GA_ENOMEM: return "out of memory, workspace too small or budget exceeded";
    case GA_EAGAIN: return "queue full";
    case GA_EDEVICE: return "device (HIP) error";
    case GA_ENOTFOUND: return "not found";
    case GA_EUNSUPPORTED: return "grid edge not supported";
    default: return "unknown status";
  }
}

const char* ga_version(void) { return kVersion; }

int32_t ga_supported_n(int32_t n) {
  return dispatch_axis(n, []<int N>() {}) ? 1 : 0;
}

ga_status ga_plan_create(ga_plan** plan, int32_t n, int32_t max_batch, uint32_t flags) {
  if (!plan) return GA_EINVAL;
  *plan = nullptr;
  if (n < 8 || (n & 1) || max_batch < 1 || (flags & ~GA_PLAN_AXIS_PASSES) != 0) return GA_EINVAL;
  if (!ga_supported_n(n)) return GA_EUNSUPPORTED;
  ga_plan* p = new (std::nothrow) ga_plan{};
  if (!p) return GA_ENOMEM;
  p->n = n;
  p->max_batch = max_batch;
  p->flags = flags;
  if (hipGetDevice(&p->device) != hipSuccess || scratch_address(p->device, &p->scratch) != GA_OK) {
    delete p;
    return GA_EDEVICE;
  }
  std::vector<float2> tw(n);
  const double two_pi = 6.283185307179586476925286766559;
  for (int k = 0; k < n; ++k) {
    const double a = two_pi * (double)k / (double)n;
    tw[k] = make_float2((float)std::cos(a), (float)(-std::sin(a)));
  }
  if (hipMalloc(&p->d_tw, sizeof(float2) * n) != hipSuccess) {
    delete p;
    return GA_ENOMEM;
  }
  if (hipMemcpy(p->d_tw, tw.data(), sizeof(float2) * n, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(p->d_tw);
    delete p;
    return GA_EDEVICE;
  }
  *plan = p;
  return GA_OK;
}

ga_status ga_plan_destroy(ga_plan* plan) {
  if (!plan) return GA_EINVAL;
  prof_drain(plan);
  if (plan->aux) {
    (void)hipStreamSynchronize(plan->aux);
    for (hipEvent_t e : plan->ev)
      if (e) (void)hipEventDestroy(e);
    (void)hipStreamDestroy(plan->aux);
  }
  if (plan->d_tw) (void)hipFree(plan->d_tw);
  delete plan;
  return GA_OK;
}

ga_status ga_plan_set_overlap(ga_plan* plan, int32_t chunks) {
  if (!valid_stream_call(plan) || (chunks != 1 && chunks != 2 && chunks != ga_plan::kMaxChunks)) return GA_EINVAL;
  if (chunks > 1 && !plan->aux) {
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess || hipSetDevice(plan->device) != hipSuccess) return GA_EDEVICE;
    bool ok = hipStreamCreateWithFlags(&plan->aux, hipStreamNonBlocking) == hipSuccess;
    for (hipEvent_t& e : plan->ev) ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
    (void)hipSetDevice(cur);
    if (!ok) {
      for (hipEvent_t& e : plan->ev)
        if (e) (void)hipEventDestroy(e), e = nullptr;
      if (plan->aux) (void)hipStreamDestroy(plan->aux), plan->aux = nullptr;
      return GA_EDEVICE;
    }
  }
  plan->chunks = chunks;
  return GA_OK;
}

int32_t ga_plan_get_overlap(const ga_plan* plan) { return plan ? plan->chunks : 0; }

int32_t ga_plan_n(const ga_plan* plan) { return plan ? plan->n : 0; }

size_t ga_workspace_size(const ga_plan* plan, int32_t op, int32_t batch, int64_t n_items) {
  if (!plan || batch < 0 || n_items < 0) return 0;
  const int n = plan->n;
  const size_t spec = spectrum_elems(n) * sizeof(float2);
  const size_t real = (size_t)n * n * n * sizeof(float);
  switch (op) {
    case GA_OP_FFT_C2R:
    case GA_OP_CORRELATE: return (size_t)batch * spec;
    case GA_OP_ENERGY:
      if (axis_mode(plan)) return (size_t)batch * (spec + real);
      return bin_offset(n, batch) + bin_bytes(n, batch, n_items);
    case GA_OP_FORCE_FIELDS: return 7 * spec + 7 * real;
    case GA_OP_FORCE_SINGLE: return (size_t)n_items * nsingle_of(n) * 7 * sizeof(double);
    case GA_OP_FIELD_GRAD: return 6 * spec + 3 * real;
    case GA_OP_SCORE: return (n_items >= 1 && n_items <= 2) ? (size_t)batch * (size_t)n_items * spec : 0;
    case GA_OP_POSE_LOCAL:
      return (size_t)batch * sizeof(QueryItem) + (size_t)batch * nlocal_of(n_items) * 7 * sizeof(double);
    case GA_OP_POSE_SPECTRAL:
      if (!plane_edge(n)) return 0;
      return pose_spectral_layout(n, batch, n_items).total;
    default: return 0;
  }
}

ga_status ga_splat(const ga_plan* plan, const float* d_xyzr, const float* d_w, int64_t n_pts, const float* h_R,
                   const float* h_c, float sigma, int32_t channels, float* d_grid, hipStream_t stream) {
  if (!valid_stream_call(plan) || !d_grid || n_pts < 0 || (n_pts > 0 && (!d_xyzr || !d_w))) return GA_EINVAL;
  if (!all_aligned(d_xyzr, d_grid)) return GA_EINVAL;
  if ((channels != 1 && channels != 4) || !valid_sigma(sigma)) return GA_EINVAL;
  if ((h_R == nullptr) != (h_c == nullptr)) return GA_EINVAL;
  if (h_R && !rotation_ok(h_R)) return GA_EINVAL;
  if (h_c && !(std::isfinite(h_c[0]) && std::isfinite(h_c[1]) && std::isfinite(h_c[2]))) return GA_EINVAL;
  const int n = plan->n;
  const size_t n3 = (size_t)n * n * n;
  SplatParams sp = make_splat(d_xyzr, d_w, n_pts, nullptr, h_R, h_c, sigma);
  if (axis_mode(plan)) {
    ProfScope ps(plan, GA_K_SPLAT, stream);
    dispatch_axis(n, [&]<int N>() { Axis<N>::splat(sp, channels, d_grid, 1, stream); });
    return launch_status();
  }
  if (n_pts == 0) {
    // a fill kernel rather than a memset node, so the call can be captured
    const long long n4 = (long long)(n3 * channels / 4);
    hipLaunchKernelGGL(k_zero4, dim3((unsigned)std::min<long long>((n4 + 255) / 256, 65535)), dim3(256), 0, stream,
                       reinterpret_cast<float4*>(d_grid), n4);
    return launch_status();
  }
  dispatch(n, [&]<int N>() {
    ProfScope ps(plan, GA_K_SPLAT, stream);
    hipLaunchKernelGGL(k_splat_real<N>, dim3(N), dim3(Plane<N>::THREADS), 0, stream, sp, channels, d_grid);
  });
  return launch_status();
}

ga_status ga_fft3d(const ga_plan* plan, int32_t dir, const void* d_in, void* d_out, int32_t batch, void* d_work,
                   size_t work_bytes, hipStream_t stream) {
  if (!valid_stream_call(plan) || !d_in || !d_out || batch < 1 || batch > plan->max_batch) return GA_EINVAL;
  if (!all_aligned(d_in, d_out, d_work)) return GA_EINVAL;
  if (dir != GA_R2C && dir != GA_C2R) return GA_EINVAL;
  const int n = plan->n;
  const size_t real_b = (size_t)batch * n * n * n * sizeof(float);
  const size_t spec_b = (size_t)batch * spectrum_elems(n) * sizeof(float2);
  if (overlaps(d_in, dir == GA_R2C ? real_b : spec_b, d_out, dir == GA_R2C ? spec_b : real_b)) return GA_EINVAL;
  if (dir == GA_C2R && (overlaps(d_work, work_bytes, d_in, spec_b) || overlaps(d_work, work_bytes, d_out, real_b)))
    return GA_EINVAL;
  if (axis_mode(plan)) {
    if (dir == GA_R2C) {
      float2* out = static_cast<float2*>(d_out);
      dispatch_axis(n, [&]<int N>() {
        {
          ProfScope ps(plan, GA_K_PLANE_FWD, stream);
          Axis<N>::zy_fwd(static_cast<const float*>(d_in), out, batch, plan->d_tw, stream);
        }
        ProfScope ps(plan, GA_K_STRIP, stream);
        Launch<N>::strip_fft(-1, out, out, batch, plan->d_tw, stream);
      });
    } else {
      if (!d_work || work_bytes < ga_workspace_size(plan, GA_OP_FFT_C2R, batch, 0)) return GA_ENOMEM;
      float2* tmp = static_cast<float2*>(d_work);
      const float scale = (float)(1.0 / ((double)n * n * n));
      dispatch_axis(n, [&]<int N>() {
        {
          ProfScope ps(plan, GA_K_STRIP, stream);
          Launch<N>::strip_fft(+1, static_cast<const float2*>(d_in), tmp, batch, plan->d_tw, stream);
        }
        ProfScope ps(plan, GA_K_PLANE_INV, stream);
        Axis<N>::yz_inv(tmp, static_cast<float*>(d_out), scale, batch, plan->d_tw, stream);
      });
    }
    return launch_status();
  }
  if (dir == GA_R2C) {
    float2* out = static_cast<float2*>(d_out);
    SplatParams sp = make_splat(nullptr, nullptr, 0, nullptr, nullptr, nullptr, 0.5f);
    dispatch(n, [&]<int N>() {
      {
        ProfScope ps(plan, GA_K_PLANE_FWD, stream);
        Launch<N>::plane_fwd(sp, static_cast<const float*>(d_in), out, batch, plan->d_tw, stream);
      }
      ProfScope ps(plan, GA_K_STRIP, stream);
      Launch<N>::strip_fft(-1, out, out, batch, plan->d_tw, stream);
    });
  } else {
    if (!d_work || work_bytes < ga_workspace_size(plan, GA_OP_FFT_C2R, batch, 0)) return GA_ENOMEM;
    float2* tmp = static_cast<float2*>(d_work);
    const float scale = (float)(1.0 / ((double)n * n * n));
    dispatch(n, [&]<int N>() {
      {
        ProfScope ps(plan, GA_K_STRIP, stream);
        Launch<N>::strip_fft(+1, static_cast<const float2*>(d_in), tmp, batch, plan->d_tw, stream);
      }
      ProfScope ps(plan, GA_K_PLANE_INV, stream);
      Launch<N>::plane_inv(tmp, static_cast<float*>(d_out), scale, batch, plan->d_tw, stream);
    });
  }
  return launch_status();
}

ga_status ga_correlate(const ga_plan* plan, const float* d_Ahat, int64_t a_stride, const float* d_Bhat,
                       int32_t batch, float* d_E, void* d_work, size_t work_bytes, hipStream_t stream) {
  if (!valid_stream_call(plan) || !d_Ahat || !d_Bhat || !d_E || batch < 1 || batch > plan->max_batch ||
      a_stride < 0)
    return GA_EINVAL;
  if (!all_aligned(d_Ahat, d_Bhat, d_E, d_work)) return GA_EINVAL;
  if (!d_work || work_bytes < ga_workspace_size(plan, GA_OP_CORRELATE, batch, 0)) return GA_ENOMEM;
  const int n = plan->n;
  {
    const size_t spec_b = (size_t)batch * spectrum_elems(n) * sizeof(float2);
    const size_t a_b = (size_t)((batch - 1) * a_stride + (int64_t)spectrum_elems(n)) * sizeof(float2);
    const size_t real_b = (size_t)batch * n * n * n * sizeof(float);
    if (overlaps(d_E, real_b, d_Bhat, spec_b) || overlaps(d_E, real_b, d_Ahat, a_b) ||
        overlaps(d_work, work_bytes, d_E, real_b) || overlaps(d_work, work_bytes, d_Bhat, spec_b) ||
        overlaps(d_work, work_bytes, d_Ahat, a_b))
      return GA_EINVAL;
  }
  float2* tmp = static_cast<float2*>(d_work);
  const float scale = (float)(1.0 / ((double)n * n * n));
  if (axis_mode(plan)) {
    dispatch_axis(n, [&]<int N>() {
      {
        ProfScope ps(plan, GA_K_STRIP, stream);
        Launch<N>::strip_corr(false, reinterpret_cast<const float2*>(d_Ahat), a_stride,
                              reinterpret_cast<const float2*>(d_Bhat), tmp, batch, plan->d_tw, stream);
      }
      ProfScope ps(plan, GA_K_PLANE_INV, stream);
      Axis<N>::yz_inv(tmp, d_E, scale, batch, plan->d_tw, stream);
    });
    return launch_status();
  }
  dispatch(n, [&]<int N>() {
    {
      ProfScope ps(plan, GA_K_STRIP, stream);
      Launch<N>::strip_corr(false, reinterpret_cast<const float2*>(d_Ahat), a_stride,
                            reinterpret_cast<const float2*>(d_Bhat), tmp, batch, plan->d_tw, stream);
    }
    ProfScope ps(plan, GA_K_PLANE_INV, stream);
    Launch<N>::plane_inv(tmp, d_E, scale, batch, plan->d_tw, stream);
  });
  return launch_status();
}

ga_status ga_score(const ga_plan* plan, const float* d_A2, int64_t a_stride, const float* d_B2, int32_t batch,
                   uint32_t parts, float* d_out, void* d_work, size_t work_bytes, hipStream_t stream) {
  if (!valid_stream_call(plan) || !d_A2 || !d_B2 || !d_out || batch < 1 || batch > plan->max_batch || a_stride < 0 ||
      parts < 1 || parts > (GA_SCORE_RE | GA_SCORE_IM))
    return GA_EINVAL;
  if (!all_aligned(d_A2, d_B2, d_out, d_work)) return GA_EINVAL;
  const int nparts = (parts == (GA_SCORE_RE | GA_SCORE_IM)) ? 2 : 1;
  const int first = (parts == GA_SCORE_IM) ? 1 : 0;
  if (!d_work || work_bytes < ga_workspace_size(plan, GA_OP_SCORE, batch, nparts)) return GA_ENOMEM;
  const int n = plan->n;
  const size_t spec_e = spectrum_elems(n);
  {
    const size_t b_b = (size_t)batch * 2 * spec_e * sizeof(float2);
    const size_t a_b = (size_t)((batch - 1) * a_stride + 2 * (int64_t)spec_e) * sizeof(float2);
    const size_t out_b = (size_t)batch * nparts * n * n * n * sizeof(float);
    if (overlaps(d_out, out_b, d_B2, b_b) || overlaps(d_out, out_b, d_A2, a_b) ||
        overlaps(d_work, work_bytes, d_out, out_b) || overlaps(d_work, work_bytes, d_B2, b_b) ||
        overlaps(d_work, work_bytes, d_A2, a_b))
      return GA_EINVAL;
  }
  float2* tmp = static_cast<float2*>(d_work);
  const float2* A2 = reinterpret_cast<const float2*>(d_A2);
  const float2* B2 = reinterpret_cast<const float2*>(d_B2);
  const float scale = (float)(1.0 / ((double)n * n * n));
  if (axis_mode(plan)) {
    dispatch_axis(n, [&]<int N>() {
      {
        ProfScope ps(plan, GA_K_STRIP, stream);
        Launch<N>::strip_score(A2, a_stride, B2, tmp, batch, first, nparts, plan->d_tw, stream);
      }
      ProfScope ps(plan, GA_K_PLANE_INV, stream);
      Axis<N>::yz_inv(tmp, d_out, scale, batch * nparts, plan->d_tw, stream);
    });
    return launch_status();
  }
  dispatch(n, [&]<int N>() {
    {
      ProfScope ps(plan, GA_K_STRIP, stream);
      Launch<N>::strip_score(A2, a_stride, B2, tmp, batch, first, nparts, plan->d_tw, stream);
    }
    ProfScope ps(plan, GA_K_PLANE_INV, stream);
    Launch<N>::plane_inv(tmp, d_out, scale, batch * nparts, plan->d_tw, stream);
  });
  return launch_status();
}

ga_status ga_energy_fields(const ga_plan* plan, const float* d_Ahat, const float* d_xyzr, const float* d_w,
                           int64_t n_pts, const float* d_R, const float* h_c, float sigma, int32_t batch,
                           float* d_E, void* d_work, size_t work_bytes, hipStream_t stream) {
  if (!valid_stream_call(plan) || !d_Ahat || !d_R || !h_c || !d_E || batch < 1 || batch > plan->max_batch ||
      n_pts < 0 || (n_pts > 0 && (!d_xyzr || !d_w)) || !valid_sigma(sigma))
    return GA_EINVAL;
  if (!all_aligned(d_Ahat, d_xyzr, d_E, d_work)) return GA_EINVAL;
  if (!(std::isfinite(h_c[0]) && std::isfinite(h_c[1]) && std::isfinite(h_c[2]))) return GA_EINVAL;
  if (!d_work || work_bytes < ga_workspace_size(plan, GA_OP_ENERGY, batch, n_pts)) return GA_ENOMEM;
  const int n = plan->n;
  {
    const size_t real_b = (size_t)batch * n * n * n * sizeof(float);
    const size_t spec_b = spectrum_elems(n) * sizeof(float2);
    if (overlaps(d_work, work_bytes, d_E, real_b) || overlaps(d_work, work_bytes, d_Ahat, spec_b) ||
        overlaps(d_E, real_b, d_Ahat, spec_b))
      return GA_EINVAL;
  }
  float2* tmp = static_cast<float2*>(d_work);
  const float scale = (float)(1.0 / ((double)n * n * n));
  SplatParams sp = make_splat(d_xyzr, d_w, n_pts, d_R, nullptr, h_c, sigma);
  const int groups = plan->tune_groups ? plan->tune_groups : 4;
  if (axis_mode(plan)) {
    float* real = reinterpret_cast<float*>(static_cast<char*>(d_work) + (size_t)batch * spectrum_elems(n) * sizeof(float2));
    dispatch_axis(n, [&]<int N>() {
      const int k = plan->tune_k ? plan->tune_k : Launch<N>::kCorrK;
      {
        ProfScope ps(plan, GA_K_SPLAT, stream);
        Axis<N>::splat(sp, 1, real, batch, stream);
      }
      {
        ProfScope ps(plan, GA_K_PLANE_FWD, stream);
        Axis<N>::zy_fwd(real, tmp, batch, plan->d_tw, stream);
      }
      {
        ProfScope ps(plan, GA_K_STRIP, stream);
        Launch<N>::corr_fwd_tuned(groups, k, plan->tune_xcd == 1, plan->tune_radix,
                                  reinterpret_cast<const float2*>(d_Ahat), 0, tmp, batch, plan->d_tw, stream);
      }
      ProfScope ps(plan, GA_K_PLANE_INV, stream);
      Axis<N>::yz_inv(tmp, d_E, scale, batch, plan->d_tw, stream);
    });
    return launch_status();
  }
  char* bins = static_cast<char*>(d_work) + bin_offset(n, batch);
  const BinLayout bl(n, batch, n_pts);
  Placed* rec = reinterpret_cast<Placed*>(bins + bl.rec);
  int* off = reinterpret_cast<int*>(bins + bl.off);
  float* rmax = reinterpret_cast<float*>(bins + bl.rmax);
  int4* cand = reinterpret_cast<int4*>(bins + bl.cand);
  unsigned* pmask = reinterpret_cast<unsigned*>(bins + bl.pmask);
  // chunked, two-stream execution (ga_plan_set_overlap); one stream under
  // graph capture
  int chunks = std::min(plan->chunks, (int)batch);
  if (chunks > 1) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (!plan->aux || hipStreamIsCapturing(stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) chunks = 1;
  }
  if (chunks > 1) {  // the second stream starts after the caller's earlier work
    (void)hipEventRecord(plan->ev[0], stream);
    (void)hipStreamWaitEvent(plan->aux, plan->ev[0], 0);
  }
  dispatch(n, [&]<int N>() {
    const int k = plan->tune_k ? plan->tune_k : Launch<N>::kCorrK;
    // parts of whole workgroups of the x pass (k members each), whole
    // pipelines alternating between the caller's stream and the second one
    const int per = ((batch + chunks - 1) / chunks + k - 1) / k * k;
    int ci = 0;
    for (int c0 = 0; c0 < batch; c0 += per, ++ci) {
      const int nb = std::min(per, batch - c0);
      hipStream_t sc = (ci & 1) ? plan->aux : stream;
      SplatParams spc = sp;
      spc.Rdev = sp.Rdev + (size_t)9 * c0;
      Placed* rc = rec + (size_t)c0 * (size_t)n_pts;
      int* oc = off + (size_t)c0 * (N + 1);
      float* mc = rmax + c0;
      int4* cc = cand + (size_t)c0 * N;
      float2* tc = tmp + (size_t)c0 * spectrum_elems(n);
      unsigned* pc = pmask + (size_t)c0 * kPlaneMaskWords<N>;
      spc.pmask = pc;  // cleared by the binning, set by pass 1, read by the x pass
      {
        ProfScope pb(plan, GA_K_BIN, sc);
        Launch<N>::bin_samples(spc, rc, oc, mc, cc, nb, sc);
      }
      spc.rec = rc;
      spc.off = oc;
      spc.rmax = mc;
      spc.cand = cc;
      {
        ProfScope ps(plan, GA_K_PLANE_FWD, sc);
        Launch<N>::plane_fwd(spc, nullptr, tc, nb, plan->d_tw, sc);
      }
      {
        ProfScope ps(plan, GA_K_STRIP, sc);
        Launch<N>::corr_fwd_tuned(groups, k, plan->tune_xcd == 1, plan->tune_radix,
                                  reinterpret_cast<const float2*>(d_Ahat), 0, tc, nb, plan->d_tw, sc, pc);
      }
      ProfScope ps(plan, GA_K_PLANE_INV, sc);
      Launch<N>::plane_inv(tc, d_E + (size_t)c0 * n * n * n, scale, nb, plan->d_tw, sc);
    }
    if (chunks > 1) {
      (void)hipEventRecord(plan->ev[ga_plan::kMaxChunks], plan->aux);
      (void)hipStreamWaitEvent(stream, plan->ev[ga_plan::kMaxChunks], 0);
    }
  });
  return launch_status();
}

ga_status ga_force_torque(const ga_plan* plan, const float* d_Ahat, const float* d_Bhat4, const float* d_t,
                          int32_t n_poses, uint32_t mode, float* d_out7, void* d_work, size_t work_bytes,
                          hipStream_t stream) {
  if (!valid_stream_call(plan) || !d_Ahat || !d_Bhat4 || n_poses < 0 || (n_poses > 0 && (!d_t || !d_out7)))
    return GA_EINVAL;
  if (!all_aligned(d_Ahat, d_Bhat4, d_work)) return GA_EINVAL;
  if (mode != GA_FIELDS && mode != GA_SINGLE) return GA_EINVAL;
  if (n_poses == 0) return GA_OK;
  const int n = plan->n;
  const int op = (mode == GA_FIELDS) ? GA_OP_FORCE_FIELDS : GA_OP_FORCE_SINGLE;
  if (!d_work || work_bytes < ga_workspace_size(plan, op, 1, (int64_t)n_poses)) return GA_ENOMEM;
  {
    const size_t spec_b = spectrum_elems(n) * sizeof(float2);
    if (overlaps(d_work, work_bytes, d_Ahat, spec_b) || overlaps(d_work, work_bytes, d_Bhat4, 4 * spec_b) ||
        overlaps(d_work, work_bytes, d_out7, sizeof(float) * 7 * (size_t)n_poses))
      return GA_EINVAL;
  }
  const float2* A = reinterpret_cast<const float2*>(d_Ahat);
  const float2* B4 = reinterpret_cast<const float2*>(d_Bhat4);
  if (mode == GA_FIELDS) {
    float2* spec7 = static_cast<float2*>(d_work);
    float* fields7 = reinterpret_cast<float*>(spec7 + 7 * spectrum_elems(n));
    const float scale = (float)(1.0 / ((double)n * n * n));
    const bool ax = axis_mode(plan);
    dispatch_axis(n, [&]<int N>() {
      {
        ProfScope ps(plan, GA_K_READOUT, stream);
        Launch<N>::ft_fields(A, B4, spec7, plan->d_tw, stream);
      }
      ProfScope ps(plan, GA_K_PLANE_INV, stream);
      if (ax) Axis<N>::yz_inv(spec7, fields7, scale, 7, plan->d_tw, stream);
    });
    if (!ax) {
      dispatch(n, [&]<int N>() {
        ProfScope ps(plan, GA_K_PLANE_INV, stream);
        Launch<N>::plane_inv(spec7, fields7, scale, 7, plan->d_tw, stream);
      });
    }
    ProfScope ps(plan, GA_K_READOUT, stream);
    const int threads = 256, total = n_poses * 7;
    hipLaunchKernelGGL(k_gather7, dim3((total + threads - 1) / threads), dim3(threads), 0, stream, fields7, n, d_t,
                       n_poses, d_out7);
  } else {
    launch_single(plan, A, B4, d_t, n_poses, static_cast<double*>(d_work), d_out7, stream);
  }
  return launch_status();
}

ga_status ga_force_torque_noalloc(const ga_plan* plan, const float* d_Ahat, const float* d_Bhat4, const float* d_t,
                                  int32_t n_poses, float* d_out7, hipStream_t stream) {
  if (!valid_stream_call(plan) || !plan->scratch || !d_Ahat || !d_Bhat4 || n_poses < 0 ||
      (n_poses > 0 && (!d_t || !d_out7)))
    return GA_EINVAL;
  if (!all_aligned(d_Ahat, d_Bhat4)) return GA_EINVAL;
  if (n_poses == 0) return GA_OK;
  const size_t need = ga_workspace_size(plan, GA_OP_FORCE_SINGLE, 1, (int64_t)n_poses);
  if (need == 0 || need > GA_NOALLOC_SCRATCH_BYTES) return GA_ENOMEM;
  const size_t spec_b = spectrum_elems(plan->n) * sizeof(float2);
  if (overlaps(d_out7, sizeof(float) * 7 * (size_t)n_poses, d_Ahat, spec_b) ||
      overlaps(d_out7, sizeof(float) * 7 * (size_t)n_poses, d_Bhat4, 4 * spec_b))
    return GA_EINVAL;
  launch_single(plan, reinterpret_cast<const float2*>(d_Ahat), reinterpret_cast<const float2*>(d_Bhat4), d_t,
                n_poses, static_cast<double*>(plan->scratch), d_out7, stream);
  return launch_status();
}

ga_status ga_field_grad(const ga_plan* plan, const float* d_uA, const float* d_Ahat, float* d_FA4, void* d_work,
                        size_t work_bytes, hipStream_t stream) {
  if (!valid_stream_call(plan) || !d_uA || !d_Ahat || !d_FA4) return GA_EINVAL;
  if (!all_aligned(d_uA, d_Ahat, d_FA4, d_work)) return GA_EINVAL;
  if (!d_work || work_bytes < ga_workspace_size(plan, GA_OP_FIELD_GRAD, 1, 0)) return GA_ENOMEM;
  const int n = plan->n;
  const size_t spec = spectrum_elems(n);
  const size_t n3 = (size_t)n * n * n;
  if (overlaps(d_work, work_bytes, d_FA4, 16 * n3) || overlaps(d_work, work_bytes, d_uA, 4 * n3) ||
      overlaps(d_work, work_bytes, d_Ahat, 8 * spec) || overlaps(d_FA4, 16 * n3, d_uA, 4 * n3) ||
      overlaps(d_FA4, 16 * n3, d_Ahat, 8 * spec))
    return GA_EINVAL;
  float2* g3 = static_cast<float2*>(d_work);
  float2* tmp = g3 + 3 * spec;
  float* real3 = reinterpret_cast<float*>(tmp + 3 * spec);
  const float scale = (float)(1.0 / ((double)n * n * n));
  const bool ax = axis_mode(plan);
  dispatch_axis(n, [&]<int N>() {
    ProfScope ps(plan, GA_K_READOUT, stream);
    const int threads = 256;
    hipLaunchKernelGGL(k_grad_spectra<N>, dim3((unsigned)((spec + threads - 1) / threads)), dim3(threads), 0, stream,
                       reinterpret_cast<const float2*>(d_Ahat), g3);
    Launch<N>::strip_fft(+1, g3, tmp, 3, plan->d_tw, stream);
    if constexpr (plane_fits<N>()) {
      if (!ax) Launch<N>::plane_inv(tmp, real3, scale, 3, plan->d_tw, stream);
      else Axis<N>::yz_inv(tmp, real3, scale, 3, plan->d_tw, stream);
    } else {
      Axis<N>::yz_inv(tmp, real3, scale, 3, plan->d_tw, stream);
    }
    hipLaunchKernelGGL(k_pack4, dim3((unsigned)((n3 + threads - 1) / threads)), dim3(threads), 0, stream, d_uA,
                       (const float*)real3, reinterpret_cast<float4*>(d_FA4), (long long)n3);
  });
  return launch_status();
}

ga_status ga_pose_local(const ga_plan* plan, const float* d_FA4, const float* d_xyzr, const float* d_w, int64_t n_pts,
                        const float* d_R, const float* h_c, float sigma, const float* d_t, int32_t n_poses,
                        float* d_out7, void* d_work, size_t work_bytes, hipStream_t stream) {
  if (!valid_stream_call(plan) || !d_FA4 || n_pts < 0 || (n_pts > 0 && (!d_xyzr || !d_w)) || !h_c ||
      !valid_sigma(sigma) || n_poses < 0 || (n_poses > 0 && (!d_R || !d_t || !d_out7)))
    return GA_EINVAL;
  if (!all_aligned(d_FA4, d_xyzr, d_work)) return GA_EINVAL;
  if (!(std::isfinite(h_c[0]) && std::isfinite(h_c[1]) && std::isfinite(h_c[2]))) return GA_EINVAL;
  if (n_poses == 0) return GA_OK;
  if (!d_work || work_bytes < ga_workspace_size(plan, GA_OP_POSE_LOCAL, n_poses, n_pts)) return GA_ENOMEM;
  if (overlaps(d_work, work_bytes, d_out7, sizeof(float) * 7 * (size_t)n_poses)) return GA_EINVAL;
  const int n = plan->n;
  if (n > 256) return GA_EUNSUPPORTED;
  QueryItem* items = static_cast<QueryItem*>(d_work);
  double* part = reinterpret_cast<double*>(items + n_poses);
  const int nblk = nlocal_of(n_pts);
  SplatParams sp = make_splat(nullptr, nullptr, 0, nullptr, nullptr, nullptr, sigma);
  ProfScope ps(plan, GA_K_READOUT, stream);
  hipLaunchKernelGGL(k_make_items, dim3((n_poses + 63) / 64), dim3(64), 0, stream, items, n_poses,
                     reinterpret_cast<const float4*>(d_xyzr), d_w, (long long)n_pts,
                     reinterpret_cast<const float4*>(d_FA4), (const float2*)nullptr, d_R, d_t, h_c[0], h_c[1],
                     h_c[2], n);
  dispatch_axis(n, [&]<int N>() {
    if constexpr (N <= 256) {
    hipLaunchKernelGGL(k_local_query<N>, dim3(nblk, n_poses), dim3(256), 0, stream, (const QueryItem*)items, part,
                       sp.sig_c, sp.e0, sp.inv1me0);
    }
  });
  hipLaunchKernelGGL(k_reduce_partials, dim3(n_poses), dim3(64), 0, stream, (const double*)part, nblk, d_out7, 1.0,
                     (const QueryItem*)items);
  return launch_status();
}

ga_status ga_pose_prepare(const ga_plan* plan, const float* d_Ahat, float* d_AX2, hipStream_t stream) {
  if (!valid_stream_call(plan) || !d_Ahat || !d_AX2) return GA_EINVAL;
  if (!all_aligned(d_Ahat, d_AX2)) return GA_EINVAL;
  const int n = plan->n;
  if (!plane_edge(n)) return GA_EUNSUPPORTED;
  const size_t spec_b = spectrum_elems(n) * sizeof(float2);
  if (overlaps(d_Ahat, spec_b, d_AX2, 2 * spec_b)) return GA_EINVAL;
  ProfScope ps(plan, GA_K_READOUT, stream);
  dispatch(n, [&]<int N>() {
    Launch<N>::ax_prepare(reinterpret_cast<const float2*>(d_Ahat), reinterpret_cast<float2*>(d_AX2), plan->d_tw,
                          stream);
  });
  return launch_status();
}

ga_status ga_pose_spectral(const ga_plan* plan, const float* d_AX2, const float* d_xyzr, const float* d_w,
                           int64_t n_pts, const float* d_R, const float* h_c, float sigma, const float* d_t,
                           int32_t n_poses, float* d_out7, void* d_work, size_t work_bytes, hipStream_t stream) {
  if (!valid_stream_call(plan) || !d_AX2 || n_pts < 0 || (n_pts > 0 && (!d_xyzr || !d_w)) || !h_c ||
      !valid_sigma(sigma) || n_poses < 0 || n_poses > 65535 || (n_poses > 0 && (!d_R || !d_t || !d_out7)))
    return GA_EINVAL;
  if (!all_aligned(d_AX2, d_xyzr, d_work)) return GA_EINVAL;
  if (!(std::isfinite(h_c[0]) && std::isfinite(h_c[1]) && std::isfinite(h_c[2]))) return GA_EINVAL;
  const int n = plan->n;
  if (!plane_edge(n)) return GA_EUNSUPPORTED;
  if (n_poses == 0) return GA_OK;
  const PoseSpectralLayout ly = pose_spectral_layout(n, n_poses, n_pts);
  if (!d_work || work_bytes < ly.total) return GA_ENOMEM;
  if (overlaps(d_work, work_bytes, d_out7, sizeof(float) * 7 * (size_t)n_poses) ||
      overlaps(d_work, work_bytes, d_AX2, 2 * spectrum_elems(n) * sizeof(float2)))
    return GA_EINVAL;
  char* wk = static_cast<char*>(d_work);
  QueryItem* items = reinterpret_cast<QueryItem*>(wk + ly.items);
  char* bins = wk + ly.bins;
  const BinLayout bl(n, n_poses, n_pts);
  double* part = reinterpret_cast<double*>(wk + ly.part);
  SplatParams sp = make_splat(nullptr, nullptr, 0, nullptr, nullptr, nullptr, sigma);
  ProfScope ps(plan, GA_K_READOUT, stream);
  hipLaunchKernelGGL(k_make_items, dim3((n_poses + 63) / 64), dim3(64), 0, stream, items, n_poses,
                     reinterpret_cast<const float4*>(d_xyzr), d_w, (long long)n_pts, (const float4*)nullptr,
                     reinterpret_cast<const float2*>(d_AX2), d_R, d_t, h_c[0], h_c[1], h_c[2], n);
  dispatch(n, [&]<int N>() {
    Placed* rec = reinterpret_cast<Placed*>(bins + bl.rec);
    int* off = reinterpret_cast<int*>(bins + bl.off);
    float* rmax = reinterpret_cast<float*>(bins + bl.rmax);
    int4* cand = reinterpret_cast<int4*>(bins + bl.cand);
    hipLaunchKernelGGL(k_bin_items<N>, dim3(n_poses), dim3(1024), 0, stream, (const QueryItem*)items, sp,
                       (long long)n_pts, rec, off, rmax, cand);
    SplatParams sq = sp;
    sq.rec = rec;
    sq.off = off;
    sq.rmax = rmax;
    sq.cand = cand;
    sq.n_pts = n_pts;
    Launch<N>::plane_single(sq, items, part, n_poses, plan->d_tw, stream);
  });
  const double scale = 1.0 / ((double)n * n * n);
  hipLaunchKernelGGL(k_reduce_partials, dim3(n_poses), dim3(64), 0, stream, (const double*)part, single_blocks_of(n),
                     d_out7, scale, (const QueryItem*)items);
  return launch_status();
}

// Times the fused x-pass candidates groups (4, 8) x k (1, 2, 4, 8) on the
// grids in xcds (plain 2, XCD-aware 1) on d_work (zeroed first) against
// d_Ahat: one warm-up and three timed launches each. h_us (n_us entries) gets
// the per-launch times in the order xcd x groups x k; the fastest is returned.
static ga_status time_strip_candidates(const ga_plan* plan, const float* d_Ahat, int32_t batch, void* d_work,
                                       hipStream_t stream, const int* xcds, int nx, float* h_us, int32_t n_us,
                                       TuneEntry& best) {
  int nradix = 1;
  dispatch_axis(plan->n, [&]<int N>() { nradix = Launch<N>::kAltRadix ? 2 : 1; });
  const int n = plan->n;
  float2* tmp = static_cast<float2*>(d_work);
  const long long n4 = (long long)((size_t)batch * spectrum_elems(n) * sizeof(float2) / sizeof(float4));
  hipLaunchKernelGGL(k_zero4, dim3((unsigned)std::min<long long>((n4 + 255) / 256, 65535)), dim3(256), 0, stream,
                     static_cast<float4*>(d_work), n4);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return GA_EDEVICE;
  }
  static constexpr int kGroups[2] = {4, 8}, kKs[4] = {1, 2, 4, 8};
  ga_status st = GA_OK;
  int idx = 0;
  for (int xi = 0; xi < nx && st == GA_OK; ++xi)
    for (int rx = 0; rx < 2 && st == GA_OK; ++rx)
    for (int gi = 0; gi < 2 && st == GA_OK; ++gi)
      for (int ki = 0; ki < 4 && st == GA_OK; ++ki, ++idx) {
        if (rx >= nradix) {  // no alternative schedule: the slot stays 0
          if (idx < n_us) h_us[idx] = 0.f;
          continue;
        }
        const int g = kGroups[gi], k = kKs[ki], x = xcds[xi];
        auto run = [&]() {
          dispatch_axis(n, [&]<int N>() {
            Launch<N>::corr_fwd_tuned(g, k, x == 1, rx, reinterpret_cast<const float2*>(d_Ahat), 0, tmp, batch,
                                      plan->d_tw, stream);
          });
        };
        run();  // warm-up
        (void)hipEventRecord(e0, stream);
        for (int r = 0; r < 3; ++r) run();
        (void)hipEventRecord(e1, stream);
        float ms = 0.f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
          st = GA_EDEVICE;
          break;
        }
        const float us = ms * 1000.f / 3.f;
        if (idx < n_us) h_us[idx] = us;
        if (idx == 0 || us < best.us) {
          best.us = us;
          best.groups = g;
          best.k = k;
          best.xcd = x;
          best.radix = rx;
        }
      }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != GA_OK) return st;
  return launch_status();
}

ga_status ga_plan_autotune(ga_plan* plan, const float* d_Ahat, int32_t batch, void* d_work, size_t work_bytes,
                           hipStream_t stream, float* h_us, int32_t n_us) {
  if (!valid_stream_call(plan) || !d_Ahat || batch < 1 || batch > plan->max_batch || n_us < 0 || (n_us > 0 && !h_us))
    return GA_EINVAL;
  if (!all_aligned(d_Ahat, d_work)) return GA_EINVAL;
  const size_t spec_b = spectrum_elems(plan->n) * sizeof(float2);
  const size_t tmp_b = (size_t)batch * spec_b;
  if (!d_work || work_bytes < tmp_b) return GA_ENOMEM;
  if (overlaps(d_work, tmp_b, d_Ahat, spec_b)) return GA_EINVAL;
  static constexpr int kPlain[1] = {2};
  TuneEntry best;
  const ga_status st = time_strip_candidates(plan, d_Ahat, batch, d_work, stream, kPlain, 1, h_us, n_us, best);
  if (st != GA_OK) return st;
  plan->tune_groups = best.groups;
  plan->tune_k = best.k;
  plan->tune_xcd = best.xcd;
  plan->tune_radix = best.radix;
  return GA_OK;
}

ga_status ga_plan_tune(ga_plan* plan, const float* d_Ahat, const float* d_xyzr, const float* d_w, int64_t n_pts,
                       const float* d_R, const float* h_c, float sigma, int32_t batch, float* d_E, void* d_work,
                       size_t work_bytes, uint32_t flags, const char* cache_path, hipStream_t stream,
                       ga_tuning* result) {
  if (!valid_stream_call(plan) || !result || (flags & ~(GA_TUNE_XCD | GA_TUNE_OVERLAP)) != 0) return GA_EINVAL;
  if (plan->n > 192 || axis_mode(plan)) return GA_EUNSUPPORTED;
  if (batch < 1 || batch > plan->max_batch) return GA_EINVAL;
  if (!d_work || work_bytes < ga_workspace_size(plan, GA_OP_ENERGY, batch, n_pts)) return GA_ENOMEM;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, plan->device) != hipSuccess) return GA_EDEVICE;
  const std::string key = tune_key(prop.gcnArchName, plan->n, batch, 1);
  std::map<std::string, TuneEntry> cache;
  bool exists = false;
  if (cache_path && !tune_cache_load(cache_path, cache, exists)) return GA_EINVAL;  // unreadable or malformed
  auto apply = [&](const TuneEntry& e, int from_cache) -> ga_status {
    if (e.radix == 1 && !has_alt_radix(plan->n)) return GA_EINVAL;
    plan->tune_groups = e.groups;
    plan->tune_k = e.k;
    plan->tune_xcd = e.xcd;
    plan->tune_radix = e.radix;
    const ga_status s = ga_plan_set_overlap(plan, e.overlap);
    if (s != GA_OK) return s;
    result->groups = e.groups;
    result->k = e.k;
    result->xcd = e.xcd;
    result->radix = e.radix;
    result->overlap = e.overlap;
    result->us = (float)e.us;
    result->from_cache = from_cache;
    return GA_OK;
  };
  if (const auto it = cache.find(key); it != cache.end()) return apply(it->second, 1);
  // the fused x pass alone, on the workspace's spectrum part
  static constexpr int kPlain[1] = {2}, kBoth[2] = {2, 1};
  TuneEntry best;
  ga_status st = (flags & GA_TUNE_XCD) ? time_strip_candidates(plan, d_Ahat, batch, d_work, stream, kBoth, 2, nullptr, 0, best)
                                       : time_strip_candidates(plan, d_Ahat, batch, d_work, stream, kPlain, 1, nullptr, 0, best);
  if (st != GA_OK) return st;
  plan->tune_groups = best.groups;
  plan->tune_k = best.k;
  plan->tune_xcd = best.xcd;
  plan->tune_radix = best.radix;
  // whole calls for the part counts: two rounds over the candidates, the
  // best time of each kept
  static constexpr int kParts[3] = {1, 2, 4};
  const int nparts = (flags & GA_TUNE_OVERLAP) ? 3 : 1;
  const int keep_overlap = plan->chunks;
  float part_us[3] = {0.f, 0.f, 0.f};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return GA_EDEVICE;
  }
  for (int round = 0; round < 2 && st == GA_OK; ++round)
    for (int pi = 0; pi < nparts && st == GA_OK; ++pi) {
      st = ga_plan_set_overlap(plan, nparts == 1 ? keep_overlap : kParts[pi]);
      auto call = [&]() {
        return ga_energy_fields(plan, d_Ahat, d_xyzr, d_w, n_pts, d_R, h_c, sigma, batch, d_E, d_work, work_bytes,
                                stream);
      };
      for (int r = 0; r < 2 && st == GA_OK; ++r) st = call();
      if (st != GA_OK) break;
      (void)hipEventRecord(e0, stream);
      for (int r = 0; r < 5 && st == GA_OK; ++r) st = call();
      (void)hipEventRecord(e1, stream);
      float ms = 0.f;
      if (st == GA_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        st = GA_EDEVICE;
      const float us = ms * 1000.f / 5.f;
      if (round == 0 || us < part_us[pi]) part_us[pi] = us;
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != GA_OK) {
    (void)ga_plan_set_overlap(plan, keep_overlap);
    return st;
  }
  int bi = 0;
  for (int pi = 1; pi < nparts; ++pi)
    if (part_us[pi] < part_us[bi]) bi = pi;
  best.overlap = (nparts == 1) ? keep_overlap : kParts[bi];
  best.us = part_us[bi];
  st = apply(best, 0);
  if (st != GA_OK) return st;
  if (cache_path) {
    cache[key] = best;
    if (!tune_cache_store(cache_path, cache)) return GA_EINVAL;
  }
  return GA_OK;
}

ga_status ga_plan_set_tuning(ga_plan* plan, int32_t groups, int32_t k, int32_t xcd) {
  if (!plan || !(groups == 0 || groups == 4 || groups == 8) || !(k == 0 || k == 1 || k == 2 || k == 4 || k == 8) ||
      !(xcd == 0 || xcd == 1 || xcd == 2))
    return GA_EINVAL;
  plan->tune_groups = groups;
  plan->tune_k = k;
  plan->tune_xcd = xcd;
  return GA_OK;
}

ga_status ga_plan_set_radix(ga_plan* plan, int32_t radix) {
  if (!plan || (radix != 0 && radix != 1) || (radix == 1 && !has_alt_radix(plan->n))) return GA_EINVAL;
  plan->tune_radix = radix;
  return GA_OK;
}

int32_t ga_plan_get_radix(const ga_plan* plan) { return plan ? plan->tune_radix : -1; }

int32_t ga_plan_has_alt_radix(const ga_plan* plan) { return (plan && has_alt_radix(plan->n)) ? 1 : 0; }

ga_status ga_plan_get_tuning(const ga_plan* plan, int32_t* groups, int32_t* k, int32_t* xcd) {
  if (!plan || !groups || !k || !xcd) return GA_EINVAL;
  *groups = plan->tune_groups ? plan->tune_groups : 4;
  *k = plan->tune_k ? plan->tune_k : 4;
  *xcd = plan->tune_xcd ? plan->tune_xcd : 2;
  return GA_OK;
}

ga_status ga_field_table(const ga_plan* plan, const float* d_Ahat, const float* d_Bhat4, int32_t n_orient,
                         float* d_tables, void* d_work, size_t work_bytes, hipStream_t stream) {
  if (!valid_stream_call(plan) || !d_Ahat || !d_Bhat4 || !d_tables || n_orient < 1) return GA_EINVAL;
  if (!all_aligned(d_Ahat, d_Bhat4, d_tables, d_work)) return GA_EINVAL;
  const int n = plan->n;
  const size_t spec = spectrum_elems(n), n3 = (size_t)n * n * n;
  if (!d_work || work_bytes < 7 * spec * sizeof(float2) + 7 * n3 * sizeof(float)) return GA_ENOMEM;
  const size_t tab_b = (size_t)n_orient * 8 * n3 * sizeof(float);
  if (overlaps(d_work, work_bytes, d_tables, tab_b) || overlaps(d_work, work_bytes, d_Ahat, spec * 8) ||
      overlaps(d_work, work_bytes, d_Bhat4, (size_t)n_orient * 4 * spec * 8) ||
      overlaps(d_tables, tab_b, d_Ahat, spec * 8) || overlaps(d_tables, tab_b, d_Bhat4, (size_t)n_orient * 4 * spec * 8))
    return GA_EINVAL;
  const float2* A = reinterpret_cast<const float2*>(d_Ahat);
  float2* spec7 = static_cast<float2*>(d_work);
  float* fields7 = reinterpret_cast<float*>(spec7 + 7 * spec);
  const float scale = (float)(1.0 / ((double)n * n * n));
  const bool ax = axis_mode(plan);
  for (int o = 0; o < n_orient; ++o) {
    const float2* B4 = reinterpret_cast<const float2*>(d_Bhat4) + (size_t)o * 4 * spec;
    dispatch_axis(n, [&]<int N>() {
      {
        ProfScope ps(plan, GA_K_READOUT, stream);
        Launch<N>::ft_fields(A, B4, spec7, plan->d_tw, stream);
      }
      ProfScope ps(plan, GA_K_PLANE_INV, stream);
      if constexpr (plane_fits<N>()) {
        if (!ax) Launch<N>::plane_inv(spec7, fields7, scale, 7, plan->d_tw, stream);
        else Axis<N>::yz_inv(spec7, fields7, scale, 7, plan->d_tw, stream);
      } else {
        Axis<N>::yz_inv(spec7, fields7, scale, 7, plan->d_tw, stream);
      }
    });
    // one 32-byte record per voxel: a query reads 8 records, not 56 scattered floats
    hipLaunchKernelGGL(k_pack8, dim3((unsigned)std::min<size_t>((n3 + 255) / 256, 65535)), dim3(256), 0, stream,
                       fields7, reinterpret_cast<float4*>(d_tables) + (size_t)o * 2 * n3, (long long)n3);
  }
  return launch_status();
}

ga_status ga_field_table_query(const ga_plan* plan, const float* d_tables, int32_t n_orient, const int32_t* d_orient,
                               const float* d_t, int32_t n_q, float* d_out7, hipStream_t stream) {
  if (!valid_stream_call(plan) || !d_tables || n_orient < 1 || n_q < 0 || (n_q > 0 && (!d_orient || !d_t || !d_out7)))
    return GA_EINVAL;
  if (!all_aligned(d_tables)) return GA_EINVAL;
  if (n_q == 0) return GA_OK;
  const int threads = 256;
  ProfScope ps(plan, GA_K_READOUT, stream);
  hipLaunchKernelGGL(k_table_query, dim3((n_q + threads - 1) / threads), dim3(threads), 0, stream,
                     reinterpret_cast<const float4*>(d_tables), plan->n, (int)n_orient, d_orient, d_t, (int)n_q,
                     d_out7);
  return launch_status();
}

ga_status ga_spectral_rotate(const ga_plan* plan, const float* d_in, int32_t channels, const float* d_R, int32_t batch,
                             float* d_out, hipStream_t stream) {
  if (!valid_stream_call(plan) || !d_in || !d_R || !d_out || batch < 1 || (channels != 1 && channels != 4))
    return GA_EINVAL;
  if (!all_aligned(d_in, d_out)) return GA_EINVAL;
  const int n = plan->n;
  const size_t spec_b = spectrum_elems(n) * sizeof(float2);
  if (overlaps(d_in, channels * spec_b, d_out, (size_t)batch * channels * spec_b) ||
      overlaps(d_R, sizeof(float) * 9 * (size_t)batch, d_out, (size_t)batch * channels * spec_b))
    return GA_EINVAL;
  ProfScope ps(plan, GA_K_READOUT, stream);
  const auto in = reinterpret_cast<const float2*>(d_in);
  launch_rotate<PlanarSrc>(n, [&]<int N>() { return PlanarSrc<N>{in, (int)channels}; }, d_R, batch, d_out, stream);
  return launch_status();
}

ga_status ga_spectral_pack4(const ga_plan* plan, const float* d_in4, float* d_packed, hipStream_t stream) {
  if (!valid_stream_call(plan) || !d_in4 || !d_packed) return GA_EINVAL;
  if (!all_aligned(d_in4, d_packed)) return GA_EINVAL;
  const size_t spec = spectrum_elems(plan->n), bytes = 4 * spec * sizeof(float2);
  if (overlaps(d_in4, bytes, d_packed, bytes)) return GA_EINVAL;
  const long long blocks = std::min<long long>(((long long)spec + 255) / 256, 65535);
  hipLaunchKernelGGL(k_pack4, dim3((unsigned)blocks), dim3(256), 0, stream, reinterpret_cast<const float2*>(d_in4),
                     reinterpret_cast<float4*>(d_packed), (long long)spec);
  return launch_status();
}

ga_status ga_spectral_rotate_packed(const ga_plan* plan, const float* d_packed, const float* d_R, int32_t batch,
                                    float* d_out, hipStream_t stream) {
  if (!valid_stream_call(plan) || !d_packed || !d_R || !d_out || batch < 1) return GA_EINVAL;
  if (!all_aligned(d_packed, d_out)) return GA_EINVAL;
  const int n = plan->n;
  const size_t spec_b = spectrum_elems(n) * sizeof(float2), out_b = (size_t)batch * 4 * spec_b;
  if (overlaps(d_packed, 4 * spec_b, d_out, out_b) || overlaps(d_R, sizeof(float) * 9 * (size_t)batch, d_out, out_b))
    return GA_EINVAL;
  ProfScope ps(plan, GA_K_READOUT, stream);
  const auto P = reinterpret_cast<const float4*>(d_packed);
  launch_rotate<PackedSrc>(n, [&]<int N>() { return PackedSrc<N>{P}; }, d_R, batch, d_out, stream);
  return launch_status();
}

ga_status ga_lowpass(const ga_plan* plan, int32_t L, uint32_t mode, const float* d_in, float* d_out, int32_t batch,
                     float scale, hipStream_t stream) {
  if (!valid_stream_call(plan) || !d_in || !d_out || batch < 1 || !std::isfinite(scale)) return GA_EINVAL;
  if (!all_aligned(d_in, d_out)) return GA_EINVAL;
  const int n = plan->n;
  if (L < 4 || (L & 1) || L > n || (mode != GA_LOWPASS_COARSE && mode != GA_LOWPASS_ZEROPAD)) return GA_EINVAL;
  const int m = (mode == GA_LOWPASS_COARSE) ? L : n;
  const size_t in_b = (size_t)batch * spectrum_elems(n) * sizeof(float2);
  const size_t out_b = (size_t)batch * spectrum_elems(m) * sizeof(float2);
  if (overlaps(d_in, in_b, d_out, out_b)) return GA_EINVAL;
  // grid: (kz-ky runs of one kx plane, kx, batch members)
  const unsigned bx = (unsigned)((m * (m / 2 + 1) + 255) / 256);
  ProfScope ps(plan, GA_K_READOUT, stream);
  hipLaunchKernelGGL(k_lowpass, dim3(bx, (unsigned)m, (unsigned)std::min(batch, 65535)), dim3(256), 0, stream,
                     reinterpret_cast<const float2*>(d_in), reinterpret_cast<float2*>(d_out), n, L,
                     mode == GA_LOWPASS_COARSE ? 1 : 0, (int)batch, scale);
  return launch_status();
}

ga_status ga_profile_enable(ga_plan* plan, int32_t enable) {
  if (!plan) return GA_EINVAL;
  prof_drain(plan);
  for (int k = 0; k < GA_K_COUNT; ++k) {
    plan->prof_ms[k] = 0.0;
    plan->prof_count[k] = 0;
  }
  plan->prof = enable != 0;
  return GA_OK;
}

ga_status ga_profile_read(ga_plan* plan, int32_t kind, double* total_ms, int64_t* launches) {
  if (!plan || kind < 0 || kind >= GA_K_COUNT || !total_ms || !launches) return GA_EINVAL;
  prof_drain(plan);
  *total_ms = plan->prof_ms[kind];
  *launches = plan->prof_count[kind];
  return GA_OK;
}

}  // extern "C"
