// ga_lib.hip -- C ABI of libga.so: plans, argument checks and kernel launches.
// The operations, layouts and error behaviour are documented in include/ga.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <new>
#include <vector>

#include "ga.h"
#include "ga_kernels.hpp"

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
  // per-kernel timing (ga_profile_*); mutable because compute calls take a const plan
  mutable bool prof = false;
  mutable std::vector<ga_prof_entry> prof_pending;
  mutable double prof_ms[GA_K_COUNT] = {};
  mutable long long prof_count[GA_K_COUNT] = {};
};

namespace {

using namespace ga;

constexpr const char* kVersion = "ga 0.1.0 (gfx950)";

bool valid_stream_call(const ga_plan* p) { return p != nullptr && p->d_tw != nullptr; }

// Brackets one kernel launch with events on its stream when profiling is on.
struct ProfScope {
  const ga_plan* plan;
  hipStream_t stream;
  ga_prof_entry e{};
  bool on;
  ProfScope(const ga_plan* p, int kind, hipStream_t s) : plan(p), stream(s), on(p->prof) {
    if (!on) return;
    e.kind = kind;
    if (hipEventCreate(&e.start) != hipSuccess || hipEventCreate(&e.stop) != hipSuccess) {
      on = false;
      return;
    }
    (void)hipEventRecord(e.start, stream);
  }
  ~ProfScope() {
    if (!on) return;
    (void)hipEventRecord(e.stop, stream);
    plan->prof_pending.push_back(e);
  }
};

void prof_drain(const ga_plan* p) {
  for (auto& e : p->prof_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(e.stop) == hipSuccess && hipEventElapsedTime(&ms, e.start, e.stop) == hipSuccess) {
      p->prof_ms[e.kind] += ms;
      p->prof_count[e.kind] += 1;
    }
    (void)hipEventDestroy(e.start);
    (void)hipEventDestroy(e.stop);
  }
  p->prof_pending.clear();
}

ga_status launch_status() {
  const hipError_t e = hipGetLastError();
  return (e == hipSuccess) ? GA_OK : GA_EDEVICE;
}

size_t spectrum_elems(int n) { return (size_t)n * n * (n / 2 + 1); }

// Strip width per grid edge: four transforms-per-wave groups, i.e. 4 waves.
template <int N> constexpr int strip_g() { return 4 * ffts_per_wave<N>(); }
constexpr int kSingleG = 64;

template <int N> struct Launch {
  using P = Plane<N>;
  static constexpr int G = strip_g<N>();
  using T = Strip<N, G>;
  static int nstrips() { return (T::C + G - 1) / G; }
  static int nsingle() { return (T::C + kSingleG - 1) / kSingleG; }

  static void bin_samples(const SplatParams& sp, Placed* rec, int* off, float* rmax, int batch, hipStream_t s) {
    hipLaunchKernelGGL(k_bin_samples<N>, dim3(batch), dim3(256), 0, s, sp, rec, off, rmax);
  }
  // pass 1 from real grids (nch = 1) or from binned samples (nch = 1 or 4)
  static void plane_fwd(const SplatParams& sp, const float* grid, int nch, float2* out, int batch, const float2* tw,
                        hipStream_t s) {
    if (grid)
      hipLaunchKernelGGL((k_plane_fwd<N, true, 1>), dim3(N, batch), dim3(P::THREADS), 0, s, sp, grid, out, tw);
    else if (nch == 4)
      hipLaunchKernelGGL((k_plane_fwd<N, false, 4>), dim3(N, batch), dim3(P::THREADS), 0, s, sp, grid, out, tw);
    else
      hipLaunchKernelGGL((k_plane_fwd<N, false, 1>), dim3(N, batch), dim3(P::THREADS), 0, s, sp, grid, out, tw);
  }
  static void plane_inv(const float2* in, float* out, float scale, int batch, const float2* tw, hipStream_t s) {
    hipLaunchKernelGGL(k_plane_inv<N>, dim3(N, batch), dim3(P::THREADS), 0, s, in, out, scale, tw);
  }
  static void strip_fft(int dir, const float2* in, float2* out, int batch, const float2* tw, hipStream_t s) {
    if (dir < 0)
      hipLaunchKernelGGL((k_strip_fft<N, G, -1>), dim3(nstrips(), batch), dim3(T::THREADS), 0, s, in, out, tw);
    else
      hipLaunchKernelGGL((k_strip_fft<N, G, +1>), dim3(nstrips(), batch), dim3(T::THREADS), 0, s, in, out, tw);
  }
  static void strip_corr(bool fwd, const float2* A, long long a_stride, const float2* B, float2* out, int batch,
                         const float2* tw, hipStream_t s) {
    if (fwd)
      hipLaunchKernelGGL((k_strip_corr<N, G, true>), dim3(nstrips(), batch), dim3(T::THREADS), 0, s, A, a_stride, B,
                         out, tw);
    else
      hipLaunchKernelGGL((k_strip_corr<N, G, false>), dim3(nstrips(), batch), dim3(T::THREADS), 0, s, A, a_stride, B,
                         out, tw);
  }
  static void ft_fields(const float2* A, const float2* B4, float2* out7, const float2* tw, hipStream_t s) {
    hipLaunchKernelGGL((k_strip_ft_fields<N, G>), dim3(nstrips(), 7), dim3(T::THREADS), 0, s, A, B4, out7, tw);
  }
  static void single(const float2* A, const float2* B4, const float* poses, int n_poses, double* part,
                     const float2* tw, hipStream_t s) {
    hipLaunchKernelGGL((k_single_partials<N, kSingleG>), dim3(nsingle(), n_poses), dim3(256), 0, s, A, B4, poses,
                       part, tw);
  }
};

// Calls f.template operator()<N>() for a supported N; returns false otherwise.
template <class F> bool dispatch(int n, F&& f) {
  switch (n) {
    case 16: f.template operator()<16>(); return true;
    case 24: f.template operator()<24>(); return true;
    case 32: f.template operator()<32>(); return true;
    case 48: f.template operator()<48>(); return true;
    case 64: f.template operator()<64>(); return true;
    case 96: f.template operator()<96>(); return true;
    case 128: f.template operator()<128>(); return true;
    case 192: f.template operator()<192>(); return true;
    default: return false;
  }
}

int nstrips_of(int n) {
  int v = 0;
  dispatch(n, [&]<int N>() { v = Launch<N>::nstrips(); });
  return v;
}
int nsingle_of(int n) {
  int v = 0;
  dispatch(n, [&]<int N>() { v = Launch<N>::nsingle(); });
  return v;
}

bool valid_sigma(float s) { return std::isfinite(s) && s > 0.0f; }

// Workspace of the fused field path: batch spectra, then the binned samples
// (records, bin offsets, largest radius per batch member).
size_t bin_offset(int n, int batch) { return (size_t)batch * spectrum_elems(n) * sizeof(float2); }
size_t bin_bytes(int n, int batch, int64_t n_pts) {
  const size_t rec = (size_t)batch * (size_t)n_pts * sizeof(Placed);
  const size_t off = ((size_t)batch * (n + 1) * sizeof(int) + 15) / 16 * 16;
  return rec + off + (size_t)batch * sizeof(float);
}

SplatParams make_splat(const float* xyzr, const float* w, int64_t n_pts, const float* Rdev, const float* hR,
                       const float* hc, float sigma) {
  SplatParams p{};
  p.rec = nullptr;
  p.off = nullptr;
  p.rmax = nullptr;
  p.xyzr = reinterpret_cast<const float4*>(xyzr);
  p.w = w;
  p.n_pts = n_pts;
  p.Rdev = Rdev;
  for (int i = 0; i < 9; ++i) p.Rh[i] = hR ? hR[i] : ((i % 4 == 0) ? 1.f : 0.f);
  for (int i = 0; i < 3; ++i) p.c[i] = hc ? hc[i] : 0.f;
  const double sc = 1.0 / (2.0 * (double)sigma * (double)sigma);
  const double e0 = std::exp(-sc);
  p.sig_c = (float)sc;
  p.e0 = (float)e0;
  p.inv1me0 = (float)(1.0 / (1.0 - e0));
  return p;
}

bool rotation_ok(const float* R) {
  double M[9];
  for (int i = 0; i < 9; ++i) {
    if (!std::isfinite(R[i])) return false;
    M[i] = R[i];
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int k = 0; k < 3; ++k) s += M[i * 3 + k] * M[j * 3 + k];
      if (std::fabs(s - (i == j ? 1.0 : 0.0)) > 1e-4) return false;
    }
  const double det = M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) +
                     M[2] * (M[3] * M[7] - M[4] * M[6]);
  return std::fabs(det - 1.0) < 1e-4;
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
  return dispatch(n, []<int N>() {}) ? 1 : 0;
}

ga_status ga_plan_create(ga_plan** plan, int32_t n, int32_t max_batch, uint32_t flags) {
  if (!plan) return GA_EINVAL;
  *plan = nullptr;
  if (n < 8 || (n & 1) || max_batch < 1 || flags != 0) return GA_EINVAL;
  if (!ga_supported_n(n)) return GA_EUNSUPPORTED;
  ga_plan* p = new (std::nothrow) ga_plan{};
  if (!p) return GA_ENOMEM;
  p->n = n;
  p->max_batch = max_batch;
  p->flags = flags;
  if (hipGetDevice(&p->device) != hipSuccess) {
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
  if (plan->d_tw) (void)hipFree(plan->d_tw);
  delete plan;
  return GA_OK;
}

int32_t ga_plan_n(const ga_plan* plan) { return plan ? plan->n : 0; }

size_t ga_workspace_size(const ga_plan* plan, int32_t op, int32_t batch, int64_t n_items) {
  if (!plan || batch < 0 || n_items < 0) return 0;
  const int n = plan->n;
  const size_t spec = spectrum_elems(n) * sizeof(float2);
  const size_t real = (size_t)n * n * n * sizeof(float);
  switch (op) {
    case GA_OP_FFT_C2R:
    case GA_OP_CORRELATE: return (size_t)batch * spec;
    case GA_OP_ENERGY: return bin_offset(n, batch) + bin_bytes(n, batch, n_items);
    case GA_OP_FORCE_FIELDS: return 7 * spec + 7 * real;
    case GA_OP_FORCE_SINGLE: return (size_t)n_items * nsingle_of(n) * 7 * sizeof(double);
    default: return 0;
  }
}

ga_status ga_splat(const ga_plan* plan, const float* d_xyzr, const float* d_w, int64_t n_pts, const float* h_R,
                   const float* h_c, float sigma, int32_t channels, float* d_grid, hipStream_t stream) {
  if (!valid_stream_call(plan) || !d_grid || n_pts < 0 || (n_pts > 0 && (!d_xyzr || !d_w))) return GA_EINVAL;
  if ((channels != 1 && channels != 4) || !valid_sigma(sigma)) return GA_EINVAL;
  if ((h_R == nullptr) != (h_c == nullptr)) return GA_EINVAL;
  if (h_R && !rotation_ok(h_R)) return GA_EINVAL;
  if (h_c && !(std::isfinite(h_c[0]) && std::isfinite(h_c[1]) && std::isfinite(h_c[2]))) return GA_EINVAL;
  const int n = plan->n;
  const size_t n3 = (size_t)n * n * n;
  if (n_pts == 0) {
    (void)hipMemsetAsync(d_grid, 0, sizeof(float) * n3 * channels, stream);
    return launch_status();
  }
  SplatParams sp = make_splat(d_xyzr, d_w, n_pts, nullptr, h_R, h_c, sigma);
  dispatch(n, [&]<int N>() {
    ProfScope ps(plan, GA_K_SPLAT, stream);
    hipLaunchKernelGGL(k_splat_real<N>, dim3(N), dim3(Plane<N>::THREADS), 0, stream, sp, channels, d_grid);
  });
  return launch_status();
}

ga_status ga_fft3d(const ga_plan* plan, int32_t dir, const void* d_in, void* d_out, int32_t batch, void* d_work,
                   size_t work_bytes, hipStream_t stream) {
  if (!valid_stream_call(plan) || !d_in || !d_out || batch < 1 || batch > plan->max_batch) return GA_EINVAL;
  if (dir != GA_R2C && dir != GA_C2R) return GA_EINVAL;
  const int n = plan->n;
  if (dir == GA_R2C) {
    float2* out = static_cast<float2*>(d_out);
    SplatParams sp = make_splat(nullptr, nullptr, 0, nullptr, nullptr, nullptr, 0.5f);
    dispatch(n, [&]<int N>() {
      {
        ProfScope ps(plan, GA_K_PLANE_FWD, stream);
        Launch<N>::plane_fwd(sp, static_cast<const float*>(d_in), 1, out, batch, plan->d_tw, stream);
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
  if (!d_work || work_bytes < ga_workspace_size(plan, GA_OP_CORRELATE, batch, 0)) return GA_ENOMEM;
  const int n = plan->n;
  float2* tmp = static_cast<float2*>(d_work);
  const float scale = (float)(1.0 / ((double)n * n * n));
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

ga_status ga_energy_fields(const ga_plan* plan, const float* d_Ahat, const float* d_xyzr, const float* d_w,
                           int64_t n_pts, const float* d_R, const float* h_c, float sigma, int32_t batch,
                           float* d_E, void* d_work, size_t work_bytes, hipStream_t stream) {
  if (!valid_stream_call(plan) || !d_Ahat || !d_R || !h_c || !d_E || batch < 1 || batch > plan->max_batch ||
      n_pts < 0 || (n_pts > 0 && (!d_xyzr || !d_w)) || !valid_sigma(sigma))
    return GA_EINVAL;
  if (!(std::isfinite(h_c[0]) && std::isfinite(h_c[1]) && std::isfinite(h_c[2]))) return GA_EINVAL;
  if (!d_work || work_bytes < ga_workspace_size(plan, GA_OP_ENERGY, batch, n_pts)) return GA_ENOMEM;
  const int n = plan->n;
  float2* tmp = static_cast<float2*>(d_work);
  const float scale = (float)(1.0 / ((double)n * n * n));
  SplatParams sp = make_splat(d_xyzr, d_w, n_pts, d_R, nullptr, h_c, sigma);
  char* bins = static_cast<char*>(d_work) + bin_offset(n, batch);
  Placed* rec = reinterpret_cast<Placed*>(bins);
  int* off = reinterpret_cast<int*>(bins + (size_t)batch * (size_t)n_pts * sizeof(Placed));
  float* rmax = reinterpret_cast<float*>(reinterpret_cast<char*>(off) +
                                         ((size_t)batch * (n + 1) * sizeof(int) + 15) / 16 * 16);
  dispatch(n, [&]<int N>() {
    {
      {
        ProfScope pb(plan, GA_K_BIN, stream);
        Launch<N>::bin_samples(sp, rec, off, rmax, batch, stream);
      }
      ProfScope ps(plan, GA_K_PLANE_FWD, stream);
      SplatParams spb = sp;
      spb.rec = rec;
      spb.off = off;
      spb.rmax = rmax;
      Launch<N>::plane_fwd(spb, nullptr, 1, tmp, batch, plan->d_tw, stream);
    }
    {
      ProfScope ps(plan, GA_K_STRIP, stream);
      Launch<N>::strip_corr(true, reinterpret_cast<const float2*>(d_Ahat), 0, tmp, tmp, batch, plan->d_tw, stream);
    }
    ProfScope ps(plan, GA_K_PLANE_INV, stream);
    Launch<N>::plane_inv(tmp, d_E, scale, batch, plan->d_tw, stream);
  });
  return launch_status();
}

ga_status ga_force_torque(const ga_plan* plan, const float* d_Ahat, const float* d_Bhat4, const float* d_t,
                          int32_t n_poses, uint32_t mode, float* d_out7, void* d_work, size_t work_bytes,
                          hipStream_t stream) {
  if (!valid_stream_call(plan) || !d_Ahat || !d_Bhat4 || n_poses < 0 || (n_poses > 0 && (!d_t || !d_out7)))
    return GA_EINVAL;
  if (mode != GA_FIELDS && mode != GA_SINGLE) return GA_EINVAL;
  if (n_poses == 0) return GA_OK;
  const int n = plan->n;
  const int op = (mode == GA_FIELDS) ? GA_OP_FORCE_FIELDS : GA_OP_FORCE_SINGLE;
  if (!d_work || work_bytes < ga_workspace_size(plan, op, 1, (int64_t)n_poses)) return GA_ENOMEM;
  const float2* A = reinterpret_cast<const float2*>(d_Ahat);
  const float2* B4 = reinterpret_cast<const float2*>(d_Bhat4);
  if (mode == GA_FIELDS) {
    float2* spec7 = static_cast<float2*>(d_work);
    float* fields7 = reinterpret_cast<float*>(spec7 + 7 * spectrum_elems(n));
    const float scale = (float)(1.0 / ((double)n * n * n));
    dispatch(n, [&]<int N>() {
      {
        ProfScope ps(plan, GA_K_READOUT, stream);
        Launch<N>::ft_fields(A, B4, spec7, plan->d_tw, stream);
      }
      ProfScope ps(plan, GA_K_PLANE_INV, stream);
      Launch<N>::plane_inv(spec7, fields7, scale, 7, plan->d_tw, stream);
    });
    ProfScope ps(plan, GA_K_READOUT, stream);
    const int threads = 256, total = n_poses * 7;
    hipLaunchKernelGGL(k_gather7, dim3((total + threads - 1) / threads), dim3(threads), 0, stream, fields7, n, d_t,
                       n_poses, d_out7);
  } else {
    double* part = static_cast<double*>(d_work);
    ProfScope ps(plan, GA_K_READOUT, stream);
    dispatch(n, [&]<int N>() { Launch<N>::single(A, B4, d_t, n_poses, part, plan->d_tw, stream); });
    const double scale = 1.0 / ((double)n * n * n);
    hipLaunchKernelGGL(k_reduce_partials, dim3(n_poses), dim3(64), 0, stream, part, nsingle_of(n), d_out7, scale);
  }
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
