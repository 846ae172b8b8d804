// ga_launch.hpp -- launch helpers (grid and block shapes of every kernel) and
// workspace layout shared by the library's translation units (ga_lib.hip,
// ga_server.hip, ga_batch.hip); the plan object is in ga_plan.hpp.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "ga.h"
#include "ga_kernels.hpp"
#include "ga_plan.hpp"

namespace ga_detail {

using namespace ga;

inline constexpr const char* kVersion = "ga 0.1.0 (gfx950)";

inline bool valid_stream_call(const ga_plan* p) { return p != nullptr && p->d_tw != nullptr; }

// Device buffers are read and written with 16-byte vector accesses.
template <class... P> inline bool all_aligned(P... p) {
  return ((reinterpret_cast<uintptr_t>(p) % 16 == 0) && ...);
}

// Brackets one kernel launch with events on its stream when profiling is on.
struct ProfScope {
  const ga_plan* plan;
  hipStream_t stream;
  ga_prof_entry e{};
  bool on;
  ProfScope(const ga_plan* p, int kind, hipStream_t s) : plan(p), stream(s), on(p->prof) {
    if (!on) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) {
      on = false;  // no timing events inside a captured graph
      return;
    }
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

inline void prof_drain(const ga_plan* p) {
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

inline ga_status launch_status() {
  const hipError_t e = hipGetLastError();
  return (e == hipSuccess) ? GA_OK : GA_EDEVICE;
}

inline size_t spectrum_elems(int n) { return (size_t)n * n * (n / 2 + 1); }

// Strip width per grid edge: four transforms-per-wave groups, i.e. 4 waves,
// and at least 16 columns (128-byte runs of global memory per x row).
template <int N> constexpr int strip_g() { return 4 * ffts_per_wave<N>() < 16 ? 16 : 4 * ffts_per_wave<N>(); }
constexpr int kSingleG = 64;

template <int N> struct Launch {
  using P = Plane<N>;
  static constexpr int G = strip_g<N>();
  using T = Strip<N, G>;
  static int nstrips() { return (T::C + G - 1) / G; }
  static int nsingle() { return (T::C + kSingleG - 1) / kSingleG; }

  static void bin_samples(const SplatParams& sp, Placed* rec, int* off, float* rmax, int4* cand, int batch,
                          hipStream_t s) {
    // one workgroup per member: 1024 threads, as a batch has far fewer members than CUs
    hipLaunchKernelGGL(k_bin_samples<N>, dim3(batch), dim3(1024), 0, s, sp, rec, off, rmax, cand);
  }
  // pass 1 from real grids, or from binned samples when grid is null
  static void plane_fwd(const SplatParams& sp, const float* grid, float2* out, int batch, const float2* tw,
                        hipStream_t s) {
    if (grid)
      hipLaunchKernelGGL((k_plane_fwd<N, true>), dim3(N, batch), dim3(P::THREADS), 0, s, sp, grid, out, tw);
    else
      plane_splat(sp, out, batch, tw, s);
  }
  // pass 1 from binned samples (sp.rec, sp.cand): the spectra of u
  static void plane_splat(const SplatParams& sp, float2* out, int batch, const float2* tw, hipStream_t s) {
    if constexpr (PlaneP<N>::ok)
      hipLaunchKernelGGL((k_plane_splat_fwd<N>), dim3(N, batch), dim3(PlaneP<N>::THREADS), 0, s, sp, out, tw);
    else
      hipLaunchKernelGGL((k_plane_fwd<N, false>), dim3(N, batch), dim3(P::THREADS), 0, s, sp, nullptr, out, tw);
  }
  // Re-correlated single-translation sums of `batch` queries (binned samples
  // sp.rec, sp.cand; items with the pair's AX): part = batch x
  // single_blocks() x 7 partial sums.
  static int single_blocks() { return 3 * N; }
  static void plane_single(const SplatParams& sp, const QueryItem* items, double* part, int batch, const float2* tw,
                           hipStream_t s) {
    if constexpr (PlaneP<N>::ok)
      hipLaunchKernelGGL(k_plane_single<N>, dim3(N, batch, 3), dim3(PlaneP<N>::THREADS), 0, s, sp, items, part, tw);
    else
      hipLaunchKernelGGL(k_plane_single_gen<N>, dim3(N, batch, 3), dim3(P::THREADS), 0, s, sp, items, part, tw);
  }
  // AX = x-inverse transforms of Ahat and of 2 pi i omega(kx) Ahat (2 spectra)
  static void ax_prepare(const float2* A, float2* ax2, const float2* tw, hipStream_t s) {
    const size_t spec = (size_t)N * N * (N / 2 + 1);
    hipLaunchKernelGGL(k_ax_inputs<N>, dim3((unsigned)((spec + 255) / 256)), dim3(256), 0, s, A, ax2);
    strip_fft(+1, ax2, ax2, 2, tw, s);
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
  // Fused correlation strip pass. With a shared stationary spectrum a
  // workgroup takes K batch members (default 4) on strips of G = groups x
  // transforms-per-wave columns (default 4 groups), with the x transforms on
  // the default radix schedule or its alternative (radix = 1); the
  // autotuner picks all three per plan.
  static constexpr int kCorrK = 4;
  // bmask: the plane masks of buf's members from pass 1 (or null: dense)
  template <int GG, int K, class SH>
  static void corr_fwd(const float2* A, long long a_stride, float2* buf, int batch, bool xcd, const float2* tw,
                       hipStream_t s, const unsigned* bmask) {
    using TT = Strip<N, GG, SH>;
    const int ns = (TT::C + GG - 1) / GG, m = (batch + K - 1) / K;
    if (xcd)
      hipLaunchKernelGGL((k_strip_corr<N, GG, true, K, SH>), dim3((unsigned)(((ns + 7) / 8) * 8 * m)),
                         dim3(TT::THREADS), 0, s, A, a_stride, buf, buf, batch, m, tw, bmask);
    else
      hipLaunchKernelGGL((k_strip_corr<N, GG, true, K, SH>), dim3(ns, m), dim3(TT::THREADS), 0, s, A, a_stride, buf,
                         buf, batch, 0, tw, bmask);
  }
  template <int GG, class SH>
  static void corr_fwd_k(int k, const float2* A, long long a_stride, float2* buf, int batch, bool xcd,
                         const float2* tw, hipStream_t s, const unsigned* bmask) {
    switch (k) {
      case 1: corr_fwd<GG, 1, SH>(A, a_stride, buf, batch, xcd, tw, s, bmask); break;
      case 2: corr_fwd<GG, 2, SH>(A, a_stride, buf, batch, xcd, tw, s, bmask); break;
      case 8: corr_fwd<GG, 8, SH>(A, a_stride, buf, batch, xcd, tw, s, bmask); break;
      default: corr_fwd<GG, 4, SH>(A, a_stride, buf, batch, xcd, tw, s, bmask); break;
    }
  }
  // groups in {4, 8}, k in {1, 2, 4, 8}; k > 1 only with a shared spectrum.
  // Above 256 (few transforms per wavefront, large register footprint) the
  // strip keeps its default width and one member per workgroup.
  template <class SH>
  static constexpr bool tunable() {
    return N <= 256 && 4 * ffts_per_wave<N, SH>() >= 16;
  }
  static constexpr bool kTunable = tunable<Shape<N>>();
  // whether the alternative radix schedule exists for this edge
  static constexpr bool kAltRadix = ShapeAlt<N>::kDistinct && tunable<ShapeAlt<N>>();
  static void corr_fwd_tuned(int groups, int k, bool xcd, int radix, const float2* A, long long a_stride, float2* buf,
                             int batch, const float2* tw, hipStream_t s, const unsigned* bmask = nullptr) {
    if (a_stride != 0 || batch == 1) k = 1;
    if constexpr (!kTunable) {
      corr_fwd<G, 1, Shape<N>>(A, a_stride, buf, batch, xcd, tw, s, bmask);
    } else {
      if constexpr (kAltRadix) {
        if (radix == 1) {
          using SA = ShapeAlt<N>;
          if (groups == 8) corr_fwd_k<8 * ffts_per_wave<N, SA>(), SA>(k, A, a_stride, buf, batch, xcd, tw, s, bmask);
          else corr_fwd_k<4 * ffts_per_wave<N, SA>(), SA>(k, A, a_stride, buf, batch, xcd, tw, s, bmask);
          return;
        }
      }
      if (groups == 8) corr_fwd_k<8 * ffts_per_wave<N>(), Shape<N>>(k, A, a_stride, buf, batch, xcd, tw, s, bmask);
      else corr_fwd_k<4 * ffts_per_wave<N>(), Shape<N>>(k, A, a_stride, buf, batch, xcd, tw, s, bmask);
    }
  }
  static void strip_corr(bool fwd, const float2* A, long long a_stride, const float2* B, float2* out, int batch,
                         const float2* tw, hipStream_t s) {
    if (fwd && B == out) {
      corr_fwd_tuned(4, kCorrK, false, 0, A, a_stride, out, batch, tw, s);
    } else if (fwd) {
      hipLaunchKernelGGL((k_strip_corr<N, G, true, 1>), dim3(nstrips(), batch), dim3(T::THREADS), 0, s, A, a_stride, B,
                         out, batch, 0, tw, nullptr);
    } else {
      hipLaunchKernelGGL((k_strip_corr<N, G, false, 1>), dim3(nstrips(), batch), dim3(T::THREADS), 0, s, A, a_stride,
                         B, out, batch, 0, tw, nullptr);
    }
  }
  // complex score: nparts = 1 or 2 product spectra per member from part `first`
  // (both parts from one read of the spectra where the Im products fit in
  // registers: at most 16 strip elements per thread, and power-of-two edges,
  // whose transforms hold fewer registers than the radix-3 ones)
  static void strip_score(const float2* A2, long long a_stride, const float2* B2, float2* out, int batch, int first,
                          int nparts, const float2* tw, hipStream_t s) {
    constexpr int IT = (N * G + T::THREADS - 1) / T::THREADS;
    if (nparts == 2 && IT <= 16 && (N & (N - 1)) == 0)
      hipLaunchKernelGGL((k_strip_score<N, G, true>), dim3(nstrips(), batch), dim3(T::THREADS), 0, s, A2, a_stride,
                         B2, out, 0, tw);
    else
      hipLaunchKernelGGL((k_strip_score<N, G, false>), dim3(nstrips(), batch, nparts), dim3(T::THREADS), 0, s, A2,
                         a_stride, B2, out, first, tw);
  }
  // the 7 force/torque products with the inverse x FFT: spectra read once per
  // strip where the products fit in registers (at most 16 strip elements per
  // thread), else one output per workgroup
  static void ft_fields(const float2* A, const float2* B4, float2* out7, const float2* tw, hipStream_t s) {
    constexpr int IT = (N * G + T::THREADS - 1) / T::THREADS;
    if constexpr (IT <= 16)
      hipLaunchKernelGGL((k_strip_ft_fields2<N, G>), dim3(nstrips(), 2), dim3(T::THREADS), 0, s, A, B4, out7, tw);
    else
      hipLaunchKernelGGL((k_strip_ft_fields<N, G>), dim3(nstrips(), 7), dim3(T::THREADS), 0, s, A, B4, out7, tw);
  }
  static void single(const float2* A, const float2* B4, const float* poses, int n_poses, double* part,
                     const float2* tw, hipStream_t s) {
    hipLaunchKernelGGL((k_single_partials<N, kSingleG>), dim3(nsingle(), n_poses), dim3(256), 0, s, A, B4, poses,
                       part, tw);
  }
};

// Whether one x-plane of edge N fits in LDS (plane path kernels exist).
template <int N> constexpr bool plane_fits() { return N <= 192; }

// Separate-axis path of a grid edge (see k_splat_atomic ... k_pencil_fft).
template <int N> struct Axis {
  using LN = Launch<N>;
  static constexpr int G = strip_g<N>();
  using T = Strip<N, G>;
  static constexpr int H = N / 2 + 1;
  // zeroed real grids [batch][nch][N^3], then the splat of every batch member
  static void splat(const SplatParams& sp, int nch, float* out, int batch, hipStream_t s) {
    const long long n4 = (long long)batch * nch * N * N * N / 4;
    hipLaunchKernelGGL(k_zero4, dim3((unsigned)std::min<long long>((n4 + 255) / 256, 65535)), dim3(256), 0, s,
                       reinterpret_cast<float4*>(out), n4);
    if (sp.n_pts > 0)
      hipLaunchKernelGGL(k_splat_atomic<N>, dim3((unsigned)((sp.n_pts + 3) / 4), batch), dim3(256), 0, s, sp, nch,
                         out);
  }
  static void rows_fwd(const float* in, float2* out, long long planes, const float2* tw, hipStream_t s) {
    const long long nrp = planes * (N / 2);
    hipLaunchKernelGGL(k_rows_fwd<N>, dim3((unsigned)((nrp + Rows<N>::PER_WG - 1) / Rows<N>::PER_WG)), dim3(256), 0,
                       s, in, out, nrp, tw);
  }
  static void rows_inv(const float2* in, float* out, float scale, long long planes, const float2* tw, hipStream_t s) {
    const long long nrp = planes * (N / 2);
    hipLaunchKernelGGL(k_rows_inv<N>, dim3((unsigned)((nrp + Rows<N>::PER_WG - 1) / Rows<N>::PER_WG)), dim3(256), 0,
                       s, in, out, scale, nrp, tw);
  }
  // y transforms of every column of `planes` x-planes, in place
  static void pencil_y(int dir, float2* buf, long long planes, const float2* tw, hipStream_t s) {
    const dim3 grid((H + G - 1) / G, (unsigned)planes);
    if (dir < 0)
      hipLaunchKernelGGL((k_pencil_fft<N, G, -1>), grid, dim3(T::THREADS), 0, s, buf, buf, (long long)H, H,
                         (long long)N * H, tw);
    else
      hipLaunchKernelGGL((k_pencil_fft<N, G, +1>), grid, dim3(T::THREADS), 0, s, buf, buf, (long long)H, H,
                         (long long)N * H, tw);
  }
  // real grids -> half spectra with z and y transformed (x not yet)
  static void zy_fwd(const float* in, float2* out, int batch, const float2* tw, hipStream_t s) {
    rows_fwd(in, out, (long long)batch * N, tw, s);
    pencil_y(-1, out, (long long)batch * N, tw, s);
  }
  // spectra with x already inverse-transformed -> real grids (y, z inverse)
  static void yz_inv(float2* spec, float* out, float scale, int batch, const float2* tw, hipStream_t s) {
    pencil_y(+1, spec, (long long)batch * N, tw, s);
    rows_inv(spec, out, scale, (long long)batch * N, tw, s);
  }
};

// Calls f.template operator()<N>() for a grid edge of the separate-axis
// path (every supported edge); returns false otherwise.
template <class F> bool dispatch_axis(int n, F&& f) {
  switch (n) {
    case 16: f.template operator()<16>(); return true;
    case 24: f.template operator()<24>(); return true;
    case 32: f.template operator()<32>(); return true;
    case 48: f.template operator()<48>(); return true;
    case 64: f.template operator()<64>(); return true;
    case 96: f.template operator()<96>(); return true;
    case 128: f.template operator()<128>(); return true;
    case 192: f.template operator()<192>(); return true;
    case 256: f.template operator()<256>(); return true;
    case 384: f.template operator()<384>(); return true;
    case 512: f.template operator()<512>(); return true;
    default: return false;
  }
}

// Calls f.template operator()<N>() for a grid edge whose x-plane fits in LDS
// (the plane path); returns false otherwise.
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

inline int nstrips_of(int n) {
  int v = 0;
  dispatch_axis(n, [&]<int N>() { v = Launch<N>::nstrips(); });
  return v;
}
inline int single_blocks_of(int n) {
  int v = 0;
  dispatch(n, [&]<int N>() { v = Launch<N>::single_blocks(); });
  return v;
}
inline int nsingle_of(int n) {
  int v = 0;
  dispatch_axis(n, [&]<int N>() { v = Launch<N>::nsingle(); });
  return v;
}
// Whether a plan runs the separate-axis path (edges whose plane does not fit
// in LDS, or GA_PLAN_AXIS_PASSES).
inline bool plane_edge(int n) {
  return dispatch(n, []<int N>() {});
}
inline bool axis_mode(const ga_plan* p) { return (p->flags & GA_PLAN_AXIS_PASSES) != 0 || !plane_edge(p->n); }

// Whether the byte ranges [a, a + na) and [b, b + nb) overlap.
inline bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  if (!a || !b || na == 0 || nb == 0) return false;
  const char* pa = static_cast<const char*>(a);
  const char* pb = static_cast<const char*>(b);
  return pa < pb + nb && pb < pa + na;
}

// Workgroups of the local single-pose sums for a part of n_pts samples.
inline int nlocal_of(int64_t n_pts) { return (int)((n_pts + kLocalSPB - 1) / kLocalSPB > 0 ? (n_pts + kLocalSPB - 1) / kLocalSPB : 1); }

inline bool valid_sigma(float s) { return std::isfinite(s) && s > 0.0f; }

// Workspace of the fused field path: batch spectra, then the binned samples
// (records, bin offsets, largest radius, per-plane candidate runs and the
// plane mask of pass 1 per batch member), each part 16-byte aligned.
inline size_t bin_offset(int n, int batch) { return (size_t)batch * spectrum_elems(n) * sizeof(float2); }
struct BinLayout {
  size_t rec, off, rmax, cand, pmask, total;  // byte offsets from the start of the binned part
  BinLayout(int n, int batch, int64_t n_pts) {
    auto up = [](size_t v) { return (v + 15) / 16 * 16; };
    rec = 0;
    off = up((size_t)batch * (size_t)n_pts * sizeof(Placed));
    rmax = off + up((size_t)batch * (n + 1) * sizeof(int));
    cand = rmax + up((size_t)batch * sizeof(float));
    pmask = cand + up((size_t)batch * n * sizeof(int4));
    total = pmask + (size_t)batch * ((n + 31) / 32) * sizeof(unsigned);
  }
};
inline size_t bin_bytes(int n, int batch, int64_t n_pts) { return BinLayout(n, batch, n_pts).total; }

inline SplatParams make_splat(const float* xyzr, const float* w, int64_t n_pts, const float* Rdev, const float* hR,
                       const float* hc, float sigma) {
  SplatParams p{};
  p.rec = nullptr;
  p.off = nullptr;
  p.rmax = nullptr;
  p.cand = nullptr;
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

// Workspace of ga_pose_spectral: query items, the binned samples of every
// query, the per-plane partial sums; 16-byte aligned parts.
struct PoseSpectralLayout {
  size_t items, bins, part, total;
};
inline PoseSpectralLayout pose_spectral_layout(int n, int n_poses, int64_t n_pts) {
  auto up = [](size_t v) { return (v + 15) / 16 * 16; };
  PoseSpectralLayout l;
  l.items = 0;
  l.bins = up((size_t)n_poses * sizeof(QueryItem));
  l.part = l.bins + up(bin_bytes(n, n_poses, n_pts));
  l.total = l.part + (size_t)n_poses * single_blocks_of(n) * 7 * sizeof(double);
  return l;
}

inline bool rotation_ok(const float* R) {
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

}  // namespace ga_detail
