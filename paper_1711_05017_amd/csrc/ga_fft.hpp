// ga_fft.hpp -- wavefront-resident mixed-radix FFT engine for gfx950.
//
// One length-N complex transform is owned by L = N/E lanes of a single
// 64-lane wavefront; each lane holds E elements per stage. Stages are
// Stockham autosort steps (radix 2, 3, 4, 8 or 16) computed in place in an LDS
// region: every lane of the wave reads all its inputs, then writes all its
// outputs, so no workgroup barrier is needed between stages (a wave executes
// its LDS instructions in order). Twiddles depend only on the lane's position
// in its transform, so they are loaded once per kernel into registers.
//
// The transform computes X(k) = sum_n x(n) exp(DIR 2 pi i k n / N) with
// DIR = -1 (forward) or +1 (inverse, unnormalised): the discrete sums of
// Sec. 3.2 (eq. 7a/7b), by the Cooley-Tukey factorisation.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

namespace ga {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {  // a * conj(b)
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// a * w for DIR = -1, a * conj(w) for DIR = +1 (w = exp(-2 pi i m / N) from the table).
template <int DIR>
__device__ __forceinline__ float2 twmul(float2 a, float2 w) {
  if constexpr (DIR < 0) return cmul(a, w);
  else return cmulc(a, w);
}
// a * (DIR i)
template <int DIR>
__device__ __forceinline__ float2 mul_di(float2 a) {
  if constexpr (DIR < 0) return make_float2(a.y, -a.x);
  else return make_float2(-a.y, a.x);
}

// Compiler barrier for wave-synchronous LDS use: memory operations are not
// moved across it; the hardware keeps a wave's LDS operations in order.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---- butterflies: in-register DFTs of size R, exp(DIR 2 pi i / R) --------
template <int R, int DIR> struct Bfly;

template <int DIR> struct Bfly<2, DIR> {
  __device__ __forceinline__ static void run(float2* v) {
    const float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <int DIR> struct Bfly<3, DIR> {
  __device__ __forceinline__ static void run(float2* v) {
    constexpr float H3 = 0.86602540378443864676f;  // sin(2 pi / 3)
    const float2 a0 = v[0];
    const float2 t = cadd(v[1], v[2]);
    const float2 d = csub(v[1], v[2]);
    const float2 m = make_float2(a0.x - 0.5f * t.x, a0.y - 0.5f * t.y);
    const float2 r = cscale(mul_di<DIR>(d), H3);  // DIR i sqrt(3)/2 (a1 - a2)
    v[0] = cadd(a0, t);
    v[1] = cadd(m, r);
    v[2] = csub(m, r);
  }
};

template <int DIR> struct Bfly<4, DIR> {
  __device__ __forceinline__ static void run(float2* v) {
    const float2 t0 = cadd(v[0], v[2]);
    const float2 t1 = csub(v[0], v[2]);
    const float2 t2 = cadd(v[1], v[3]);
    const float2 t3 = mul_di<DIR>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  }
};

template <int DIR> struct Bfly<8, DIR> {
  __device__ __forceinline__ static void run(float2* v) {
    constexpr float C8 = 0.70710678118654752440f;  // cos(pi / 4)
    float2 e[4] = {v[0], v[2], v[4], v[6]};
    float2 o[4] = {v[1], v[3], v[5], v[7]};
    Bfly<4, DIR>::run(e);
    Bfly<4, DIR>::run(o);
    // o[k] *= exp(DIR 2 pi i k / 8)
    const float2 o1 = make_float2(C8 * (o[1].x - DIR * o[1].y), C8 * (o[1].y + DIR * o[1].x));
    const float2 o2 = mul_di<DIR>(o[2]);
    const float2 o3 = make_float2(C8 * (-o[3].x - DIR * o[3].y), C8 * (-o[3].y + DIR * o[3].x));
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
  }
};

// exp(DIR i pi m / 8) for a compile-time m in [0, 9]
template <int DIR>
__device__ __forceinline__ constexpr float2 w16(int m) {
  constexpr float C1 = 0.92387953251128675613f;  // cos(pi / 8)
  constexpr float S1 = 0.38268343236508977173f;  // sin(pi / 8)
  constexpr float C2 = 0.70710678118654752440f;  // cos(pi / 4)
  const float c[10] = {1.f, C1, C2, S1, 0.f, -S1, -C2, -C1, -1.f, -C1};
  const float s[10] = {0.f, S1, C2, C1, 1.f, C1, C2, S1, 0.f, -S1};
  return make_float2(c[m], DIR * s[m]);
}

// 16 = 4 x 4: DFT4 over n1 for each n2, twiddle exp(DIR 2 pi i n2 k1 / 16),
// DFT4 over n2 for each k1; output index k1 + 4 k2.
template <int DIR> struct Bfly<16, DIR> {
  __device__ __forceinline__ static void run(float2* v) {
    float2 a[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
      float2 t[4] = {v[n2], v[4 + n2], v[8 + n2], v[12 + n2]};
      Bfly<4, DIR>::run(t);
#pragma unroll
      for (int k1 = 0; k1 < 4; ++k1) a[n2][k1] = (n2 * k1 == 0) ? t[k1] : cmul(t[k1], w16<DIR>(n2 * k1));
    }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      float2 t[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
      Bfly<4, DIR>::run(t);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = t[k2];
    }
  }
};

// ---- radix schedules --------------------------------------------------------
// E elements per lane; every radix divides E; the product of radices is N.
// Shape<N> is the default schedule of edge N; ShapeAlt<N> another order of
// radices (same or different E) that the autotuner can pick for the strip
// pass; where none is defined it is the default schedule (kDistinct false).
template <int N> struct Shape;
#define GA_SHAPE(NN, EE, NSTAGES, ...)                       \
  template <> struct Shape<NN> {                             \
    static constexpr bool kDistinct = true;                  \
    static constexpr int E = EE;                             \
    static constexpr int NST = NSTAGES;                      \
    static constexpr int R[NSTAGES] = {__VA_ARGS__};         \
  };
GA_SHAPE(16, 4, 2, 4, 4)
GA_SHAPE(24, 12, 3, 3, 2, 4)
GA_SHAPE(32, 8, 2, 8, 4)
GA_SHAPE(48, 12, 3, 3, 4, 4)
GA_SHAPE(64, 8, 2, 8, 8)
GA_SHAPE(96, 24, 3, 3, 4, 8)
GA_SHAPE(128, 16, 2, 8, 16)
GA_SHAPE(192, 24, 3, 3, 8, 8)
GA_SHAPE(256, 8, 3, 8, 8, 4)
GA_SHAPE(384, 24, 4, 3, 8, 8, 2)
GA_SHAPE(512, 8, 3, 8, 8, 8)
#undef GA_SHAPE
template <int N> struct ShapeAlt : Shape<N> {
  static constexpr bool kDistinct = false;
};
#define GA_SHAPE_ALT(NN, EE, NSTAGES, ...)                   \
  template <> struct ShapeAlt<NN> {                          \
    static constexpr bool kDistinct = true;                  \
    static constexpr int E = EE;                             \
    static constexpr int NST = NSTAGES;                      \
    static constexpr int R[NSTAGES] = {__VA_ARGS__};         \
  };
GA_SHAPE_ALT(32, 8, 2, 4, 8)
GA_SHAPE_ALT(64, 16, 2, 4, 16)
GA_SHAPE_ALT(96, 24, 3, 3, 8, 4)
GA_SHAPE_ALT(128, 16, 2, 16, 8)
GA_SHAPE_ALT(192, 24, 3, 8, 8, 3)
#undef GA_SHAPE_ALT

template <int N, class SH = Shape<N>> constexpr int lanes_per_fft() { return N / SH::E; }
template <int N, class SH = Shape<N>> constexpr int ffts_per_wave() { return 64 / lanes_per_fft<N, SH>(); }
template <int N, class SH> constexpr int ns_before(int s) {
  int p = 1;
  for (int i = 0; i < s; ++i) p *= SH::R[i];
  return p;
}
template <int N, class SH> constexpr int tw_off(int s) {
  int o = 0;
  for (int i = 1; i < s; ++i) o += (SH::E / SH::R[i]) * (SH::R[i] - 1);
  return o;
}
template <int N, class SH> constexpr int tw_count() { return tw_off<N, SH>(SH::NST); }

template <int N, class SH = Shape<N>> struct Twiddles {
  using Sched = SH;
  float2 v[tw_count<N, SH>()];
};

// The same twiddles read from a table tab[m] = exp(-2 pi i m / N), m < N
// (typically in LDS), for kernels whose registers cannot hold them.
template <int N, class SH = Shape<N>> struct TwiddlesTab {
  using Sched = SH;
  const float2* tab;
};

// Twiddle r of butterfly b at stage S for transform lane `lane`.
template <int N, int S, class SH>
__device__ __forceinline__ float2 tw_at(const Twiddles<N, SH>& tw, int lane, int b, int r) {
  (void)lane;
  return tw.v[tw_off<N, SH>(S) + b * (SH::R[S] - 1) + r - 1];
}
template <int N, int S, class SH>
__device__ __forceinline__ float2 tw_at(const TwiddlesTab<N, SH>& tw, int lane, int b, int r) {
  constexpr int L = N / SH::E, R = SH::R[S], NS = ns_before<N, SH>(S);
  const int k = (lane + L * b) % NS;
  return tw.tab[r * k * (N / (NS * R))];
}

// Per-lane twiddles: stage s > 0, butterfly b, element r uses
// exp(-2 pi i r k / (NS R)) with k = j mod NS, j = lane + L b.
template <int N, int S, class SH>
__device__ __forceinline__ void load_twiddles_stage(Twiddles<N, SH>& tw, const float2* __restrict__ table, int lane) {
  if constexpr (S < SH::NST) {
    if constexpr (S > 0) {
      constexpr int E = SH::E, L = N / E, R = SH::R[S], NS = ns_before<N, SH>(S), NB = E / R;
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int j = lane + L * b;
        const int k = j % NS;
#pragma unroll
        for (int r = 1; r < R; ++r) tw.v[tw_off<N, SH>(S) + b * (R - 1) + r - 1] = table[r * k * (N / (NS * R))];
      }
    }
    load_twiddles_stage<N, S + 1, SH>(tw, table, lane);
  }
}
template <int N, class SH>
__device__ __forceinline__ void load_twiddles(Twiddles<N, SH>& tw, const float2* __restrict__ table, int lane) {
  load_twiddles_stage<N, 0, SH>(tw, table, lane);
}

// One Stockham stage, in place in LDS: element `pos` of the transform lives
// at at(pos) (a float2 pointer; any layout, e.g. strided or swizzled against
// bank conflicts). Stage 0 takes its inputs from ld(pos) and the last stage
// hands its outputs to st(pos, v), or st(pos, v, e) with e the output's
// element index in the lane (fft_out_pos); positions are natural indices.
// The schedule SH comes with the twiddles.
template <int N, int S, int DIR, class TW, class At, class Ld, class St>
__device__ __forceinline__ void fft_stage(int lane, const TW& tw, At& at, Ld& ld, St& st) {
  using SH = typename TW::Sched;
  constexpr int E = SH::E, L = N / E, R = SH::R[S], NS = ns_before<N, SH>(S), NB = E / R;
  constexpr bool first = (S == 0), last = (S == SH::NST - 1);
  float2 v[E];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = lane + L * b;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int pos = j + r * (N / R);
      if constexpr (first) v[b * R + r] = ld(pos);
      else v[b * R + r] = *at(pos);
    }
  }
  wave_sync();
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    if constexpr (S > 0) {
#pragma unroll
      for (int r = 1; r < R; ++r) v[b * R + r] = twmul<DIR>(v[b * R + r], tw_at<N, S>(tw, lane, b, r));
    }
    Bfly<R, DIR>::run(&v[b * R]);
  }
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = lane + L * b;
    const int k = j % NS;
    const int base = (j - k) * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int pos = base + r * NS;
      if constexpr (last) {
        if constexpr (std::is_invocable_v<St&, int, float2, int>) st(pos, v[b * R + r], b * R + r);
        else st(pos, v[b * R + r]);
      }
      else *at(pos) = v[b * R + r];
    }
  }
  wave_sync();
  if constexpr (!last) fft_stage<N, S + 1, DIR>(lane, tw, at, ld, st);
}

// Natural position of output element e of transform lane `lane` (as the
// last stage of fft_stage stores it) under schedule SH.
template <int N, class SH>
__device__ __forceinline__ int fft_out_pos(int lane, int e) {
  constexpr int S = SH::NST - 1, E = SH::E, L = N / E, R = SH::R[S], NS = ns_before<N, SH>(S);
  const int b = e / R, r = e % R, j = lane + L * b, k = j % NS;
  return (j - k) * R + k + r * NS;
}

// Transform of length N on the L lanes [0, L) of this transform (`lane` is
// the index within the transform), element pos at at(pos).
template <int N, int DIR, class TW, class At, class Ld, class St>
__device__ __forceinline__ void fft_at(int lane, const TW& tw, At at, Ld ld, St st) {
  fft_stage<N, 0, DIR>(lane, tw, at, ld, st);
}
template <int N, int DIR, class TW, class At>
__device__ __forceinline__ void fft_inplace_at(int lane, const TW& tw, At at) {
  auto ld = [&](int pos) { return *at(pos); };
  auto st = [&](int pos, float2 v) { *at(pos) = v; };
  fft_stage<N, 0, DIR>(lane, tw, at, ld, st);
}

// The same with data in buf[pos * es].
template <int N, int DIR, class TW, class Ld, class St>
__device__ __forceinline__ void fft_lanes(int lane, const TW& tw, float2* buf, int es, Ld ld, St st) {
  auto at = [=](int pos) { return buf + pos * es; };
  fft_stage<N, 0, DIR>(lane, tw, at, ld, st);
}
template <int N, int DIR, class TW>
__device__ __forceinline__ void fft_inplace(int lane, const TW& tw, float2* buf, int es) {
  auto at = [=](int pos) { return buf + pos * es; };
  fft_inplace_at<N, DIR>(lane, tw, at);
}

}  // namespace ga
