// ga_kernels.hpp -- HIP kernels of the correlation path (gfx950).
//
// Data flow of one energy field (three HBM passes):
//   plane_fwd  per x-plane: splat (or load) the real plane into LDS, z R2C of
//              row pairs, y FFT of the n/2+1 columns, write the plane.
//   strip_*    per strip of G (ky, kz) columns: x FFT in LDS, fused with the
//              conjugate product (and the spectral-gradient multipliers) and
//              the inverse x FFT, or with the single-pose partial sum.
//   plane_inv  per x-plane: inverse y FFT, z C2R of row pairs, write reals.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ga_fft.hpp"

namespace ga {

constexpr float kTwoPi = 6.28318530717958647692f;

template <int N> struct Plane {
  static constexpr int H = N / 2 + 1;    // half-spectrum length along z
  static constexpr int PAIR = 2 * H;     // float2 per row-pair region
  static constexpr int SIZE = N * H;     // float2 per plane
  static constexpr int L = lanes_per_fft<N>();
  static constexpr int TPW = ffts_per_wave<N>();
  static constexpr int WAVES = (N >= 192) ? 8 : 4;
  static constexpr int THREADS = 64 * WAVES;
};

constexpr int kChunk = 256;  // samples scanned per round; bounds the LDS hit list

struct SplatParams {
  const float4* xyzr;  // n_pts x (x, y, z, r)
  const float* w;      // n_pts
  long long n_pts;
  const float* Rdev;   // batch x 9 (row-major) or null -> Rh
  float Rh[9];
  float c[3];
  float sig_c;    // 1 / (2 sigma^2)
  float e0;       // exp(-1 / (2 sigma^2)) = K offset (independent of rho)
  float inv1me0;  // 1 / (1 - e0)
};

struct Hit {
  float4 a;  // dx (signed, minimum image), fy, fz, rho
  float2 b;  // packed (by, bz) as int bits, w
};

__device__ __forceinline__ int wrapn(int v, int n) {
  v = (v < 0) ? v + n : v;
  return (v >= n) ? v - n : v;
}
__device__ __forceinline__ float yhat(int q, int n) { return (float)((q < n / 2) ? q : q - n); }

// Placement of one sample, y = R (x - c) in float64, split into an integer
// voxel base (mod n) and a float32 fraction in [0, 1). Returns false for a
// sample that is not finite or whose radius reaches n/2.
template <int N>
__device__ __forceinline__ bool place_sample(const SplatParams& p, const double* R, long long s, float& fx, float& fy,
                                             float& fz, int& bx, int& by, int& bz, float& rho, float& w) {
  const float4 q = p.xyzr[s];
  w = p.w[s];
  rho = fmaxf(q.w, 1.0f);
  if (!(rho < 0.5f * N) || !isfinite(w)) return false;
  const double dx0 = (double)q.x - (double)p.c[0];
  const double dy0 = (double)q.y - (double)p.c[1];
  const double dz0 = (double)q.z - (double)p.c[2];
  const double yx = R[0] * dx0 + R[1] * dy0 + R[2] * dz0;
  const double yy = R[3] * dx0 + R[4] * dy0 + R[5] * dz0;
  const double yz = R[6] * dx0 + R[7] * dy0 + R[8] * dz0;
  if (!(fabs(yx) < 1.0e7 && fabs(yy) < 1.0e7 && fabs(yz) < 1.0e7)) return false;
  const double fbx = floor(yx), fby = floor(yy), fbz = floor(yz);
  fx = (float)(yx - fbx);
  fy = (float)(yy - fby);
  fz = (float)(yz - fbz);
  long long ix = (long long)fbx % N, iy = (long long)fby % N, iz = (long long)fbz % N;
  bx = (int)(ix < 0 ? ix + N : ix);
  by = (int)(iy < 0 ? iy + N : iy);
  bz = (int)(iz < 0 ? iz + N : iz);
  return true;
}

// Splat the samples that reach plane x into the LDS real plane Wf (voxel
// (y, z) at Wf[idx(y, z)]), each voxel value multiplied by yhat_y (chan 2)
// or yhat_z (chan 3).
template <int N, class Idx>
__device__ void splat_plane(const SplatParams& p, const double* R, int x, int chan, float* Wf, Hit* hits,
                            int* nhits, Idx idx) {
  using P = Plane<N>;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (long long c0 = 0; c0 < p.n_pts; c0 += kChunk) {
    if (tid == 0) *nhits = 0;
    __syncthreads();
    if (tid < kChunk && c0 + tid < p.n_pts) {
      float fx, fy, fz, rho, w;
      int bx, by, bz;
      if (place_sample<N>(p, R, c0 + tid, fx, fy, fz, bx, by, bz, rho, w)) {
        int m = x - bx;
        m = (m >= N / 2) ? m - N : m;
        m = (m < -N / 2) ? m + N : m;
        float dx = (float)m - fx;
        dx = (dx < -0.5f * N) ? dx + (float)N : dx;
        if (fabsf(dx) < rho && w != 0.0f) {
          const int slot = atomicAdd(nhits, 1);
          Hit h;
          h.a = make_float4(dx, fy, fz, rho);
          h.b = make_float2(__int_as_float(by | (bz << 16)), w);
          hits[slot] = h;
        }
      }
    }
    __syncthreads();
    const int nh = *nhits;
    for (int i = wave; i < nh; i += P::WAVES) {
      const Hit h = hits[i];
      const float dx = h.a.x, fy = h.a.y, fz = h.a.z, rho = h.a.w, w = h.b.y;
      const int packed = __float_as_int(h.b.x);
      const int by = packed & 0xffff, bz = packed >> 16;
      const float rho2 = rho * rho;
      const float rd = sqrtf(fmaxf(rho2 - dx * dx, 0.0f));
      const int ylo = (int)ceilf(fy - rd), yhi = (int)floorf(fy + rd);
      const int zlo = (int)ceilf(fz - rd), zhi = (int)floorf(fz + rd);
      const int sz = zhi - zlo + 1;
      const int cnt = (yhi - ylo + 1) * sz;
      const float inv2s2 = p.sig_c / rho2;
      for (int v = lane; v < cnt; v += 64) {
        const int oy = ylo + v / sz, oz = zlo + v % sz;
        const float ddy = (float)oy - fy, ddz = (float)oz - fz;
        const float d2 = dx * dx + ddy * ddy + ddz * ddz;
        if (d2 < rho2) {
          const int yy = wrapn(by + oy, N), zz = wrapn(bz + oz, N);
          float val = w * (__expf(-d2 * inv2s2) - p.e0) * p.inv1me0;
          if (chan == 2) val *= yhat(yy, N);
          if (chan == 3) val *= yhat(zz, N);
          atomicAdd(&Wf[idx(yy, zz)], val);
        }
      }
    }
    __syncthreads();
  }
}

// z R2C of every row pair and y FFT of every column, in the LDS plane W.
// On entry W holds the pair-packed real plane; on exit the plane's 2D
// spectrum [ky][kz] with row stride H.
template <int N>
__device__ void plane_forward_lds(float2* W, const Twiddles<N>& tw) {
  using P = Plane<N>;
  constexpr int L = P::L, TPW = P::TPW, H = P::H;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l = lane % L;
  // z: one complex FFT per pair of real rows, then split into the two halves
  for (int t0 = wave * TPW; t0 < N / 2; t0 += P::WAVES * TPW) {
    const int t = t0 + lane / L;
    if (t < N / 2) {
      float2* reg = W + t * P::PAIR;
      fft_inplace<N, -1>(l, tw, reg, 1);
      constexpr int KPL = (H + L - 1) / L;
      float2 za[KPL], zb[KPL];
#pragma unroll
      for (int e = 0; e < KPL; ++e) {
        const int k = l + L * e;
        if (k < H) {
          za[e] = reg[k];
          zb[e] = reg[(N - k) % N];
        }
      }
      wave_sync();
#pragma unroll
      for (int e = 0; e < KPL; ++e) {
        const int k = l + L * e;
        if (k < H) {
          const float2 a = za[e];
          const float2 b = make_float2(zb[e].x, -zb[e].y);  // conj Z(N-k)
          reg[k] = make_float2(0.5f * (a.x + b.x), 0.5f * (a.y + b.y));          // (Z + conj Z')/2
          reg[H + k] = make_float2(0.5f * (a.y - b.y), -0.5f * (a.x - b.x));     // (Z - conj Z')/(2i)
        }
      }
      wave_sync();
    }
  }
  __syncthreads();
  // y: one FFT per kz column (stride H)
  for (int t0 = wave * TPW; t0 < H; t0 += P::WAVES * TPW) {
    const int t = t0 + lane / L;
    if (t < H) fft_inplace<N, -1>(l, tw, W + t, H);
  }
  __syncthreads();
}

// Pass 1. grid = (N planes, batch). Source: splatted samples (p.xyzr != null)
// or real grids `grid` [batch][nch_in... = 1][N^3]. Writes nch spectra planes
// per batch member: out[((b*nch + c)*N + x)*N*H].
template <int N>
__global__ void __launch_bounds__(Plane<N>::THREADS) k_plane_fwd(SplatParams p, const float* __restrict__ grid,
                                                                 int nch, float2* __restrict__ out,
                                                                 const float2* __restrict__ table) {
  using P = Plane<N>;
  __shared__ float2 W[P::SIZE];
  __shared__ Hit hits[kChunk];
  __shared__ int nhits;
  const int x = blockIdx.x, b = blockIdx.y, tid = threadIdx.x;
  Twiddles<N> tw;
  load_twiddles<N>(tw, table, (tid & 63) % P::L);
  float* Wf = reinterpret_cast<float*>(W);
  double R[9];
  if (p.Rdev) {
#pragma unroll
    for (int i = 0; i < 9; ++i) R[i] = (double)p.Rdev[b * 9 + i];
  } else {
#pragma unroll
    for (int i = 0; i < 9; ++i) R[i] = (double)p.Rh[i];
  }
  const size_t plane_sz = (size_t)N * P::H;
  const int npass = (nch == 4) ? 3 : 1;
  for (int pass = 0; pass < npass; ++pass) {
    const int chan = (pass == 0) ? 0 : pass + 1;  // 0, 2, 3
    if (grid) {
      const float* src = grid + ((size_t)b * N + x) * N * N;
      for (int i = tid; i < N * N; i += P::THREADS) {
        const int y = i / N, z = i % N;
        Wf[((y >> 1) * P::PAIR + z) * 2 + (y & 1)] = src[i];
      }
      // the padding columns of each pair region are not read before written
    } else {
      for (int i = tid; i < P::SIZE; i += P::THREADS) W[i] = make_float2(0.f, 0.f);
      __syncthreads();
      splat_plane<N>(p, R, x, chan, Wf, hits, &nhits,
                     [](int yy, int zz) { return ((yy >> 1) * P::PAIR + zz) * 2 + (yy & 1); });
    }
    __syncthreads();
    plane_forward_lds<N>(W, tw);
    float2* dst = out + (((size_t)b * nch + chan) * N + x) * plane_sz;
    for (int i = tid; i < P::SIZE; i += P::THREADS) dst[i] = W[i];
    if (nch == 4 && chan == 0) {
      const float sx = yhat(x, N);
      float2* dx = out + (((size_t)b * nch + 1) * N + x) * plane_sz;
      for (int i = tid; i < P::SIZE; i += P::THREADS) dx[i] = cscale(W[i], sx);
    }
    __syncthreads();
  }
}

// The density itself: grid = (N planes). Writes nch real grids
// out[(c*N + x)*N*N + y*N + z]: u, then yhat_x u, yhat_y u, yhat_z u.
template <int N>
__global__ void __launch_bounds__(Plane<N>::THREADS) k_splat_real(SplatParams p, int nch, float* __restrict__ out) {
  using P = Plane<N>;
  __shared__ float U[N * N];
  __shared__ Hit hits[kChunk];
  __shared__ int nhits;
  const int x = blockIdx.x, tid = threadIdx.x;
  double R[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) R[i] = (double)p.Rh[i];
  for (int i = tid; i < N * N; i += P::THREADS) U[i] = 0.f;
  __syncthreads();
  splat_plane<N>(p, R, x, 0, U, hits, &nhits, [](int yy, int zz) { return yy * N + zz; });
  __syncthreads();
  const size_t n3 = (size_t)N * N * N;
  for (int i = tid; i < N * N; i += P::THREADS) {
    const float u = U[i];
    const size_t o = (size_t)x * N * N + i;
    out[o] = u;
    if (nch == 4) {
      out[n3 + o] = yhat(x, N) * u;
      out[2 * n3 + o] = yhat(i / N, N) * u;
      out[3 * n3 + o] = yhat(i % N, N) * u;
    }
  }
}

// Pass 3. grid = (N planes, batch). in: spectra after the inverse x pass,
// [b][x][ky][kz]; out: real grids [b][x][y][z] times `scale`.
template <int N>
__global__ void __launch_bounds__(Plane<N>::THREADS) k_plane_inv(const float2* __restrict__ in, float* __restrict__ out,
                                                                 float scale, const float2* __restrict__ table) {
  using P = Plane<N>;
  constexpr int L = P::L, TPW = P::TPW, H = P::H;
  __shared__ float2 W[P::SIZE];
  const int x = blockIdx.x, b = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l = lane % L;
  Twiddles<N> tw;
  load_twiddles<N>(tw, table, l);
  const float2* src = in + ((size_t)b * N + x) * (size_t)P::SIZE;
  for (int i = tid; i < P::SIZE; i += P::THREADS) W[i] = src[i];
  __syncthreads();
  for (int t0 = wave * TPW; t0 < H; t0 += P::WAVES * TPW) {
    const int t = t0 + lane / L;
    if (t < H) fft_inplace<N, +1>(l, tw, W + t, H);
  }
  __syncthreads();
  float* dst = out + ((size_t)b * N + x) * (size_t)N * N;
  for (int t0 = wave * TPW; t0 < N / 2; t0 += P::WAVES * TPW) {
    const int t = t0 + lane / L;
    if (t < N / 2) {
      float2* reg = W + t * P::PAIR;
      // Z(k) = A(k) + i B(k), completed by Hermitian symmetry; A, B are the
      // spectra of rows 2t and 2t+1 (imaginary parts dropped at k = 0, N/2)
      auto ld = [&](int k) -> float2 {
        if (k < H) {
          float2 a = reg[k], bb = reg[H + k];
          if (k == 0 || k == N / 2) {
            a.y = 0.f;
            bb.y = 0.f;
          }
          return make_float2(a.x - bb.y, a.y + bb.x);
        }
        const float2 a = reg[N - k], bb = reg[H + N - k];
        return make_float2(a.x + bb.y, bb.x - a.y);
      };
      float* r0 = dst + (size_t)(2 * t) * N;
      auto st = [&](int k, float2 v) {
        r0[k] = v.x * scale;
        r0[N + k] = v.y * scale;
      };
      fft_lanes<N, +1>(l, tw, reg, 1, ld, st);
    }
  }
}

template <int N, int G> struct Strip {
  static constexpr int H = N / 2 + 1;
  static constexpr int C = N * H;  // columns per x-plane
  static constexpr int L = lanes_per_fft<N>();
  static constexpr int TPW = ffts_per_wave<N>();
  static constexpr int WAVES = G / TPW;
  static constexpr int THREADS = 64 * WAVES;
  static constexpr int LD = G + 1;  // padded LDS row
  static_assert(G % TPW == 0, "strip width must be a whole number of transforms per wave");
};

template <int N, int G>
__device__ __forceinline__ void strip_load(float2* S, const float2* __restrict__ src, int c0) {
  using T = Strip<N, G>;
  for (int i = threadIdx.x; i < N * G; i += T::THREADS) {
    const int x = i / G, g = i % G, c = c0 + g;
    S[x * T::LD + g] = (c < T::C) ? src[(size_t)x * T::C + c] : make_float2(0.f, 0.f);
  }
}
template <int N, int G>
__device__ __forceinline__ void strip_store(const float2* S, float2* __restrict__ dst, int c0) {
  using T = Strip<N, G>;
  for (int i = threadIdx.x; i < N * G; i += T::THREADS) {
    const int x = i / G, g = i % G, c = c0 + g;
    if (c < T::C) dst[(size_t)x * T::C + c] = S[x * T::LD + g];
  }
}
template <int N, int G, int DIR>
__device__ __forceinline__ void strip_fft(float2* S, const Twiddles<N>& tw) {
  using T = Strip<N, G>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = wave * T::TPW + lane / T::L;
  fft_inplace<N, DIR>(lane % T::L, tw, S + g, T::LD);
}

// x FFT of a strip of columns, in place or out of place.
// grid = (ceil(C/G), batch); element stride between batch members = N*C.
template <int N, int G, int DIR>
__global__ void __launch_bounds__((Strip<N, G>::THREADS)) k_strip_fft(const float2* __restrict__ in,
                                                                    float2* __restrict__ out,
                                                                    const float2* __restrict__ table) {
  using T = Strip<N, G>;
  __shared__ float2 S[N * T::LD];
  Twiddles<N> tw;
  load_twiddles<N>(tw, table, (threadIdx.x & 63) % T::L);
  const size_t off = (size_t)blockIdx.y * N * T::C;
  const int c0 = blockIdx.x * G;
  strip_load<N, G>(S, in + off, c0);
  __syncthreads();
  strip_fft<N, G, DIR>(S, tw);
  __syncthreads();
  strip_store<N, G>(S, out + off, c0);
}

// Conjugate product with the stationary spectrum and inverse x FFT.
// FWD = true: `B` holds pass-1 output (x not yet transformed): forward x FFT
// first (the fused field path). FWD = false: `B` is a full spectrum.
template <int N, int G, bool FWD>
__global__ void __launch_bounds__((Strip<N, G>::THREADS)) k_strip_corr(const float2* __restrict__ A, long long a_stride,
                                                                     const float2* __restrict__ B,
                                                                     float2* __restrict__ out,
                                                                     const float2* __restrict__ table) {
  using T = Strip<N, G>;
  __shared__ float2 S[N * T::LD];
  Twiddles<N> tw;
  load_twiddles<N>(tw, table, (threadIdx.x & 63) % T::L);
  const size_t boff = (size_t)blockIdx.y * N * T::C;
  const float2* Ab = A + (size_t)blockIdx.y * (size_t)a_stride;
  const int c0 = blockIdx.x * G;
  if constexpr (FWD) {
    strip_load<N, G>(S, B + boff, c0);
    __syncthreads();
    strip_fft<N, G, -1>(S, tw);
    __syncthreads();
    for (int i = threadIdx.x; i < N * G; i += T::THREADS) {
      const int x = i / G, g = i % G, c = c0 + g;
      const float2 a = (c < T::C) ? Ab[(size_t)x * T::C + c] : make_float2(0.f, 0.f);
      S[x * T::LD + g] = cmulc(a, S[x * T::LD + g]);
    }
  } else {
    for (int i = threadIdx.x; i < N * G; i += T::THREADS) {
      const int x = i / G, g = i % G, c = c0 + g;
      float2 v = make_float2(0.f, 0.f);
      if (c < T::C) v = cmulc(Ab[(size_t)x * T::C + c], B[boff + (size_t)x * T::C + c]);
      S[x * T::LD + g] = v;
    }
  }
  __syncthreads();
  strip_fft<N, G, +1>(S, tw);
  __syncthreads();
  strip_store<N, G>(S, out + boff, c0);
}

// kappa(k)/N for a half-spectrum index: k for k < N/2, k - N above, 0 at N/2.
template <int N>
__device__ __forceinline__ float omega_of(int k) {
  return (k == N / 2) ? 0.f : (float)((k < N / 2) ? k : k - N) / (float)N;
}

// The 7 spectral products of eq. 5, 6a, 6b at one element (unscaled):
// P_E = A conj(B); P_F = -2 pi i w P_E; P_tau = 2 pi i (w x conj M) A.
__device__ __forceinline__ void products7(float2 a, float2 bu, float2 mx, float2 my, float2 mz, float wx, float wy,
                                          float wz, float2* o) {
  const float2 pe = cmulc(a, bu);
  o[0] = pe;
  // -2 pi i w pe = 2 pi w (pe.y, -pe.x)
  o[1] = make_float2(kTwoPi * wx * pe.y, -kTwoPi * wx * pe.x);
  o[2] = make_float2(kTwoPi * wy * pe.y, -kTwoPi * wy * pe.x);
  o[3] = make_float2(kTwoPi * wz * pe.y, -kTwoPi * wz * pe.x);
  // V_a = (w x conj M)_a, P = 2 pi i V A
  const float2 cx = make_float2(mx.x, -mx.y), cy = make_float2(my.x, -my.y), cz = make_float2(mz.x, -mz.y);
  const float2 vx = make_float2(wy * cz.x - wz * cy.x, wy * cz.y - wz * cy.y);
  const float2 vy = make_float2(wz * cx.x - wx * cz.x, wz * cx.y - wx * cz.y);
  const float2 vz = make_float2(wx * cy.x - wy * cx.x, wx * cy.y - wy * cx.y);
  const float2 ax = cmul(vx, a), ay = cmul(vy, a), az = cmul(vz, a);
  o[4] = make_float2(-kTwoPi * ax.y, kTwoPi * ax.x);
  o[5] = make_float2(-kTwoPi * ay.y, kTwoPi * ay.x);
  o[6] = make_float2(-kTwoPi * az.y, kTwoPi * az.x);
}

// Force/torque fields: 7 products of full spectra, inverse x FFT each.
// grid = (ceil(C/G), 7). B4 = 4 spectra (u, m_x, m_y, m_z); out7 = 7 spectra.
template <int N, int G>
__global__ void __launch_bounds__((Strip<N, G>::THREADS)) k_strip_ft_fields(const float2* __restrict__ A,
                                                                          const float2* __restrict__ B4,
                                                                          float2* __restrict__ out7,
                                                                          const float2* __restrict__ table) {
  using T = Strip<N, G>;
  __shared__ float2 S[N * T::LD];
  Twiddles<N> tw;
  load_twiddles<N>(tw, table, (threadIdx.x & 63) % T::L);
  const size_t spec = (size_t)N * T::C;
  const int o = blockIdx.y;
  const int c0 = blockIdx.x * G;
  for (int i = threadIdx.x; i < N * G; i += T::THREADS) {
    const int x = i / G, g = i % G, c = c0 + g;
    float2 v = make_float2(0.f, 0.f);
    if (c < T::C) {
      const size_t e = (size_t)x * T::C + c;
      const float wx = omega_of<N>(x), wy = omega_of<N>(c / T::H), wz = omega_of<N>(c % T::H);
      float2 pr[7];
      products7(A[e], B4[e], B4[spec + e], B4[2 * spec + e], B4[3 * spec + e], wx, wy, wz, pr);
#pragma unroll
      for (int q = 0; q < 7; ++q) v = (q == o) ? pr[q] : v;  // keeps pr in registers
    }
    S[x * T::LD + g] = v;
  }
  __syncthreads();
  strip_fft<N, G, +1>(S, tw);
  __syncthreads();
  strip_store<N, G>(S, out7 + (size_t)o * spec, c0);
}

// Single-pose partial sums (eq. 7b at one translation): for pose p and strip
// c0, sum over the strip's elements of w(kz) Re[P_o(k) exp(+2 pi i k.t/N)] in
// float64, written to part[(p * nblk + blk) * 7 + o]. Full spectra in.
// grid = (nblk = ceil(C/G), n_poses).
template <int N, int G>
__global__ void __launch_bounds__(256) k_single_partials(const float2* __restrict__ A, const float2* __restrict__ B4,
                                                         const float* __restrict__ poses, double* __restrict__ part,
                                                         const float2* __restrict__ table) {
  using T = Strip<N, G>;
  __shared__ float2 tab[N];
  __shared__ double red[256 / 64][7];
  const int tid = threadIdx.x, p = blockIdx.y;
  for (int i = tid; i < N; i += 256) tab[i] = table[i];
  __syncthreads();
  const size_t spec = (size_t)N * T::C;
  int t3[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float tf = poses[p * 3 + a];
    long long ti = (long long)roundf(tf) % N;  // nearest lattice point, ties away from zero
    t3[a] = (int)(ti < 0 ? ti + N : ti);
  }
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  const int c0 = blockIdx.x * G;
  for (int i = tid; i < N * G; i += 256) {
    const int x = i / G, g = i % G, c = c0 + g;
    if (c < T::C) {
      const int ky = c / T::H, kz = c % T::H;
      const size_t e = (size_t)x * T::C + c;
      float2 pr[7];
      products7(A[e], B4[e], B4[spec + e], B4[2 * spec + e], B4[3 * spec + e], omega_of<N>(x), omega_of<N>(ky),
                omega_of<N>(kz), pr);
      const int m = (int)(((long long)x * t3[0] + (long long)ky * t3[1] + (long long)kz * t3[2]) % N);
      const float2 ph = tab[m];  // exp(-2 pi i m/N); the sum needs its conjugate
      const double wgt = (kz == 0 || kz == N / 2) ? 1.0 : 2.0;
#pragma unroll
      for (int o = 0; o < 7; ++o) acc[o] += wgt * ((double)pr[o].x * ph.x + (double)pr[o].y * ph.y);
    }
  }
  // wave reduction then across waves, fixed order (deterministic)
#pragma unroll
  for (int o = 0; o < 7; ++o) {
    double v = acc[o];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((tid & 63) == 0) red[tid >> 6][o] = v;
  }
  __syncthreads();
  if (tid < 7) {
    double s = 0;
    for (int wv = 0; wv < 256 / 64; ++wv) s += red[wv][tid];
    part[((size_t)p * gridDim.x + blockIdx.x) * 7 + tid] = s;
  }
}

// Sum of the per-strip partials of each pose in a fixed order, times scale.
// grid = n_poses, block = 64.
__global__ void __launch_bounds__(64) k_reduce_partials(const double* __restrict__ part, int nblk, float* __restrict__ out7,
                                                        double scale) {
  __shared__ double red[7][64];
  const int p = blockIdx.x, tid = threadIdx.x;
  for (int o = 0; o < 7; ++o) {
    double s = 0;
    for (int i = tid; i < nblk; i += 64) s += part[((size_t)p * nblk + i) * 7 + o];
    red[o][tid] = s;
  }
  __syncthreads();
  if (tid < 7) {
    double s = 0;
    for (int i = 0; i < 64; ++i) s += red[tid][i];
    out7[p * 7 + tid] = (float)(s * scale);
  }
}

// Trilinear readout of 7 real fields [7][N^3] at poses (exact on lattice).
__global__ void k_gather7(const float* __restrict__ fields, int n, const float* __restrict__ poses, int n_poses,
                          float* __restrict__ out7) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_poses * 7) return;
  const int p = i / 7, o = i % 7;
  const size_t n3 = (size_t)n * n * n;
  const float* f = fields + (size_t)o * n3;
  float fl[3], a[3];
  int i0[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float t = poses[p * 3 + d];
    fl[d] = floorf(t);
    a[d] = t - fl[d];
    long long q = (long long)fl[d] % n;
    i0[d] = (int)(q < 0 ? q + n : q);
  }
  float acc = 0.f;
#pragma unroll
  for (int dx = 0; dx < 2; ++dx)
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
      for (int dz = 0; dz < 2; ++dz) {
        const float wgt = (dx ? a[0] : 1.f - a[0]) * (dy ? a[1] : 1.f - a[1]) * (dz ? a[2] : 1.f - a[2]);
        const int ix = (i0[0] + dx) % n, iy = (i0[1] + dy) % n, iz = (i0[2] + dz) % n;
        acc += wgt * f[((size_t)ix * n + iy) * n + iz];
      }
  out7[p * 7 + o] = acc;
}

}  // namespace ga
