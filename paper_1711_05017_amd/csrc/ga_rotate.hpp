// ga_rotate.hpp -- spectral rotation (Sec. 3.2, step 1) on gfx950.
//
// The moving part's resident spectra are interpolated trilinearly over the
// rotated frequency grid instead of re-splatting the rotated part:
// out_b(k) = X(R_b^T kappa(k)), kappa the signed frequency; with the 4
// channels (u and the moment densities of eq. 6b) the moment channels rotate
// as a vector. Two resident layouts: planar half spectra (one array per
// channel) and packed spectra (the 4 channels of a frequency in one 32-byte
// record, so that one corner read serves every channel).
#pragma once

#include <hip/hip_runtime.h>

#include "ga_kernels.hpp"

namespace ga {

// Position of signed integer frequency (a, b, c) in a half spectrum
// [N][N][N/2+1]: false beyond the band (|component| > N/2); mirror when the
// value is the conjugate of the stored one (X(-k) = conj X(k) for c < 0).
template <int N>
__device__ __forceinline__ bool locate_freq(int a, int b, int c, size_t& idx, bool& mirror) {
  constexpr int h = N / 2;
  if (a > h || a < -h || b > h || b < -h || c > h || c < -h) return false;
  mirror = c < 0;
  if (mirror) {
    a = -a;
    b = -b;
    c = -c;
  }
  a += (a < 0) ? N : 0;
  b += (b < 0) ? N : 0;
  idx = ((size_t)a * N + (size_t)b) * (h + 1) + c;
  return true;
}

__device__ __forceinline__ float2 conj_each(float2 v) { return make_float2(v.x, -v.y); }
__device__ __forceinline__ float4 conj_each(float4 v) { return make_float4(v.x, -v.y, v.z, -v.w); }
__device__ __forceinline__ void axpy(float w, float2 v, float2& acc) {
  acc.x += w * v.x;
  acc.y += w * v.y;
}
__device__ __forceinline__ void axpy(float w, float4 v, float4& acc) {
  acc.x += w * v.x;
  acc.y += w * v.y;
  acc.z += w * v.z;
  acc.w += w * v.w;
}
template <class V> __device__ __forceinline__ V zero_value();
template <> __device__ __forceinline__ float2 zero_value<float2>() { return make_float2(0.f, 0.f); }
template <> __device__ __forceinline__ float4 zero_value<float4>() { return make_float4(0.f, 0.f, 0.f, 0.f); }

using u32x4 = __attribute__((ext_vector_type(4))) unsigned;

// Byte offset that no source holds: a raw buffer load beyond the resource's
// size returns zeros (offsets + 16 stay below 2^32 and above every size).
constexpr unsigned kNoElem = 0xFFFFFF00u;

// Planar resident spectra: channel ph at X + ph * SPEC (nch = 1 or 4).
// load_at: element at byte offset off of channel ph (raw buffer load, zeros
// for kNoElem); load: element idx, conjugated when mirror.
template <int N>
struct PlanarSrc {
  using V = float2;
  // phases, bytes per element, threads of the LDS rotation kernel (measured:
  // 256 with 4 phases, 512 with the packed source's 2)
  static constexpr int MAX_PHASES = 4, REC = 8, THREADS = 256;
  static constexpr size_t SPEC = (size_t)N * N * (N / 2 + 1);
  const float2* X;
  int nch;
  __device__ int phases() const { return nch; }
  __device__ V load_at(int ph, unsigned off) const {
    const auto rs = buffer_rsrc(const_cast<float2*>(X + (size_t)ph * SPEC), (unsigned)(SPEC * sizeof(float2)));
    const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)off, 0, 0);
    return make_float2(__uint_as_float(v.x), __uint_as_float(v.y));
  }
  __device__ V load(int ph, size_t idx, bool mirror) const {
    const float2 v = X[(size_t)ph * SPEC + idx];
    return mirror ? conj_each(v) : v;
  }
  __device__ void put(float2* acc, int ph, V v) const { acc[ph] = v; }
};

// Packed resident spectra: record k = P[2k] = {u, yhat_x u}(k) and
// P[2k + 1] = {yhat_y u, yhat_z u}(k); phase ph reads channel pair ph.
template <int N>
struct PackedSrc {
  using V = float4;
  static constexpr int MAX_PHASES = 2, REC = 32, THREADS = 512;
  static constexpr size_t SPEC = (size_t)N * N * (N / 2 + 1);
  const float4* P;
  __device__ int phases() const { return 2; }
  __device__ V load_at(int ph, unsigned off) const {
    const auto rs = buffer_rsrc(const_cast<float4*>(P), (unsigned)(2 * SPEC * sizeof(float4)));
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, ph * 16, 0);
    return make_float4(__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z), __uint_as_float(v.w));
  }
  __device__ V load(int ph, size_t idx, bool mirror) const {
    const float4 v = P[2 * idx + ph];
    return mirror ? conj_each(v) : v;
  }
  __device__ void put(float2* acc, int ph, V v) const {
    acc[2 * ph] = make_float2(v.x, v.y);
    acc[2 * ph + 1] = make_float2(v.z, v.w);
  }
};

// Conjugate by sign bit: s = 0 or 0x80000000.
__device__ __forceinline__ float2 flip_imag(float2 v, unsigned s) {
  return make_float2(v.x, __uint_as_float(__float_as_uint(v.y) ^ s));
}
__device__ __forceinline__ float4 flip_imag(float4 v, unsigned s) {
  return make_float4(v.x, __uint_as_float(__float_as_uint(v.y) ^ s), v.z, __uint_as_float(__float_as_uint(v.w) ^ s));
}

// Value of phase ph of a source at signed frequency (a, b, c); zero beyond
// the band.
template <int N, class Src>
__device__ __forceinline__ typename Src::V src_at(const Src& s, int ph, int a, int b, int c) {
  size_t idx = 0;
  bool mirror = false;
  if (!locate_freq<N>(a, b, c, idx, mirror)) return zero_value<typename Src::V>();
  return s.load(ph, idx, mirror);
}

// Trilinear interpolation at q (corner indices i0 + {0, 1}, weights from the
// fractions a); at(ix, iy, iz) returns the value at a corner. Corners of
// weight 0 are not read.
template <class V, class At>
__device__ __forceinline__ V trilinear_at(const int* i0, const float* a, At at) {
  V acc = zero_value<V>();
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int dx = c >> 2, dy = (c >> 1) & 1, dz = c & 1;
    const float w = (dx ? a[0] : 1.f - a[0]) * (dy ? a[1] : 1.f - a[1]) * (dz ? a[2] : 1.f - a[2]);
    if (w == 0.f) continue;
    axpy(w, at(i0[0] + dx, i0[1] + dy, i0[2] + dz), acc);
  }
  return acc;
}

// q = R^T kappa in float64, split into the lower corner and the fractions.
__device__ __forceinline__ void rotate_frequency(const double* R, double k0, double k1, double k2, int* i0, float* a) {
  const double q[3] = {R[0] * k0 + R[3] * k1 + R[6] * k2, R[1] * k0 + R[4] * k1 + R[7] * k2,
                       R[2] * k0 + R[5] * k1 + R[8] * k2};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double f = floor(q[d]);
    a[d] = (float)(q[d] - f);
    i0[d] = (int)f;
  }
}

// The moment channels rotate as a vector: o[1 + a] = sum_b R[a][b] acc[1 + b]
// (R as float).
__device__ __forceinline__ void store_rotated(float2* o, size_t spec, int nch, const float* R, const float2* acc) {
  o[0] = acc[0];
  if (nch == 4) {
    for (int a = 0; a < 3; ++a) {
      const float ra = R[3 * a], rb = R[3 * a + 1], rc = R[3 * a + 2];
      o[(size_t)(1 + a) * spec] = make_float2(ra * acc[1].x + rb * acc[2].x + rc * acc[3].x,
                                              ra * acc[1].y + rb * acc[2].y + rc * acc[3].y);
    }
  }
}

// Tile of a workgroup under the XCD-aware order: workgroups are dealt to
// the 8 XCDs round-robin, so XCD x takes the x-th eighth of the tiles in
// order (kz tiles of one row back to back: the two halves of an output cache
// line are written through the same L2, and neighbouring tiles' input boxes
// overlap in it). A tail of tiles % 8 keeps the plain order.
__device__ __forceinline__ int xcd_tile(int bid, int tiles) {
  const int per = tiles >> 3;
  return (bid < (per << 3)) ? (bid & 7) * per + (bid >> 3) : bid;
}

// Spectral rotation, out: batch x nch half spectra (nch = 1, or 4 with the
// moment channels rotated as a vector). The signed frequency of index N/2 is
// -N/2 on every axis.
//
// A workgroup (Src::THREADS = 256 or 512 threads) owns an 8 x 8 x 8 tile of
// outputs, two or one per thread. Per rotation it bounds the tile's preimage
// R^T kappa (a rotated cube) by an integer box of at most BOX per axis. Each
// thread locates its box elements in the half spectrum once (element
// i = tid + THREADS k; rows
// along kz, so reads are contiguous); per phase (a channel, or a channel pair
// of the packed source) it loads them into registers with all loads in
// flight, moves them to LDS, issues the next phase's loads and interpolates
// from LDS while they are in flight. Weights and the LDS address of the
// lower corner are computed once per output; an output whose 2 x 2 x 2
// corners are not all in the box (a box cut at BOX, or rounding at its edge)
// reads them from global memory. Needs N/2 divisible by 8 (signed
// frequencies contiguous in every tile). grid = (tiles, min(batch, 65535)).
template <int N, class Src>
__global__ void __launch_bounds__(Src::THREADS) k_spectral_rotate(Src src, const float* __restrict__ Rm, int batch,
                                                                  float2* __restrict__ out) {
  using V = typename Src::V;
  constexpr int PH = Src::MAX_PHASES;
  constexpr int HN = N / 2 + 1, T = 8, NT = N / T, NTZ = (HN + T - 1) / T;
  // box edge cap: the preimage of a tile spans at most floor(7 sqrt(3)) + 3 =
  // 15 lattice planes per axis, 14 or fewer for most rotations
  constexpr int BOX = 14, BOXV = BOX * BOX * BOX, TH = Src::THREADS;
  constexpr int NV = (BOXV + TH - 1) / TH, J = 512 / TH;
  constexpr size_t SPEC = (size_t)N * N * HN;
  static_assert((N / 2) % T == 0, "tiles must not straddle the sign change of the frequencies");
  static_assert(2 * SPEC * sizeof(float4) < kNoElem, "record offsets below kNoElem");
  __shared__ V box[BOXV];
  const int t = xcd_tile(blockIdx.x, NT * NT * NTZ), tid = threadIdx.x;
  const int tz = t % NTZ, ty = (t / NTZ) % NT, tx = t / (NTZ * NT);
  auto signed_k = [](int k) { return k < N / 2 ? k : k - N; };
  // signed frequency range of the tile per axis (kz beyond HN does not exist)
  const int klo[3] = {signed_k(tx * T), signed_k(ty * T), signed_k(tz * T)};
  const int kz_last = min(tz * T + T - 1, HN - 1);
  const int khi[3] = {klo[0] + T - 1, klo[1] + T - 1, signed_k(tz * T) + (kz_last - tz * T)};
  int kk[J][3];
  bool valid[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int o = tid + TH * j;
    kk[j][0] = tx * T + (o >> 6);
    kk[j][1] = ty * T + ((o >> 3) & 7);
    kk[j][2] = tz * T + (o & 7);
    valid[j] = kk[j][2] < HN;
  }
  const int nph = src.phases();
  for (int b = blockIdx.y; b < batch; b += gridDim.y) {
    double R[9];
    float Rf[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      Rf[i] = Rm[(size_t)b * 9 + i];
      R[i] = (double)Rf[i];
    }
    // integer box [lo, lo + ext) per axis holding every corner (cut at BOX)
    int lo[3], ext[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      double qmin = 0.0, qmax = 0.0;
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        const double r = R[3 * e + d], u = r * klo[e], v = r * khi[e];
        qmin += fmin(u, v);
        qmax += fmax(u, v);
      }
      lo[d] = (int)floor(qmin);
      ext[d] = min((int)floor(qmax) + 2 - lo[d], BOX);
    }
    const int ez = ext[2], eyz = ext[1] * ext[2], etot = ext[0] * eyz;
    const float inv_ez = 1.0f / (float)ez, inv_ey = 1.0f / (float)ext[1];
    // this thread's box elements: byte offset of the record (kNoElem: none,
    // or beyond the band) and whether it is read conjugated (bit k of mir)
    unsigned voff[NV], mir = 0;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const int i = tid + TH * k;
      voff[k] = kNoElem;
      if (i < etot) {
        // i < 14^3 < 2^16: (i + 1/2) / e rounds down to the exact quotient
        const int r = (int)(((float)i + 0.5f) * inv_ez), iz = i - r * ez;
        const int ix = (int)(((float)r + 0.5f) * inv_ey), iy = r - ix * ext[1];
        size_t idx = 0;
        bool mirror = false;
        if (locate_freq<N>(lo[0] + ix, lo[1] + iy, lo[2] + iz, idx, mirror)) {
          voff[k] = (unsigned)idx * (unsigned)Src::REC;
          mir |= (mirror ? 1u : 0u) << k;
        }
      }
    }
    V cur[NV];
    auto load_phase = [&](int ph) {
#pragma unroll
      for (int k = 0; k < NV; ++k) cur[k] = flip_imag(src.load_at(ph, voff[k]), ((mir >> k) & 1u) << 31);
    };
    load_phase(0);
    // per output: corner weights, lower corner, its LDS address when the
    // whole 2 x 2 x 2 cube lies in the box (else -1)
    int i0[J][3], base[J];
    float w[J][8];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      float a[3];
      rotate_frequency(R, signed_k(kk[j][0]), signed_k(kk[j][1]), signed_k(kk[j][2]), i0[j], a);
#pragma unroll
      for (int c = 0; c < 8; ++c)
        w[j][c] = ((c & 4) ? a[0] : 1.f - a[0]) * ((c & 2) ? a[1] : 1.f - a[1]) * ((c & 1) ? a[2] : 1.f - a[2]);
      const int ux = i0[j][0] - lo[0], uy = i0[j][1] - lo[1], uz = i0[j][2] - lo[2];
      const bool inside = (unsigned)ux < (unsigned)(ext[0] - 1) && (unsigned)uy < (unsigned)(ext[1] - 1) &&
                          (unsigned)uz < (unsigned)(ez - 1);
      base[j] = inside ? ux * eyz + uy * ez + uz : -1;
    }
    const int offs[8] = {0, 1, ez, ez + 1, eyz, eyz + 1, eyz + ez, eyz + ez + 1};
    float2 acc[J][4];
#pragma unroll
    for (int ph = 0; ph < PH; ++ph) {
      if (ph >= nph) break;  // uniform
      __syncthreads();       // previous readers of the box are done
      // slots from etot on are not part of this box: written, never read
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        const int i = tid + TH * k;
        if (TH * (k + 1) <= BOXV || i < BOXV) box[i] = cur[k];
      }
      __syncthreads();
      if (ph + 1 < nph) load_phase(ph + 1);  // in flight during this phase's interpolation
#pragma unroll
      for (int j = 0; j < J; ++j) {
        if (!valid[j]) continue;
        V s = zero_value<V>();
        if (base[j] >= 0) {
#pragma unroll
          for (int c = 0; c < 8; ++c) axpy(w[j][c], box[base[j] + offs[c]], s);
        } else {
#pragma unroll
          for (int c = 0; c < 8; ++c)
            axpy(w[j][c], src_at<N>(src, ph, i0[j][0] + (c >> 2), i0[j][1] + ((c >> 1) & 1), i0[j][2] + (c & 1)), s);
        }
        src.put(acc[j], ph, s);
      }
    }
    const int nch = (PH == 2) ? 4 : nph;
#pragma unroll
    for (int j = 0; j < J; ++j) {
      if (!valid[j]) continue;
      const size_t r = ((size_t)kk[j][0] * N + kk[j][1]) * HN + kk[j][2];
      store_rotated(out + (size_t)b * nch * SPEC + r, SPEC, nch, Rf, acc[j]);
    }
  }
}

// The same rotation with every corner gathered from global memory: grid
// edges whose N/2 is not a multiple of 8. A workgroup takes 2 (kx) x 8 (ky) x
// 16 (kz) outputs. grid = (tiles, min(batch, 65535)).
template <int N, class Src>
__global__ void __launch_bounds__(256) k_spectral_rotate_gather(Src src, const float* __restrict__ Rm, int batch,
                                                                float2* __restrict__ out) {
  using V = typename Src::V;
  constexpr int PH = Src::MAX_PHASES;
  constexpr int HN = N / 2 + 1, TZ = 16, TY = 8;
  constexpr int NTZ = (HN + TZ - 1) / TZ, NTY = N / TY;
  constexpr size_t SPEC = (size_t)N * N * HN;
  const int t = blockIdx.x;
  const int kz = (t % NTZ) * TZ + (int)(threadIdx.x & 15);
  const int ky = ((t / NTZ) % NTY) * TY + (int)((threadIdx.x >> 4) & 7);
  const int kx = (t / (NTZ * NTY)) * 2 + (int)(threadIdx.x >> 7);
  if (kz >= HN) return;  // no barrier below
  const size_t r = ((size_t)kx * N + ky) * HN + kz;
  const double k0 = kx < N / 2 ? kx : kx - N, k1 = ky < N / 2 ? ky : ky - N, k2 = kz < N / 2 ? kz : kz - N;
  const int nph = src.phases(), nch = (PH == 2) ? 4 : nph;
  for (int b = blockIdx.y; b < batch; b += gridDim.y) {
    double R[9];
    float Rf[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      Rf[i] = Rm[(size_t)b * 9 + i];
      R[i] = (double)Rf[i];
    }
    int i0[3];
    float a[3];
    rotate_frequency(R, k0, k1, k2, i0, a);
    float2 acc[4];
#pragma unroll
    for (int ph = 0; ph < PH; ++ph) {
      if (ph >= nph) break;
      src.put(acc, ph, trilinear_at<V>(i0, a, [&](int x, int y, int z) { return src_at<N>(src, ph, x, y, z); }));
    }
    store_rotated(out + (size_t)b * nch * SPEC + r, SPEC, nch, Rf, acc);
  }
}

// Packed spectra from 4 planar half spectra: out[2e] = {in0, in1}(e),
// out[2e + 1] = {in2, in3}(e). grid-stride over the n^2 (n/2+1) frequencies.
__global__ void __launch_bounds__(256) k_pack4(const float2* __restrict__ in, float4* __restrict__ out, long long spec) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < spec; e += (long long)gridDim.x * blockDim.x) {
    const float2 a = in[e], b = in[spec + e], c = in[2 * spec + e], d = in[3 * spec + e];
    out[2 * e] = make_float4(a.x, a.y, b.x, b.y);
    out[2 * e + 1] = make_float4(c.x, c.y, d.x, d.y);
  }
}

}  // namespace ga
