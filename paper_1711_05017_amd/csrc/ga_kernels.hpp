// ga_kernels.hpp -- HIP kernels of the correlation path (gfx950).
//
// Data flow of one energy field (three HBM passes):
//   plane_fwd  per x-plane: splat (or load) the real plane into LDS, z R2C of
//              row pairs, y FFT of the columns, write the plane spectrum.
//   strip_*    per strip of G (ky, kz) columns: x FFT in LDS, fused with the
//              conjugate product (and the spectral-gradient multipliers) and
//              the inverse x FFT, or with the single-pose partial sum.
//   plane_inv  per x-plane: inverse y FFT, z C2R of row pairs, write reals.
// After the z R2C the kz = 0 and kz = n/2 columns are real, so their y
// transforms share one complex transform (two-for-one); every y phase then
// has n/2 transforms, the same as the z phase.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "ga_fft.hpp"

namespace ga {

constexpr float kTwoPi = 6.28318530717958647692f;

// LDS layout of one x-plane: region t (PAIR float2) belongs to rows 2t and
// 2t+1. Two layouts share each region:
//  * z transforms (the two real rows packed as one complex row of N values):
//    position p at t*PAIR + (p ^ ((p >> ZS) & ZM));
//  * spectrum rows (after the z pass, and for the y transforms): row 2t at
//    the region's start, row 2t+1 at offset H + D; column c < N/2 of row y at
//    c ^ g(y), g(y) = h((y >> GS) & 7) with h linear over GF(2) given by its
//    images H1, H2, H4 of 1, 2, 4; the Nyquist column N/2 is not permuted.
// 8-byte LDS reads are served per half-wave on 32 bank pairs (slot mod 32),
// writes per quarter-wave on 16 (slot mod 16); the padding and the XORs
// spread the access shapes of the transforms (lanes along consecutive
// positions, and along positions in steps of the first radix) over distinct
// bank pairs. The XOR terms depend either on bits that are the same for all
// lanes of an access or on bits that are fixed per lane, so addresses keep
// immediate offsets. Default: the dense layout.
template <int N> struct PlaneSwz {
  static constexpr int PAIR = 2 * (N / 2 + 1), D = 0, ZS = 0, ZM = 0, GS = 0, H1 = 0, H2 = 0, H4 = 0;
};
#define GA_PLANE_SWZ(NN, PR, DD, ZS_, ZM_, GS_, A1, A2, A4)                                               \
  template <> struct PlaneSwz<NN> {                                                                       \
    static constexpr int PAIR = PR, D = DD, ZS = ZS_, ZM = ZM_, GS = GS_, H1 = A1, H2 = A2, H4 = A4;     \
  };
GA_PLANE_SWZ(128, 136, 3, 3, 7, 3, 11, 4, 8)
#undef GA_PLANE_SWZ

// INV selects the layout of the inverse pass, which measured fastest with
// the dense layout (its LDS traffic is a smaller share of its time).
template <int N> struct PlaneDense {
  static constexpr int PAIR = 2 * (N / 2 + 1), D = 0, ZS = 0, ZM = 0, GS = 0, H1 = 0, H2 = 0, H4 = 0;
};
template <int N, bool INV = false> struct Plane {
  static constexpr int H = N / 2 + 1;    // half-spectrum length along z
  using Z = std::conditional_t<INV, PlaneDense<N>, PlaneSwz<N>>;
  static constexpr int PAIR = Z::PAIR;   // float2 per row-pair region
  static constexpr int ROW1 = H + Z::D;  // offset of the odd row in its region
  static constexpr int CS = N / 2;       // columns [0, CS) are permuted
  static constexpr int SIZE = (N / 2) * PAIR;  // float2 per plane in LDS
  static_assert(ROW1 + H <= PAIR && N <= PAIR && SIZE % 2 == 0, "plane regions");
  static_assert((Z::H1 | Z::H2 | Z::H4) < 16 && CS % 16 == 0 || (Z::H1 | Z::H2 | Z::H4) == 0, "column XOR");
  static_assert(Z::ZM < (1 << Z::ZS) || Z::ZM == 0, "z XOR must not read the bits it changes");
  __device__ __forceinline__ static int g(int y) {
    const int u = (y >> Z::GS) & 7;
    return ((u & 1) ? Z::H1 : 0) ^ ((u & 2) ? Z::H2 : 0) ^ ((u & 4) ? Z::H4 : 0);
  }
  // spectrum element (row y, column c in [0, H))
  static constexpr bool kXor = (Z::H1 | Z::H2 | Z::H4) != 0;
  __device__ __forceinline__ static int yc(int y, int c) {
    const int base = (PAIR == 2 * H && Z::D == 0) ? y * H : (y >> 1) * PAIR + (y & 1) * ROW1;
    if constexpr (!kXor) return base + c;
    else return base + (c < CS ? (c ^ g(y)) : CS);
  }
  // z-transform position p in [0, N) of region t
  __device__ __forceinline__ static int zs(int t, int p) { return t * PAIR + (p ^ ((p >> Z::ZS) & Z::ZM)); }
  static constexpr int L = lanes_per_fft<N>();
  static constexpr int TPW = ffts_per_wave<N>();
  // 192: 12 waves, one round of the 96 row-pair and column transforms (the
  // plane's 149 KB of LDS admits one workgroup per CU; its twiddles are read
  // from an LDS table so that 12 waves fit the register file). 64: 8 waves
  // (the splat's hits spread over more waves: pass 1 8% and a single query's
  // fused pass 28% faster than with 4). 96 keeps 4 (its inverse pass and
  // batched single-pose launches measured slower with 8).
  static constexpr int WAVES = (N == 192) ? 12 : (N == 128 || N == 64) ? 8 : 4;
  static constexpr int THREADS = 64 * WAVES;
  // waves per SIMD the register budget must allow: two 8-wave workgroups per
  // CU at n = 128 (the plane's LDS admits two)
  static constexpr int MINW = (N == 128) ? 4 : 1;
};

// Twiddles of the generic plane kernels: in registers, or (192) read from a
// table the workgroup copies to LDS (plane_twiddles).
template <int N> constexpr bool kPlaneTwTab = (N == 192);
template <int N> using PlaneTw = std::conditional_t<kPlaneTwTab<N>, TwiddlesTab<N>, Twiddles<N>>;
// Sets up the twiddles of transform lane `l`: registers from the table, or
// the LDS copy tab[N] (filled by the whole workgroup; the caller's next
// workgroup barrier orders it before the first transform).
template <int N>
__device__ __forceinline__ void plane_twiddles(PlaneTw<N>& tw, const float2* __restrict__ table, float2* tab, int l) {
  if constexpr (kPlaneTwTab<N>) {
    for (int i = threadIdx.x; i < N; i += blockDim.x) tab[i] = table[i];
    tw.tab = tab;
  } else {
    load_twiddles<N>(tw, table, l);
  }
}

constexpr int kChunk = 256;  // records examined per round; bounds the LDS hit list

// One sample after placement: y = R (x - c) split into an integer voxel base
// (mod n) and a float32 fraction in [0, 1).
struct Placed {
  float4 a;  // fx, fy, fz, rho
  int4 b;    // bx, by, bz, weight (float bits)
};

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
  // binned samples (from k_bin_samples), per batch member: records sorted by
  // bx with bin offsets off[b*(N+1) + i]; null -> scan all samples
  const Placed* rec;
  const int* off;
  const float* rmax;
  // per batch member and plane x: cand[b*N + x] = (lo1, n1, lo2, n2), the
  // records whose x bin lies within reach of plane x (two runs when the range
  // wraps around the torus); null where the kernels do not use it
  const int4* cand;
  // per batch member, kPlaneMaskWords<N> words: bit x set when plane x of
  // the member's spectrum was written. With it, pass 1 stores no plane that
  // no sample reaches (its spectrum is zero) and readers of the spectra
  // treat unset planes as zero. Cleared by the binning kernel; null: every
  // plane is stored.
  unsigned* pmask;
};

template <int N>
constexpr int kPlaneMaskWords = (N + 31) / 32;

// A sample that reaches the current plane, with the bounding square of its
// disk in the plane: rows ylo .. ylo + sy - 1, columns zlo .. zlo + sz - 1
// (offsets from the voxel base), cnt = sy * sz voxels.
struct Hit {
  float4 a;  // dx^2, fy, fz, w
  int4 b;    // by | bz << 16, (ylo & 0xffff) | zlo << 16, sz, 1/(2 s^2) as float bits
};

// LDS state of the splat of one plane: hit list and the running voxel
// offset of each hit (hstart[i] = sum of cnt over hits before i).
struct HitList {
  Hit hits[kChunk];
  int hstart[kChunk + 1];
  int nhits;
};

// Raw buffer stores of float2: the address is the resource's base plus a
// per-lane byte offset (VGPR) and a uniform byte offset (SGPR, here a
// compile-time constant), so a run of stores at fixed distances costs no
// vector address arithmetic. Stores at or beyond `bytes` are dropped.
using u32x2 = __attribute__((ext_vector_type(2))) unsigned;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(void* base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(base, 0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ void buffer_store2(float2 v, __amdgpu_buffer_rsrc_t rs, int lane_bytes, int const_bytes) {
  const u32x2 d = {__float_as_uint(v.x), __float_as_uint(v.y)};
  __builtin_amdgcn_raw_buffer_store_b64(d, rs, lane_bytes, const_bytes, 0);
}

__device__ __forceinline__ int wrapn(int v, int n) {
  v = (v < 0) ? v + n : v;
  return (v >= n) ? v - n : v;
}
__device__ __forceinline__ float yhat(int q, int n) { return (float)((q < n / 2) ? q : q - n); }

// kappa(k)/N for a half-spectrum index: k for k < N/2, k - N above, 0 at N/2.
template <int N>
__device__ __forceinline__ float omega_of(int k) {
  return (k == N / 2) ? 0.f : (float)((k < N / 2) ? k : k - N) / (float)N;
}

__device__ __forceinline__ void load_rotation(const SplatParams& p, int b, double* R) {
  if (p.Rdev) {
#pragma unroll
    for (int i = 0; i < 9; ++i) R[i] = (double)p.Rdev[b * 9 + i];
  } else {
#pragma unroll
    for (int i = 0; i < 9; ++i) R[i] = (double)p.Rh[i];
  }
}

// Placement of sample s in float64. Returns false for a sample that is not
// finite or whose radius reaches n/2 (it contributes nothing).
template <int N>
__device__ __forceinline__ bool place_sample(const SplatParams& p, const double* R, long long s, Placed& out) {
  const float4 q = p.xyzr[s];
  const float w = p.w[s];
  const float rho = fmaxf(q.w, 1.0f);
  if (!(rho < 0.5f * N) || !isfinite(w)) return false;
  const double dx0 = (double)q.x - (double)p.c[0];
  const double dy0 = (double)q.y - (double)p.c[1];
  const double dz0 = (double)q.z - (double)p.c[2];
  const double yx = R[0] * dx0 + R[1] * dy0 + R[2] * dz0;
  const double yy = R[3] * dx0 + R[4] * dy0 + R[5] * dz0;
  const double yz = R[6] * dx0 + R[7] * dy0 + R[8] * dz0;
  if (!(fabs(yx) < 1.0e7 && fabs(yy) < 1.0e7 && fabs(yz) < 1.0e7)) return false;
  const double fbx = floor(yx), fby = floor(yy), fbz = floor(yz);
  long long ix = (long long)fbx % N, iy = (long long)fby % N, iz = (long long)fbz % N;
  out.a = make_float4((float)(yx - fbx), (float)(yy - fby), (float)(yz - fbz), rho);
  out.b = make_int4((int)(ix < 0 ? ix + N : ix), (int)(iy < 0 ? iy + N : iy), (int)(iz < 0 ? iz + N : iz),
                    __float_as_int(w));
  return true;
}

// Places every sample of one part once and counting-sorts the records by
// bx: records rb[0 .. count), bin offsets ob[0 .. N] (ob[N] = count), largest
// radius *rm. One workgroup (any size of at least 64 threads).
template <int N>
__device__ void bin_block(const SplatParams& p, const double* R, Placed* __restrict__ rb, int* __restrict__ ob,
                          float* __restrict__ rm, int4* __restrict__ cand) {
  __shared__ int cnt[N];
  __shared__ int cur[N];
  __shared__ int s_rmax;
  __shared__ int s_total;
  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += (int)blockDim.x) cnt[i] = 0;
  if (tid == 0) s_rmax = __float_as_int(1.0f);
  __syncthreads();
  for (long long s = tid; s < p.n_pts; s += blockDim.x) {
    Placed q;
    if (place_sample<N>(p, R, s, q)) {
      atomicAdd(&cnt[q.b.x], 1);
      atomicMax(&s_rmax, __float_as_int(q.a.w));  // positive floats order like their bits
    }
  }
  __syncthreads();
  if (tid < 64) {
    // exclusive scan of the N bin counts by one wave, 64 bins per step
    int carry = 0;
    for (int base = 0; base < N; base += 64) {
      const int i = base + tid;
      const int v = (i < N) ? cnt[i] : 0;
      int incl = v;
      for (int d = 1; d < 64; d <<= 1) {
        const int o = __shfl_up(incl, d, 64);
        if (tid >= d) incl += o;
      }
      if (i < N) {
        cur[i] = carry + incl - v;
        ob[i] = carry + incl - v;
      }
      carry += __shfl(incl, 63, 64);
    }
    if (tid == 0) {
      ob[N] = carry;
      s_total = carry;
      *rm = __int_as_float(s_rmax);
    }
  }
  __syncthreads();
  if (cand) {
    // candidate runs per plane: bins x - reach .. x + reach (mod N), read
    // from the exclusive scan in cur[] before the scatter below advances it
    const int reach = (int)ceilf(__int_as_float(s_rmax)) + 1;
    const int total = s_total;
    for (int x = tid; x < N; x += (int)blockDim.x) {
      int4 r = make_int4(0, total, 0, 0);
      if (2 * reach + 1 < N) {
        const int blo = x - reach, bhi = x + reach;  // inclusive, mod N
        if (blo < 0) r = make_int4(cur[blo + N], total - cur[blo + N], 0, cur[bhi + 1]);
        else if (bhi >= N) r = make_int4(cur[blo], total - cur[blo], 0, (bhi + 1 - N < N) ? cur[bhi + 1 - N] : total);
        else r = make_int4(cur[blo], ((bhi + 1 < N) ? cur[bhi + 1] : total) - cur[blo], 0, 0);
      }
      cand[x] = r;
    }
    __syncthreads();
  }
  for (long long s = tid; s < p.n_pts; s += blockDim.x) {
    Placed q;
    if (place_sample<N>(p, R, s, q)) rb[atomicAdd(&cur[q.b.x], 1)] = q;
  }
}

// Per batch member b: the moving part rotated by R_b, binned into
// rec[b*n_pts ...], off[b*(N+1) ...], rmax[b]; the member's plane mask
// (p.pmask, if set) cleared for pass 1. grid = batch, block = 1024.
template <int N>
__global__ void __launch_bounds__(1024) k_bin_samples(SplatParams p, Placed* __restrict__ rec, int* __restrict__ off,
                                                     float* __restrict__ rmax, int4* __restrict__ cand) {
  const int b = blockIdx.x;
  if (p.pmask && (int)threadIdx.x < kPlaneMaskWords<N>) p.pmask[(size_t)b * kPlaneMaskWords<N> + threadIdx.x] = 0u;
  double R[9];
  load_rotation(p, b, R);
  bin_block<N>(p, R, rec + (size_t)b * p.n_pts, off + (size_t)b * (N + 1), rmax + b,
               cand ? cand + (size_t)b * N : nullptr);
}

// One query of the serving loop: a registered pair (its moving part's
// samples and the resident stationary spectrum), a rotation about c and a
// lattice translation (already reduced mod N).
struct QueryItem {
  const float4* xyzr;
  const float* w;
  long long n_pts;
  const float2* AX;  // spectral queries: the stationary spectrum and its x derivative, x inverse-transformed (2 x 8H)
  const float4* FA;  // local queries: (u_A, grad u_A) per voxel
  float R[9];
  float c[3];
  int t[3];
  int pad;  // 1: the translation was not finite or too large (outputs NaN)
};

// Binning of heterogeneous queries: item b's samples, placed with its own
// rotation, into rec[b*stride ...]. grid = batch, block = 1024 (a serving
// launch has few queries: the block's width sets its latency).
template <int N>
__global__ void __launch_bounds__(1024) k_bin_items(const QueryItem* __restrict__ items, SplatParams base,
                                                   long long stride, Placed* __restrict__ rec, int* __restrict__ off,
                                                   float* __restrict__ rmax, int4* __restrict__ cand) {
  const int b = blockIdx.x;
  const QueryItem& it = items[b];
  SplatParams p = base;
  p.xyzr = it.xyzr;
  p.w = it.w;
  p.n_pts = it.n_pts;
  p.c[0] = it.c[0];
  p.c[1] = it.c[1];
  p.c[2] = it.c[2];
  double R[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) R[i] = (double)it.R[i];
  bin_block<N>(p, R, rec + (size_t)b * stride, off + (size_t)b * (N + 1), rmax + b,
               cand ? cand + (size_t)b * N : nullptr);
}

// Candidate hit test of one placed sample against plane x; appends it and
// its disk's voxel count to the LDS hit list.
template <int N>
__device__ __forceinline__ void test_hit(const SplatParams& p, const Placed& q, int x, HitList& hl) {
  int m = x - q.b.x;
  m = (m >= N / 2) ? m - N : m;
  m = (m < -N / 2) ? m + N : m;
  float dx = (float)m - q.a.x;
  dx = (dx < -0.5f * N) ? dx + (float)N : dx;
  const float w = __int_as_float(q.b.w);
  const float rho = q.a.w;
  if (!(fabsf(dx) < rho) || w == 0.0f) return;
  const float rd = sqrtf(fmaxf(rho * rho - dx * dx, 0.0f));
  const float fy = q.a.y, fz = q.a.z;
  const int ylo = (int)ceilf(fy - rd), yhi = (int)floorf(fy + rd);
  const int zlo = (int)ceilf(fz - rd), zhi = (int)floorf(fz + rd);
  const int sy = yhi - ylo + 1, sz = zhi - zlo + 1;
  if (sy <= 0 || sz <= 0) return;
  const int slot = atomicAdd(&hl.nhits, 1);
  Hit h;
  h.a = make_float4(dx * dx, fy, fz, w);
  h.b = make_int4(q.b.y | (q.b.z << 16), (ylo & 0xffff) | (zlo << 16), sz, __float_as_int(p.sig_c / (rho * rho)));
  hl.hits[slot] = h;
  hl.hstart[slot] = sy * sz;  // count for now; turned into offsets by hits_scan
}

// Exclusive scan of the hit counts in place (one wave), hstart[nh] = total.
__device__ __forceinline__ void hits_scan(HitList& hl) {
  const int tid = threadIdx.x;
  const int nh = hl.nhits;
  if (tid < 64) {
    int carry = 0;
    for (int base = 0; base < nh; base += 64) {
      const int i = base + tid;
      const int v = (i < nh) ? hl.hstart[i] : 0;
      int incl = v;
      for (int d = 1; d < 64; d <<= 1) {
        const int o = __shfl_up(incl, d, 64);
        if (tid >= d) incl += o;
      }
      if (i < nh) hl.hstart[i] = carry + incl - v;
      carry += __shfl(incl, 63, 64);
    }
    if (tid == 0) hl.hstart[nh] = carry;
  }
}

// Splat the hits into the LDS real plane Wf (voxel (y, z) at Wf[idx(y, z)]),
// each value multiplied by yhat_y (chan 2) or yhat_z (chan 3). The
// (hit, voxel) pairs are flattened and each wave takes a contiguous range of
// them, 64 at a time, so lanes are not left idle by small disks.
template <int N, int WAVES, class Idx>
__device__ __forceinline__ void splat_hits(const SplatParams& p, int chan, float* Wf, const HitList& hl, Idx idx) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nh = hl.nhits;
  if (nh == 0) return;
  const int V = hl.hstart[nh];
  const int per = (((V + WAVES - 1) / WAVES) + 63) & ~63;
  const int g0 = wave * per, g1 = min(V, g0 + per);
  if (g0 >= g1) return;
  int lo = 0, hi = nh - 1;  // last hit whose range starts at or before g0
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (hl.hstart[mid] <= g0) lo = mid;
    else hi = mid - 1;
  }
  int h = lo;
  for (int gb = g0; gb < g1; gb += 64) {
    const int g = gb + lane;
    if (g < g1) {
      while (hl.hstart[h + 1] <= g) ++h;
      const Hit q = hl.hits[h];
      const int v = g - hl.hstart[h];
      const int sz = q.b.z;
      // v / sz for v < 2^16: the quotient of (v + 1/2)/sz is at least
      // 1/(2 sz) away from an integer, far above the reciprocal's error
      const int qy = (int)(((float)v + 0.5f) * __builtin_amdgcn_rcpf((float)sz));
      const int oy = (int)(short)(q.b.y & 0xffff) + qy;
      const int oz = (q.b.y >> 16) + (v - qy * sz);
      const float ddy = (float)oy - q.a.y, ddz = (float)oz - q.a.z;
      const float e = (q.a.x + ddy * ddy + ddz * ddz) * __int_as_float(q.b.w);  // d^2 / (2 s^2)
      if (e < p.sig_c) {  // d < rho
        const int yy = wrapn((q.b.x & 0xffff) + oy, N), zz = wrapn((q.b.x >> 16) + oz, N);
        float val = q.a.w * (__expf(-e) - p.e0) * p.inv1me0;
        if (chan == 2) val *= yhat(yy, N);
        if (chan == 3) val *= yhat(zz, N);
        atomicAdd(&Wf[idx(yy, zz)], val);
      }
    }
  }
}

// Splat every sample that reaches plane x into Wf. With binned records only
// the bins within reach of x are examined; otherwise all samples are placed.
template <int N, int WAVES, int THREADS, class Idx>
__device__ void splat_plane(const SplatParams& p, const double* R, int b, int x, int chan, float* Wf, HitList& hl,
                            Idx idx) {
  const int tid = threadIdx.x;
  long long lo1 = 0, n1 = p.n_pts, lo2 = 0, n2 = 0;
  const Placed* rb = nullptr;
  if (p.rec) {
    const int* ob = p.off + (size_t)b * (N + 1);
    rb = p.rec + (size_t)b * p.n_pts;
    const int reach = (int)ceilf(p.rmax[b]) + 1;
    if (2 * reach + 1 >= N) {
      lo1 = 0;
      n1 = ob[N];
    } else {
      const int blo = x - reach, bhi = x + reach;  // inclusive bin range, mod N
      if (blo < 0) {
        lo1 = ob[blo + N];
        n1 = ob[N] - lo1;
        lo2 = 0;
        n2 = ob[bhi + 1];
      } else if (bhi >= N) {
        lo1 = ob[blo];
        n1 = ob[N] - lo1;
        lo2 = 0;
        n2 = ob[bhi + 1 - N];
      } else {
        lo1 = ob[blo];
        n1 = ob[bhi + 1] - lo1;
      }
    }
  }
  const long long total = n1 + n2;
  for (long long c0 = 0; c0 < total; c0 += kChunk) {
    if (tid == 0) hl.nhits = 0;
    __syncthreads();
    const long long i = c0 + tid;
    if (tid < kChunk && i < total) {
      Placed q;
      bool ok = true;
      if (rb) q = rb[(i < n1) ? lo1 + i : lo2 + (i - n1)];
      else ok = place_sample<N>(p, R, i, q);
      if (ok) test_hit<N>(p, q, x, hl);
    }
    __syncthreads();
    hits_scan(hl);
    __syncthreads();
    splat_hits<N, WAVES>(p, chan, Wf, hl, idx);
    __syncthreads();
  }
}

// z R2C of every row pair and y FFT of every column of the LDS plane W, the
// plane's 2D spectrum [ky][kz] (row stride H) written to global memory: to
// dst0, and scaled by s1 to dst1 unless dst1 is null. On entry W holds the
// pair-packed real plane (rows 2t, 2t+1 as the real and imaginary parts of
// region t). The y transforms' last stage stores each output straight to
// global memory (a wavefront's store covers 8 rows x 8 consecutive kz); the
// real columns kz = 0 and kz = N/2, transformed together, are split in LDS
// and written after. DIRECT = false: the spectrum stays in W (layout
// yc) and dst0, dst1 are not used; the caller copies it out (edges whose
// transforms leave no registers for the direct stores).
template <int N, bool DIRECT, class TW>
__device__ __forceinline__ void plane_forward_out(float2* W, const TW& tw, float2* __restrict__ dst0,
                                                  float2* __restrict__ dst1, float s1) {
  using P = Plane<N>;
  constexpr int L = P::L, TPW = P::TPW, H = P::H;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l = lane % L;
  // z: one complex FFT per pair of real rows, then split into the two halves
  for (int it = 0; it * P::WAVES * TPW < N / 2; ++it) {
    const int t = (it * P::WAVES + wave) * TPW + lane / L;
    if (t < N / 2) {
      auto reg = [=](int pos) { return W + P::zs(t, pos); };
      fft_inplace_at<N, -1>(l, tw, reg);
      // A(k) = (Z(k) + conj Z(N-k))/2 and B(k) = (Z(k) - conj Z(N-k))/(2i) are
      // the spectra of rows 2t and 2t+1; every lane reads its Z values before
      // any lane writes the rows (same region, other layout).
      constexpr int KPL = (H + L - 1) / L;
      float2 ak[KPL], bk[KPL];
#pragma unroll
      for (int e = 0; e < KPL; ++e) {
        const int k = l + L * e;
        if (k < H) {
          const float2 a = *reg(k % N);
          const float2 z = *reg((N - k) % N);
          ak[e] = make_float2(0.5f * (a.x + z.x), 0.5f * (a.y - z.y));
          bk[e] = make_float2(0.5f * (a.y + z.y), -0.5f * (a.x - z.x));
        }
      }
      wave_sync();
#pragma unroll
      for (int e = 0; e < KPL; ++e) {
        const int k = l + L * e;
        if (k < H) {
          W[P::yc(2 * t, k)] = ak[e];
          W[P::yc(2 * t + 1, k)] = bk[e];
        }
      }
      wave_sync();
    }
  }
  __syncthreads();
  // Column 0 carries the real columns kz = 0 (real part) and kz = N/2
  // (imaginary part) through one y transform. It is packed here, one thread
  // per row (each touches only its own row's slots), and split after all y
  // transforms, so that no wavefront runs the packed column's loads and its
  // split beside a plain column under its execution mask.
  static_assert(P::THREADS >= N, "one thread per row of column 0");
  if (tid < N) W[P::yc(tid, 0)].y = W[P::yc(tid, N / 2)].x;
  __syncthreads();
  // y: columns 0 .. N/2-1 in place
  for (int it = 0; it * P::WAVES * TPW < N / 2; ++it) {
    const int t = (it * P::WAVES + wave) * TPW + lane / L;
    if (t < N / 2) {
      auto col = [=](int pos) { return W + P::yc(pos, t); };
      auto ld = [&](int pos) -> float2 { return *col(pos); };
      auto st = [&](int pos, float2 v) {
        if (!DIRECT || t == 0) {
          *col(pos) = v;
          return;
        }
        dst0[(size_t)pos * H + t] = v;
        if (dst1) dst1[(size_t)pos * H + t] = make_float2(v.x * s1, v.y * s1);
      };
      fft_at<N, -1>(l, tw, col, ld, st);
    }
  }
  __syncthreads();
  // C = A + i B with A, B the spectra of the real columns kz = 0 and kz = N/2:
  // B(k) = (C(k) - conj C(N-k))/(2i), A(k) = C(k) - i B(k), one thread per k
  float2 a = make_float2(0.f, 0.f), bb = a;
  if (tid < N) {
    const int k = tid;
    const float2 c = W[P::yc(k, 0)];
    const float2 z = W[P::yc((N - k) % N, 0)];
    bb = make_float2(0.5f * (c.y + z.y), -0.5f * (c.x - z.x));
    a = make_float2(c.x + bb.y, c.y - bb.x);
    if constexpr (DIRECT) {
      dst0[(size_t)k * H] = a;
      dst0[(size_t)k * H + N / 2] = bb;
      if (dst1) {
        dst1[(size_t)k * H] = make_float2(a.x * s1, a.y * s1);
        dst1[(size_t)k * H + N / 2] = make_float2(bb.x * s1, bb.y * s1);
      }
    }
  }
  if constexpr (!DIRECT) {
    __syncthreads();  // every C(N-k) is read before column 0 is overwritten
    if (tid < N) {
      W[P::yc(tid, 0)] = a;
      W[P::yc(tid, N / 2)] = bb;
    }
  }
  __syncthreads();
}

// Copy of COUNT items by THREADS threads that issues up to 16 loads per
// thread before the first store, so one workgroup waits for one memory
// latency per 16 items instead of one per item.
template <int COUNT, int THREADS, class T, class Ld, class St>
__device__ __forceinline__ void batched_copy(Ld ld, St st) {
  constexpr int IT = (COUNT + THREADS - 1) / THREADS;
  constexpr int B = IT < 16 ? IT : 16;
#pragma unroll 1
  for (int it0 = 0; it0 < IT; it0 += B) {
    T v[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int i = threadIdx.x + (it0 + u) * THREADS;
      if ((COUNT % THREADS == 0 && IT % B == 0) || i < COUNT) v[u] = ld(i);
    }
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int i = threadIdx.x + (it0 + u) * THREADS;
      if ((COUNT % THREADS == 0 && IT % B == 0) || i < COUNT) st(i, v[u]);
    }
  }
}

// The plane's spectrum between LDS (layout of Plane<N>) and global memory
// (dense [ky][kz], row stride H), times `scale` on the way out. Two complex
// values per global access (N*H is even); up to 16 loads per thread are in
// flight before the first store.
template <int N>
__device__ __forceinline__ void plane_to_global(float2* __restrict__ dst, const float2* W, float scale) {
  using P = Plane<N>;
  constexpr int H = P::H;
  float4* d4 = reinterpret_cast<float4*>(dst);
  batched_copy<N * H / 2, P::THREADS, float4>(
      [&](int i) {
        const int e = 2 * i, y0 = e / H, c0 = e - y0 * H;
        const int y1 = (c0 + 1 == H) ? y0 + 1 : y0, c1 = (c0 + 1 == H) ? 0 : c0 + 1;
        const float2 a = W[P::yc(y0, c0)], b = W[P::yc(y1, c1)];
        return make_float4(a.x * scale, a.y * scale, b.x * scale, b.y * scale);
      },
      [&](int i, float4 v) { d4[i] = v; });
}
template <int N>
__device__ __forceinline__ void plane_from_global(float2* W, const float2* __restrict__ src) {
  using P = Plane<N, true>;
  constexpr int H = P::H;
  const float4* s4 = reinterpret_cast<const float4*>(src);
  if constexpr (P::PAIR == 2 * H && P::Z::D == 0 && !P::kXor) {
    // dense layout: element e at slot e
    float4* W4 = reinterpret_cast<float4*>(W);
    batched_copy<N * H / 2, P::THREADS, float4>([&](int i) { return s4[i]; }, [&](int i, float4 v) { W4[i] = v; });
    return;
  }
  batched_copy<N * H / 2, P::THREADS, float4>([&](int i) { return s4[i]; }, [&](int i, float4 v) {
    const int e = 2 * i, y0 = e / H, c0 = e - y0 * H;
    const int y1 = (c0 + 1 == H) ? y0 + 1 : y0, c1 = (c0 + 1 == H) ? 0 : c0 + 1;
    W[P::yc(y0, c0)] = make_float2(v.x, v.y);
    W[P::yc(y1, c1)] = make_float2(v.z, v.w);
  });
}

// One hit of the per-wave splat below: the bounding square of the sample's
// disk in the plane, rows ybase .. ybase + sy - 1 and columns zbase ..
// zbase + sz - 1 (voxel indices, not yet reduced mod N), the offsets of its
// first row and column from the disk centre, dx^2 and 1/(2 s^2).
struct WaveHit {
  int ybase, zbase, syz;  // syz = sy | sz << 16
  float offy, offz, dx2, c2s, w;
};

// Candidate c of the plane's candidate runs rg (false beyond them).
__device__ __forceinline__ bool wave_cand(const Placed* rb, int4 rg, int c, Placed& q) {
  if (c >= rg.y + rg.w) return false;
  q = rb[c < rg.y ? rg.x + c : rg.z + (c - rg.y)];
  return true;
}

// Hit test of a candidate against plane x: false for a sample that misses
// the plane.
template <int N>
__device__ __forceinline__ bool wave_hit(const SplatParams& p, const Placed& q, int x, WaveHit& h) {
  int m = x - q.b.x;
  m = (m >= N / 2) ? m - N : m;
  m = (m < -N / 2) ? m + N : m;
  float dx = (float)m - q.a.x;
  dx = (dx < -0.5f * N) ? dx + (float)N : dx;
  h.w = __int_as_float(q.b.w);
  const float rho = q.a.w;
  if (!(fabsf(dx) < rho) || h.w == 0.0f) return false;
  // disk radius from the hardware square root (within an ulp), widened by
  // 2^-20 so that the square never misses a voxel of the disk: voxels it
  // adds fail the d < rho test of the splat
  const float rd = __builtin_amdgcn_sqrtf(fmaxf(rho * rho - dx * dx, 0.0f)) * (1.0f + 0x1p-20f);
  const int ylo = (int)ceilf(q.a.y - rd), yhi = (int)floorf(q.a.y + rd);
  const int zlo = (int)ceilf(q.a.z - rd), zhi = (int)floorf(q.a.z + rd);
  const int sy = yhi - ylo + 1, sz = zhi - zlo + 1;
  if (sy <= 0 || sz <= 0) return false;
  h.ybase = q.b.y + ylo;
  h.zbase = q.b.z + zlo;
  h.syz = sy | (sz << 16);
  h.offy = (float)ylo - q.a.y;
  h.offz = (float)zlo - q.a.z;
  h.dx2 = dx * dx;
  h.c2s = p.sig_c * __builtin_amdgcn_rcpf(rho * rho);  // within an ulp or so: moves K(d) by ~1e-7 at most
  return true;
}

template <int N>
__device__ __forceinline__ int wrap_axis(int v) {  // v in [-N, 2N)
  if constexpr ((N & (N - 1)) == 0) return v & (N - 1);
  else return wrapn(v, N);
}

// Number of set bits of m below this lane.
__device__ __forceinline__ int lanes_below(unsigned long long m) {
  return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// Inclusive prefix sum over the 64 lanes of a wavefront (all lanes active):
// within each row of 16 lanes by DPP row shifts (lanes shifted in from
// outside the row read 0), then the totals of the rows below added.
__device__ __forceinline__ int wave_incl_scan(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, true);  // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, true);  // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, true);  // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, true);  // row_shr:8
  const int t0 = __builtin_amdgcn_readlane(v, 15), t1 = __builtin_amdgcn_readlane(v, 31);
  const int t2 = __builtin_amdgcn_readlane(v, 47);
  const int row = (int)(threadIdx.x & 63) >> 4;
  return v + (row >= 1 ? t0 : 0) + (row >= 2 ? t1 : 0) + (row >= 3 ? t2 : 0);
}

// The splat sums in LDS are fixed point: LDS float atomics complete at a
// small fraction of the rate of integer ones on this hardware, so each value
// is scaled by a power of two S, rounded to an integer and added with an
// integer atomic (exact and order-independent), and the plane is converted
// back (times 1/S) before its transforms. S comes from a bound on the
// magnitude of any voxel's sum in the plane: each sample adds at most |w|
// (times |yhat| <= N/2 for the channel multipliers) to a voxel, and a plane
// receives only its candidates, so sum |w| over the candidates bounds it.
// With bound * S < 2^30 no sum overflows and each add is rounded to
// bound * 2^-30 at most, a relative error of the order of float32's for the
// sums of a plane.
struct PlaneBound {
  float wsum;  // sum of |w| over the plane's candidates
  bool any;    // some candidate of the first round hits the plane
};

// All threads of the workgroup: w0 = |w| of this thread's first-round
// candidate (0 if none), hit = its hit flag; candidates beyond the first
// round (64 WAVES) are read here. red: 2 WAVES floats of LDS. Ends with a
// workgroup barrier.
template <int WAVES, int THREADS>
__device__ __forceinline__ PlaneBound plane_bound(const Placed* rb, int4 rg, int ncand, float w0, bool hit,
                                                  float* red) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  float sum = w0;
  for (int c = 64 * WAVES + tid; c < ncand; c += THREADS)
    sum += fabsf(__int_as_float(rb[c < rg.y ? rg.x + c : rg.z + (c - rg.y)].b.w));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
  const bool wany = __ballot(hit) != 0;
  if (lane == 0) {
    red[wave] = sum;
    red[WAVES + wave] = wany ? 1.f : 0.f;
  }
  __syncthreads();
  PlaneBound r{0.f, false};
#pragma unroll
  for (int i = 0; i < WAVES; ++i) {
    r.wsum += red[i];
    r.any = r.any || red[WAVES + i] != 0.f;
  }
  return r;
}

// Power of two S with bound * S < 2^30 (bound >= 0; exponent clamped).
__device__ __forceinline__ float splat_scale(float bound) {
  int e = (bound > 0.f) ? __builtin_amdgcn_frexp_expf(bound) - 1 : 0;  // floor(log2 bound)
  e = min(max(e, -96), 96);
  return ldexpf(1.0f, 29 - e);
}

// Integer sums of a plane back to float: n4 int4 of W, times inv_s, each
// element by the thread that reads it (no barrier inside).
template <int THREADS>
__device__ __forceinline__ void plane_fix_to_float(float2* W, int n4, float inv_s) {
  float4* W4 = reinterpret_cast<float4*>(W);
  const int4* I4 = reinterpret_cast<const int4*>(W);
  for (int i = threadIdx.x; i < n4; i += THREADS) {
    const int4 v = I4[i];
    W4[i] = make_float4((float)v.x * inv_s, (float)v.y * inv_s, (float)v.z * inv_s, (float)v.w * inv_s);
  }
}

// Hits one wavefront splats at a time, by plane edge (LDS per wave:
// 32 bytes a hit and 64 bytes of start flags).
template <int N>
constexpr int kSplatCap = (N > 128) ? 16 : 32;

// Per-wavefront LDS of the splat below: a batch of hits, compacted, and one
// flag byte per lane marking where a hit's first row falls.
template <int CAP>
struct WaveSplatLds {
  int4 hi[CAP];    // (ybase | zbase << 16, sz | first row << 8, offy bits, offz bits)
  float4 hf[CAP];  // (dx^2, 1/(2 s^2), S w / (1 - e0), unused)
  int flag[16];
};

// Splat of the hits one wavefront found (flag `hit`, parameters `h` in each
// lane), adding w K(d) (times yhat_y or yhat_z for channel 2 or 3) in fixed
// point, times S (splat_scale), with LDS integer atomics at Wf[idx(y, z)]. The rows of the hits' bounding squares are
// enumerated as one sequence (hit by hit in lane order) and each lane takes
// one row, 64 consecutive rows per step, walking the row's sz voxels: a
// small disk does not leave lanes idle as a one-hit-per-step layout would.
// A batch of up to CAP hits is compacted into the wave's LDS with the index
// of its first row (a prefix sum over the wave); each step flags the lanes
// at which a hit's rows start, and the hit of a lane is the number of starts
// at or below it (a ballot and a masked bit count) plus those of earlier
// steps. No search and no workgroup barrier is involved.
template <int N, int CAP, class Idx>
__device__ __forceinline__ void wave_splat(const SplatParams& p, bool hit, const WaveHit& h, int chan, float S,
                                           float* Wf, Idx idx, WaveSplatLds<CAP>& ws) {
  static_assert(N < 256 && CAP * N < (1 << 23), "packed square sizes and starts");
  const int lane = threadIdx.x & 63;
  const unsigned long long hm = __ballot(hit);
  const int nh = __popcll(hm);  // uniform
  const int rank = lanes_below(hm);
  const int sy = h.syz & 0xffff, sz = h.syz >> 16;
  unsigned char* flag8 = reinterpret_cast<unsigned char*>(ws.flag);
  for (int r0 = 0; r0 < nh; r0 += CAP) {
    const bool mine = hit && rank >= r0 && rank < r0 + CAP;
    const int cnt = mine ? sy : 0;
    const int incl = wave_incl_scan(cnt);
    const int total = __builtin_amdgcn_readlane(incl, 63);
    const int start = incl - cnt;
    wave_sync();  // the previous batch's reads of ws are done
    if (mine) {
      ws.hi[rank - r0] = make_int4((h.ybase & 0xffff) | (h.zbase << 16), sz | (start << 8), __float_as_int(h.offy),
                                   __float_as_int(h.offz));
      ws.hf[rank - r0] = make_float4(h.dx2, h.c2s, h.w * p.inv1me0 * S, 0.f);
    }
    int before = 0;  // hits whose rows start before this step's first row
    for (int base = 0; base < total; base += 64) {
      wave_sync();
      if (lane < 16) ws.flag[lane] = 0;
      wave_sync();
      if (mine && start >= base && start < base + 64) flag8[start - base] = 1;
      wave_sync();
      const bool f = flag8[lane] != 0;
      const unsigned long long fm = __ballot(f);
      const int j = before + lanes_below(fm) + (f ? 1 : 0) - 1;
      before += __popcll(fm);
      if (base + lane < total) {
        const int4 a = ws.hi[j];
        const float4 c = ws.hf[j];
        const int row = base + lane - (a.y >> 8), szj = a.y & 0xff, zb = a.x >> 16;
        const int yy = wrap_axis<N>((int)(short)(a.x & 0xffff) + row);
        const float dy = __int_as_float(a.z) + (float)row;
        const float dyy = fmaf(dy, dy, c.x);
        const float ym = (chan == 2) ? c.z * yhat(yy, N) : c.z;
        float dz = __int_as_float(a.w);
        // the hit's LDS reads complete here, not at the loop head, where the
        // wait would also hold each step until the previous atomic is done
        __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
        for (int k = 0; k < szj; ++k, dz += 1.0f) {
          const float e = fmaf(dz, dz, dyy) * c.y;  // d^2 / (2 s^2)
          if (e < p.sig_c) {                       // d < rho
            const int zz = wrap_axis<N>(zb + k);
            float val = ym * (__expf(-e) - p.e0);
            if (chan == 3) val *= yhat(zz, N);
            atomicAdd(reinterpret_cast<int*>(&Wf[idx(yy, zz)]), __float2int_rn(val));
          }
        }
      }
    }
  }
}

// Pass 1. grid = (N planes, batch). GRID: real grids `grid` [batch][N^3].
// Otherwise splat from the binned samples (p.rec, p.cand) of each batch
// member. Writes the plane spectra of every batch member,
// out[(b*N + x)*N*H].
template <int N, bool GRID>
__global__ void __launch_bounds__(Plane<N>::THREADS, Plane<N>::MINW) k_plane_fwd(SplatParams p,
                                                                               const float* __restrict__ grid,
                                                                               float2* __restrict__ out,
                                                                               const float2* __restrict__ table) {
  using P = Plane<N>;
  __shared__ __attribute__((aligned(16))) float2 W[P::SIZE];
  __shared__ float2 tw_tab[kPlaneTwTab<N> ? N : 1];
  const int x = blockIdx.x, b = blockIdx.y, tid = threadIdx.x;
  float* Wf = reinterpret_cast<float*>(W);
  const size_t plane_sz = (size_t)N * P::H;
  PlaneTw<N> tw;
  plane_twiddles<N>(tw, table, tw_tab, (tid & 63) % P::L);
  // the y transforms store the spectrum straight to global memory up to
  // edge 128; the 192 transforms need their registers (copy-out from LDS)
  constexpr bool kDirect = N <= 128;
  float2* dst0 = out + ((size_t)b * N + x) * plane_sz;
  float S = 1.0f;  // fixed-point scale of the splat sums
  if constexpr (GRID) {
    const float2* src = reinterpret_cast<const float2*>(grid + ((size_t)b * N + x) * N * N);
    // two adjacent z values of one row land in one pair-region entry each
    batched_copy<N * N / 2, P::THREADS, float2>([&](int i) { return src[i]; }, [&](int i, float2 v) {
      const int y = (2 * i) / N, z = (2 * i) % N;
      Wf[P::zs(y >> 1, z) * 2 + (y & 1)] = v.x;
      Wf[P::zs(y >> 1, z + 1) * 2 + (y & 1)] = v.y;
    });
  } else {
    // binned samples (p.rec, p.cand): each wavefront tests its candidates
    // and splats its hits (wave_splat); a plane no sample reaches has a zero
    // spectrum, written directly
    const int4 rg = p.cand[(size_t)b * N + x];
    const int ncand = rg.y + rg.w;
    if (ncand == 0) {  // no sample within reach: a zero plane, known before any load or fill
      if (p.pmask) return;
      float4* d0 = reinterpret_cast<float4*>(dst0);
      for (int i = tid; i < (int)(plane_sz / 2); i += P::THREADS) d0[i] = make_float4(0.f, 0.f, 0.f, 0.f);
      return;
    }
    const Placed* rb = p.rec + (size_t)b * p.n_pts;
    const int lane = tid & 63, wave = tid >> 6;
    auto pidx = [](int yy, int zz) { return P::zs(yy >> 1, zz) * 2 + (yy & 1); };
    Placed q;
    const bool is_cand = wave_cand(rb, rg, lane * P::WAVES + wave, q);
    float4* W4 = reinterpret_cast<float4*>(W);
    for (int i = tid; i < P::SIZE / 2; i += P::THREADS) W4[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    __shared__ WaveSplatLds<kSplatCap<N>> wsl[P::WAVES];
    __shared__ float bnd[2 * P::WAVES];
    WaveHit h{};
    bool hit = is_cand && wave_hit<N>(p, q, x, h);
    const PlaneBound pb =
        plane_bound<P::WAVES, P::THREADS>(rb, rg, ncand, is_cand ? fabsf(__int_as_float(q.b.w)) : 0.f, hit, bnd);
    if (!pb.any && ncand <= 64 * P::WAVES) {
      if (p.pmask) return;  // not stored: its mask bit stays clear
      float4* d0 = reinterpret_cast<float4*>(dst0);
      for (int i = tid; i < (int)(plane_sz / 2); i += P::THREADS) d0[i] = make_float4(0.f, 0.f, 0.f, 0.f);
      return;
    }
    if (p.pmask && tid == 0) atomicOr(&p.pmask[(size_t)b * kPlaneMaskWords<N> + (x >> 5)], 1u << (x & 31));
    S = splat_scale(pb.wsum);
    for (int c0 = 0;;) {
      wave_splat<N>(p, hit, h, 0, S, Wf, pidx, wsl[wave]);
      c0 += 64 * P::WAVES;
      if (c0 >= ncand) break;  // uniform
      const bool more = wave_cand(rb, rg, c0 + lane * P::WAVES + wave, q);
      hit = more && wave_hit<N>(p, q, x, h);
    }
  }
  __syncthreads();
  if constexpr (!GRID) {
    plane_fix_to_float<P::THREADS>(W, P::SIZE / 2, 1.0f / S);
    __syncthreads();
  }
  plane_forward_out<N, kDirect>(W, tw, dst0, nullptr, 1.0f);
  if constexpr (!kDirect) plane_to_global<N>(dst0, W, 1.0f);
}

// ---------------------------------------------------------------------------
// Pass 1 for grid edges with a two-stage transform schedule (the 128^3
// workloads): the same splat -> z R2C -> y FFT of one x-plane as k_plane_fwd,
// arranged so that every LDS address is a per-lane base plus a compile-time
// offset and the transforms' access shapes do not meet bank conflicts.
//
//  * Rows t and t + N/2 of the plane form the complex row pair t (real and
//    imaginary parts). A lane of the y transforms reads rows y and y + N/2 of
//    its column together, so the two-for-one split of the z pass happens in
//    that read: A_t(c) = Z_t(c) + conj Z_t(N-c) for row t and
//    B_t(c) = -i (Z_t(c) - conj Z_t(N-c)) for row t + N/2. The factor 1/2 of
//    the split is applied by the splat (an exact power-of-two scale), so no
//    separate split pass through LDS remains.
//  * Z_t(k) of row pair t lives at slot al(t) + be(k) with
//      al(t) = S t + 4 floor(t/4) + 2 floor(t/8),   be(k) = k + floor(k/16).
//    In every access below the compile-time part of t or k is a multiple of
//    each floor term's divisor, so the address splits into a lane base and an
//    immediate offset.
//  * The y transform of column c (1 <= c < N/2) runs in place in the slots of
//    Z_t(c) and Z_t(N-c), which no other transform reads; column 0 packs the
//    real columns kz = 0 and kz = N/2 into one transform (the slots of k = 0
//    and k = N/2) and is split after it. Its position q lives in row
//    (q & 7) | ((q >> 4) << 3) of column c or N - c by bit 3 of q, a bit that
//    is the same for all lanes of each access.
// With 8-byte LDS reads served per half-wave on 32 bank pairs (slot mod 32)
// and writes per quarter-wave on 16 (slot mod 16), S = 136 makes every z
// access conflict-free; a y access conflicts (two ways, in one lane group)
// only where four consecutive columns N - c straddle a multiple of 16.
template <int N> struct PlaneP {
  static constexpr bool ok = false;
};
template <> struct PlaneP<128> {
  static constexpr bool ok = true;
  static constexpr int R0 = 16, R1 = 8;  // stage radices
  static constexpr int E = 16, L = 8;    // elements per lane, lanes per transform
  static constexpr int NB1 = E / R1;     // stage-1 butterflies per lane
  static constexpr int TPW = 64 / L;     // transforms per wavefront
  static constexpr int WAVES = 8, THREADS = 512;
  static constexpr int H = 65, S = 136;
  __host__ __device__ static constexpr int al(int t) { return t * S + (t >> 2) * 4 + (t >> 3) * 2; }
  __host__ __device__ static constexpr int be(int k) { return k + (k >> 4); }
  static constexpr int SIZE = 8778;  // float2 slots: al(63) + be(127) + 1, rounded up to even (zeroed as float4)
};
static_assert(PlaneP<128>::TPW * PlaneP<128>::WAVES == 64, "one transform per lane group and phase");
static_assert(PlaneP<128>::be(127) < PlaneP<128>::S, "rows do not overlap");
static_assert(PlaneP<128>::al(63) + PlaneP<128>::be(127) < PlaneP<128>::SIZE && PlaneP<128>::SIZE % 2 == 0,
              "plane slots");

// Single-translation sums of one x-plane (the serving path's re-correlation):
// the partial sum of eq. 7b over the modes (k_y, k_z) of plane x after the z
// and y transforms, with the x transform folded into resident data. For the
// moving part's plane spectrum C(x, k_y, k_z) (x not transformed),
//   sum_kx Ahat(k) conj(Chat(k)) e^{2 pi i kx tx / N}
//     = sum_x conj(C(x, k_y, k_z)) AX(x + tx, k_y, k_z),
// AX(x') = sum_kx Ahat(kx, k_y, k_z) e^{+2 pi i kx x'/N} (Ahat inverse-
// transformed along x, unnormalised), and the x-derivative multiplier
// 2 pi i omega(kx) of eq. 6a goes into a second array DX the same way. Each
// plane therefore adds its own share of all 7 sums: with
// s = conj(C) AX e^{i phi}, d = conj(C) DX e^{i phi},
// phi = 2 pi (k_y t_y + k_z t_z)/N, Hermitian weight w (1 at k_z = 0, N/2,
// else 2), omega_y = omega(k_y), omega_z = omega(k_z), yx = yhat(x):
//   u channel:        E += w Re s,  F_x -= w Re d,  F_y += 2 pi w omega_y Im s,
//                     F_z += 2 pi w omega_z Im s,
//                     tau_y -= 2 pi w omega_z yx Im s,  tau_z += 2 pi w omega_y yx Im s
//                     (the moment yhat_x u is u times yx on the plane);
//   yhat_y u channel: tau_x += 2 pi w omega_z Im s,  tau_z += w Re d;
//   yhat_z u channel: tau_x -= 2 pi w omega_y Im s,  tau_y -= w Re d;
// all times N^-3 in the final reduction (eq. 6a, 6b, 7b; Sec. 3.3).
struct SingleAcc {
  double v[7] = {0, 0, 0, 0, 0, 0, 0};
  // per-lane float sums of one channel pass, folded into v by fold()
  float re = 0.f, dre = 0.f, wyim = 0.f, im = 0.f;
  __device__ __forceinline__ void add(float2 y, float2 a, float2 d, float wy) {
    const float sre = y.x * a.x + y.y * a.y, sim = y.x * a.y - y.y * a.x;  // conj(y) a
    re += sre;
    im += sim;
    wyim += wy * sim;
    dre += y.x * d.x + y.y * d.y;  // Re conj(y) d
  }
  // pass 0: u; 1: yhat_y u; 2: yhat_z u; w, wz: the lane's weight and omega_z
  __device__ __forceinline__ void fold(int pass, float w, float wz, float yx) {
    constexpr double tp = 6.283185307179586476925286766559;
    const double W = w;
    if (pass == 0) {
      v[0] += W * re;
      v[1] -= W * dre;
      v[2] += tp * W * wyim;
      v[3] += tp * W * wz * im;
      v[5] -= tp * W * wz * yx * im;
      v[6] += tp * W * yx * wyim;
    } else if (pass == 1) {
      v[4] += tp * W * wz * im;
      v[6] += W * dre;
    } else {
      v[4] -= tp * W * wyim;
      v[5] -= W * dre;
    }
    re = dre = wyim = im = 0.f;
  }
};

// Sum of the 7 accumulators over a workgroup of NT threads (fixed order),
// written by threads 0..6 to dst[0..7).
template <int NT>
__device__ __forceinline__ void block_sum7(const SingleAcc& acc, double* red /* LDS, 7 x NT/64 */, double* dst) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int o = 0; o < 7; ++o) {
    double v = acc.v[o];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) red[o * (NT / 64) + wave] = v;
  }
  __syncthreads();
  if (tid < 7) {
    double sum = 0;
    for (int wv = 0; wv < NT / 64; ++wv) sum += red[tid * (NT / 64) + wv];
    dst[tid] = sum;
  }
}

// Body of the pass-1 kernels of the two-stage layout: splat the binned
// samples of batch member blockIdx.y (p.rec, p.cand) into plane x =
// blockIdx.x, transform it along z and y.
// SINGLE = false: the plane spectrum of u goes to out[(b*N + x)*N*H].
// SINGLE = true: channel pass z = blockIdx.z (u, then yhat_y u, then
// yhat_z u; yhat_x u is u times yhat(x)) adds the plane's share of the 7
// single-translation sums of query items[b] (SingleAcc) and writes them to
// part[((b*3 + z)*N + x)*7 ..]; nothing else is written.
template <int N, bool SINGLE>
__device__ __forceinline__ void plane_splat_body(const SplatParams& p, float2* __restrict__ out,
                                                 const QueryItem* __restrict__ items, double* __restrict__ part,
                                                 const float2* __restrict__ table) {
  using P = PlaneP<N>;
  constexpr int H = P::H, L = P::L, R1 = P::R1, NB1 = P::NB1, T = N / 2;
  static_assert(P::R0 == 16 && R1 == 8 && L == 8 && NB1 == 2, "schedule of the code below");
  __shared__ __attribute__((aligned(16))) float2 W[P::SIZE];
  __shared__ float2 tabc[SINGLE ? N : 1];  // exp(+2 pi i m / N)
  __shared__ double red[SINGLE ? 7 * P::WAVES : 1];
  const int x = blockIdx.x, b = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tau = lane / L, l = lane % L;
  const int pass = SINGLE ? (int)blockIdx.z : 0;
  const int chan = (pass == 0) ? 0 : pass + 1;  // splat multiplier: 0 none, 2 yhat_y, 3 yhat_z
  // stage-1 twiddles exp(-2 pi i r j / N), j = l + L bb (both transforms):
  // in registers, or (single-translation mode, whose sums take registers)
  // read from the LDS table when needed
  float2 tw[SINGLE ? 1 : NB1][R1];
  if constexpr (!SINGLE) {
#pragma unroll
    for (int bb = 0; bb < NB1; ++bb)
#pragma unroll
      for (int r = 1; r < R1; ++r) tw[bb][r] = table[r * (l + L * bb)];
  }
  auto twid = [&](int bb, int r) -> float2 {
    if constexpr (SINGLE) {
      const float2 e = tabc[r * (l + L * bb)];
      return make_float2(e.x, -e.y);
    } else {
      return tw[bb][r];
    }
  };
  const size_t plane_sz = (size_t)N * H;
  float2* dst0 = SINGLE ? nullptr : out + ((size_t)b * N + x) * plane_sz;
  double* dstp = SINGLE ? part + (((size_t)b * 3 + pass) * N + x) * 7 : nullptr;
  const float s1 = yhat(x, N);
  // single-translation sums: the query's translation and plane x + t_x of
  // the resident AX and DX
  int ty = 0, tz = 0;
  const float2* AXp = nullptr;
  SingleAcc acc;
  if constexpr (SINGLE) {
    const QueryItem& it = items[b];
    ty = it.t[1];
    tz = it.t[2];
    AXp = it.AX + (size_t)((x + it.t[0]) % N) * plane_sz;
    for (int i = tid; i < N; i += P::THREADS) tabc[i] = make_float2(table[i].x, -table[i].y);
  }

  // splat: candidate c of the plane's runs is tested by lane c / WAVES of
  // wave c % WAVES (the first round's loads are in flight during the zero
  // fill), then each wave splats its own hits
  SplatParams sp = p;
  sp.inv1me0 *= 0.5f;  // the 1/2 of the two-for-one split
  const int4 rg = p.cand[(size_t)b * N + x];
  const int ncand = rg.y + rg.w;
  if (ncand == 0) {  // no sample within reach: a zero plane, known before any load or fill
    if constexpr (SINGLE) {
      if (tid < 7) dstp[tid] = 0.0;
    } else if (!p.pmask) {
      float4* d = reinterpret_cast<float4*>(dst0);
      for (int i = tid; i < (int)(plane_sz / 2); i += P::THREADS) d[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    return;
  }
  const Placed* rb = p.rec + (size_t)b * p.n_pts;
  auto pidx = [](int yy, int zz) { return 2 * (P::al(yy & (T - 1)) + P::be(zz)) + (yy >= T ? 1 : 0); };
  Placed q;
  const bool is_cand = wave_cand(rb, rg, lane * P::WAVES + wave, q);
  float4* W4 = reinterpret_cast<float4*>(W);
  for (int i = tid; i < P::SIZE / 2; i += P::THREADS) W4[i] = make_float4(0.f, 0.f, 0.f, 0.f);
  __shared__ WaveSplatLds<kSplatCap<N>> wsl[P::WAVES];
  __shared__ float bnd[2 * P::WAVES];
  WaveHit h{};
  bool hit = is_cand && wave_hit<N>(sp, q, x, h);
  const PlaneBound pb =
      plane_bound<P::WAVES, P::THREADS>(rb, rg, ncand, is_cand ? fabsf(__int_as_float(q.b.w)) : 0.f, hit, bnd);
  // A plane that no sample reaches is zero, and so is its spectrum: it is
  // written directly (or adds nothing), without the transforms.
  if (!pb.any && ncand <= 64 * P::WAVES) {
    if constexpr (SINGLE) {
      if (tid < 7) dstp[tid] = 0.0;
    } else if (!p.pmask) {  // with a plane mask the plane is not stored (its bit stays clear)
      float4* d = reinterpret_cast<float4*>(dst0);
      for (int i = tid; i < (int)(plane_sz / 2); i += P::THREADS) d[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    return;
  }
  if constexpr (!SINGLE) {
    if (p.pmask && tid == 0) atomicOr(&p.pmask[(size_t)b * kPlaneMaskWords<N> + (x >> 5)], 1u << (x & 31));
  }
  float* Wf = reinterpret_cast<float*>(W);
  const float S = splat_scale(chan ? pb.wsum * (0.5f * N) : pb.wsum), inv_s = 1.0f / S;
  for (int c0 = 0;;) {
    wave_splat<N>(sp, hit, h, chan, S, Wf, pidx, wsl[wave]);
    c0 += 64 * P::WAVES;
    if (c0 >= ncand) break;  // uniform
    const bool more = wave_cand(rb, rg, c0 + lane * P::WAVES + wave, q);
    hit = more && wave_hit<N>(sp, q, x, h);
  }
  __syncthreads();

  // z: complex transform of row pair t = 8 wave + tau (rows t and t + N/2)
  {
    const int t = P::TPW * wave + tau;
    float2* zb = W + P::al(t) + l;  // position l + m (m a multiple of 8) at zb[be(m)]
    float2 v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {  // the splat's fixed-point sums, back to float
      const int2 iv = reinterpret_cast<const int2*>(zb)[P::be(8 * r)];
      v[r] = make_float2((float)iv.x * inv_s, (float)iv.y * inv_s);
    }
    Bfly<16, -1>::run(v);
    float2* zw = W + P::al(t) + 17 * l;  // position 16 l + r at be(16 l + r) = 17 l + r
    wave_sync();
#pragma unroll
    for (int r = 0; r < 16; ++r) zw[r] = v[r];
    wave_sync();
    float2 u[NB1][R1];
#pragma unroll
    for (int bb = 0; bb < NB1; ++bb)
#pragma unroll
      for (int r = 0; r < R1; ++r) u[bb][r] = zb[P::be(8 * bb + 16 * r)];
    wave_sync();
#pragma unroll
    for (int bb = 0; bb < NB1; ++bb) {
#pragma unroll
      for (int r = 1; r < R1; ++r) u[bb][r] = cmul(u[bb][r], twid(bb, r));
      Bfly<8, -1>::run(u[bb]);
    }
#pragma unroll
    for (int bb = 0; bb < NB1; ++bb)
#pragma unroll
      for (int r = 0; r < R1; ++r) zb[P::be(8 * bb + 16 * r)] = u[bb][r];  // Z_t(k), k = l + 8 bb + 16 r
  }
  __syncthreads();

  // y: column transform c = 8 wave + tau over rows 0 .. N-1
  {
    const int c = P::TPW * wave + tau;
    const int b1 = P::be(c), b2 = P::be(c == 0 ? T : N - c);
    float2* r1 = W + P::al(l) + b1;  // row l + 8 m of column c at r1[al(8 m)]
    float2* r2 = W + P::al(l) + b2;  // ... of column N - c (or N/2)
    float2 v[16];
    {
      float2 z1[8], z2[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        z1[r] = r1[P::al(8 * r)];
        z2[r] = r2[P::al(8 * r)];
      }
      if (c != 0) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          v[r] = make_float2(z1[r].x + z2[r].x, z1[r].y - z2[r].y);      // row l + 8 r
          v[r + 8] = make_float2(z1[r].y + z2[r].y, z2[r].x - z1[r].x);  // row l + 8 r + N/2
        }
      } else {
        // real columns kz = 0 (real part) and kz = N/2 (imaginary part)
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          v[r] = make_float2(z1[r].x + z1[r].x, z2[r].x + z2[r].x);
          v[r + 8] = make_float2(z1[r].y + z1[r].y, z2[r].y + z2[r].y);
        }
      }
    }
    Bfly<16, -1>::run(v);
    float2* w1 = W + P::al(8 * l) + b1;  // position 16 l + r: row 8 l + (r & 7)
    float2* w2 = W + P::al(8 * l) + b2;
    wave_sync();
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      w1[P::al(r)] = v[r];
      w2[P::al(r)] = v[r + 8];
    }
    wave_sync();
    float2 u[NB1][R1];
#pragma unroll
    for (int r = 0; r < R1; ++r) {
      u[0][r] = r1[P::al(8 * r)];  // position l + 16 r
      u[1][r] = r2[P::al(8 * r)];  // position l + 8 + 16 r
    }
#pragma unroll
    for (int bb = 0; bb < NB1; ++bb) {
#pragma unroll
      for (int r = 1; r < R1; ++r) u[bb][r] = cmul(u[bb][r], twid(bb, r));
      Bfly<8, -1>::run(u[bb]);
    }
    // outputs Y(ky), ky = l + 8 bb + 16 r
    if (c != 0) {
      if constexpr (SINGLE) {
        // column kz = c, weight 2
        const int m0 = l * ty + c * tz;
        const float2* ap = AXp + l * H + c;
#pragma unroll
        for (int bb = 0; bb < NB1; ++bb) {
          // one half's loads at a time: all of them at once would take the
          // registers the transform still holds
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int r = 0; r < R1; ++r) {
            const int ky = l + 8 * bb + 16 * r;
            const float2 ph = tabc[(m0 + (8 * bb + 16 * r) * ty) & (N - 1)];
            const float2 a = cmul(ap[(8 * bb + 16 * r) * H], ph);
            const float2 d = cmul(ap[plane_sz * N + (8 * bb + 16 * r) * H], ph);
            acc.add(u[bb][r], a, d, omega_of<N>(ky));
          }
        }
        acc.fold(pass, 2.f, omega_of<N>(c), s1);
      } else {
        const int lo = (l * H + c) * (int)sizeof(float2);
        const auto rs0 = buffer_rsrc(dst0, (unsigned)(plane_sz * sizeof(float2)));
#pragma unroll
        for (int bb = 0; bb < NB1; ++bb)
#pragma unroll
          for (int r = 0; r < R1; ++r) buffer_store2(u[bb][r], rs0, lo, (8 * bb + 16 * r) * H * (int)sizeof(float2));
      }
    } else {
      // C = P + i Q with P, Q the spectra of the real columns kz = 0 and N/2:
      // P(k) = (C(k) + conj C(N-k))/2, Q(k) = -i (C(k) - conj C(N-k))/2.
      // C(k) goes back to the column's slots; the split reads it there
      // (single-translation sums: at once; spectra: after the barrier below,
      // one thread per k, so that this wavefront does not also store the
      // column while the others have finished).
      wave_sync();
#pragma unroll
      for (int r = 0; r < R1; ++r) {
        r1[P::al(8 * r)] = u[0][r];
        r2[P::al(8 * r)] = u[1][r];
      }
      if constexpr (SINGLE) {
        wave_sync();
#pragma unroll
        for (int bb = 0; bb < NB1; ++bb)
#pragma unroll
          for (int r = 0; r < R1; ++r) {
            const int k = l + 8 * bb + 16 * r, m = (N - k) & (N - 1);
            const float2 a = u[bb][r];
            const float2 z = W[P::al((m & 7) | ((m >> 4) << 3)) + (((m >> 3) & 1) ? b2 : b1)];
            const float2 pk = make_float2(0.5f * (a.x + z.x), 0.5f * (a.y - z.y));
            const float2 qk = make_float2(0.5f * (a.y + z.y), -0.5f * (a.x - z.x));
            // (k, kz = 0) and (k, kz = N/2), weight 1, omega_z = 0
            const float2* ap = AXp + (size_t)k * H;
            const float2 ph0 = tabc[(k * ty) & (N - 1)], ph1 = tabc[(k * ty + T * tz) & (N - 1)];
            acc.add(pk, cmul(ap[0], ph0), cmul(ap[plane_sz * N], ph0), omega_of<N>(k));
            acc.add(qk, cmul(ap[T], ph1), cmul(ap[plane_sz * N + T], ph1), omega_of<N>(k));
          }
        acc.fold(pass, 1.f, 0.f, s1);
      }
    }
  }
  if constexpr (SINGLE) {
    block_sum7<P::THREADS>(acc, red, dstp);
  } else {
    static_assert(P::THREADS >= N, "one thread per k of column 0");
    __syncthreads();
    if (tid < N) {
      // C(q) of column 0 sits at row (q & 7) | ((q >> 4) << 3) of the slots
      // of kz = 0 (bit 3 of q clear) or kz = N/2 (set)
      auto slot = [](int q) { return P::al((q & 7) | ((q >> 4) << 3)) + (((q >> 3) & 1) ? P::be(T) : P::be(0)); };
      const int k = tid, m = (N - k) & (N - 1);
      const float2 a = W[slot(k)], z = W[slot(m)];
      dst0[(size_t)k * H] = make_float2(0.5f * (a.x + z.x), 0.5f * (a.y - z.y));
      dst0[(size_t)k * H + T] = make_float2(0.5f * (a.y + z.y), -0.5f * (a.x - z.x));
    }
  }
}

// grid = (N planes, batch); block = 512. Pass 1 from binned samples: the
// plane spectra of u (plane_splat_body).
template <int N>
__global__ void __launch_bounds__(PlaneP<N>::THREADS, 4) k_plane_splat_fwd(SplatParams p, float2* __restrict__ out,
                                                                          const float2* __restrict__ table) {
  plane_splat_body<N, false>(p, out, nullptr, nullptr, table);
}

// grid = (N planes, queries, 3 channel passes); block = 512. Re-correlated
// single-translation sums of query b over plane x and channel pass z:
// part[((b*3 + z)*N + x)*7 + o] (plane_splat_body).
template <int N>
__global__ void __launch_bounds__(PlaneP<N>::THREADS, 4) k_plane_single(SplatParams p, const QueryItem* __restrict__ items,
                                                                     double* __restrict__ part,
                                                                     const float2* __restrict__ table) {
  plane_splat_body<N, true>(p, nullptr, items, part, table);
}

// Single-translation sums of one x-plane for grid edges without the
// two-stage layout (SingleAcc gives the sums): grid = (N planes, queries, 3
// channel passes), block = Plane<N>::THREADS. Workgroup (x, b, z) splats
// channel pass z of query b (u, then yhat_y u, then yhat_z u; yhat_x u is u
// times yhat(x)) into plane x, transforms it along z and y, and adds the
// plane's share of the 7 sums with the resident AX, DX of the query's pair
// (x + t_x plane), to part[((b*3 + z)*N + x)*7 ..]. Thread t takes column
// k_z = t mod H and rows k_y = t / H + j (THREADS / H), so its Hermitian
// weight and omega_z are fixed.
template <int N>
__global__ void __launch_bounds__(Plane<N>::THREADS, Plane<N>::MINW) k_plane_single_gen(SplatParams p,
                                                                                     const QueryItem* __restrict__ items,
                                                                                     double* __restrict__ part,
                                                                                     const float2* __restrict__ table) {
  using P = Plane<N>;
  constexpr int H = P::H, GR = P::THREADS / H;  // row groups
  static_assert(GR >= 1, "one column per thread at least");
  __shared__ __attribute__((aligned(16))) float2 W[P::SIZE];
  __shared__ float2 tabc[N];  // exp(+2 pi i m / N)
  __shared__ double red[7 * P::WAVES];
  const int x = blockIdx.x, b = blockIdx.y, pass = blockIdx.z, tid = threadIdx.x;
  const int chan = (pass == 0) ? 0 : pass + 1;  // 0, 2, 3
  double* dstp = part + (((size_t)b * 3 + pass) * N + x) * 7;
  const QueryItem& it = items[b];
  const size_t plane_sz = (size_t)N * H;
  const float2* AXp = it.AX + (size_t)((x + it.t[0]) % N) * plane_sz;
  const int ty = it.t[1], tz = it.t[2];
  __shared__ float2 tw_tab[kPlaneTwTab<N> ? N : 1];
  PlaneTw<N> tw;  // first: their loads overlap the splat
  plane_twiddles<N>(tw, table, tw_tab, (tid & 63) % P::L);
  for (int i = tid; i < N; i += P::THREADS) tabc[i] = make_float2(table[i].x, -table[i].y);
  // splat: as the binned branch of k_plane_fwd
  const int4 rg = p.cand[(size_t)b * N + x];
  const int ncand = rg.y + rg.w;
  if (ncand == 0) {  // no sample within reach: a zero plane, known before any load or fill
    if (tid < 7) dstp[tid] = 0.0;
    return;
  }
  const Placed* rb = p.rec + (size_t)b * p.n_pts;
  const int lane = tid & 63, wave = tid >> 6;
  auto pidx = [](int yy, int zz) { return P::zs(yy >> 1, zz) * 2 + (yy & 1); };
  float* Wf = reinterpret_cast<float*>(W);
  Placed q;
  const bool is_cand = wave_cand(rb, rg, lane * P::WAVES + wave, q);
  float4* W4 = reinterpret_cast<float4*>(W);
  for (int i = tid; i < P::SIZE / 2; i += P::THREADS) W4[i] = make_float4(0.f, 0.f, 0.f, 0.f);
  __shared__ WaveSplatLds<kSplatCap<N>> wsl[P::WAVES];
  __shared__ float bnd[2 * P::WAVES];
  WaveHit h{};
  bool hit = is_cand && wave_hit<N>(p, q, x, h);
  const PlaneBound pb =
      plane_bound<P::WAVES, P::THREADS>(rb, rg, ncand, is_cand ? fabsf(__int_as_float(q.b.w)) : 0.f, hit, bnd);
  if (!pb.any && ncand <= 64 * P::WAVES) {
    if (tid < 7) dstp[tid] = 0.0;
    return;
  }
  const float S = splat_scale(chan ? pb.wsum * (0.5f * N) : pb.wsum);
  for (int c0 = 0;;) {
    wave_splat<N>(p, hit, h, chan, S, Wf, pidx, wsl[wave]);
    c0 += 64 * P::WAVES;
    if (c0 >= ncand) break;  // uniform
    const bool more = wave_cand(rb, rg, c0 + lane * P::WAVES + wave, q);
    hit = more && wave_hit<N>(p, q, x, h);
  }
  // this thread's column and first rows of AX, DX: loaded before the
  // transforms so that their latency overlaps them (issued before the
  // barrier that ends the splat)
  constexpr int NJ = (N + GR - 1) / GR, CH = 8;  // rows per thread, rows per load batch
  const bool active = tid < GR * H;
  const int kz = tid % H, ky0 = tid / H;
  float2 ra[CH], rd[CH];
#pragma unroll
  for (int j = 0; j < CH; ++j) {
    const int ky = ky0 + j * GR;
    const bool in = active && j < NJ && ky < N;
    ra[j] = in ? AXp[ky * H + kz] : make_float2(0.f, 0.f);
    rd[j] = in ? AXp[plane_sz * N + ky * H + kz] : make_float2(0.f, 0.f);
  }
  __syncthreads();  // every wave's splat atomics land before any transform reads the plane
  plane_fix_to_float<P::THREADS>(W, P::SIZE / 2, 1.0f / S);
  __syncthreads();
  plane_forward_out<N, false>(W, tw, nullptr, nullptr, 0.f);  // spectrum stays in W
  SingleAcc acc;
  if (active) {
#pragma unroll 1
    for (int j0 = 0; j0 < NJ; j0 += CH) {
      float2 na[CH], nd[CH];
#pragma unroll
      for (int j = 0; j < CH; ++j) na[j] = nd[j] = make_float2(0.f, 0.f);
      if (j0 + CH < NJ) {  // next batch in flight while this one is summed
#pragma unroll
        for (int j = 0; j < CH; ++j) {
          const int ky = ky0 + (j0 + CH + j) * GR;
          const bool in = j0 + CH + j < NJ && ky < N;
          na[j] = in ? AXp[ky * H + kz] : make_float2(0.f, 0.f);
          nd[j] = in ? AXp[plane_sz * N + ky * H + kz] : make_float2(0.f, 0.f);
        }
      }
#pragma unroll
      for (int j = 0; j < CH; ++j) {
        const int ky = ky0 + (j0 + j) * GR;
        if (j0 + j < NJ && ky < N) {
          const float2 ph = tabc[(ky * ty + kz * tz) % N];
          acc.add(W[P::yc(ky, kz)], cmul(ra[j], ph), cmul(rd[j], ph), omega_of<N>(ky));
        }
      }
#pragma unroll
      for (int j = 0; j < CH; ++j) {
        ra[j] = na[j];
        rd[j] = nd[j];
      }
    }
    acc.fold(pass, (kz == 0 || kz == N / 2) ? 1.f : 2.f, omega_of<N>(kz), yhat(x, N));
  }
  block_sum7<P::THREADS>(acc, red, dstp);
}

// The x-inverse-transformed resident data of the single-translation sums:
// out[e] = Ahat[e] and out[spec + e] = 2 pi i omega(kx) Ahat[e] (the x
// derivative multiplier of eq. 6a); the x transforms follow (k_strip_fft).
template <int N>
__global__ void k_ax_inputs(const float2* __restrict__ A, float2* __restrict__ out) {
  constexpr int H = N / 2 + 1;
  const size_t spec = (size_t)N * N * H;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= spec) return;
  const float w = omega_of<N>((int)(e / ((size_t)N * H)));
  const float2 a = A[e];
  out[e] = a;
  out[spec + e] = make_float2(-kTwoPi * w * a.y, kTwoPi * w * a.x);
}

// The density itself: grid = (N planes). Writes nch real grids
// out[(c*N + x)*N*N + y*N + z]: u, then yhat_x u, yhat_y u, yhat_z u.
template <int N>
__global__ void __launch_bounds__(Plane<N>::THREADS) k_splat_real(SplatParams p, int nch, float* __restrict__ out) {
  using P = Plane<N>;
  __shared__ float U[N * N];
  __shared__ HitList hl;
  const int x = blockIdx.x, tid = threadIdx.x;
  double R[9];
  load_rotation(p, 0, R);
  for (int i = tid; i < N * N; i += P::THREADS) U[i] = 0.f;
  __syncthreads();
  splat_plane<N, P::WAVES, P::THREADS>(p, R, 0, x, 0, U, hl, [](int yy, int zz) { return yy * N + zz; });
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
__global__ void __launch_bounds__(Plane<N>::THREADS, Plane<N>::MINW) k_plane_inv(const float2* __restrict__ in, float* __restrict__ out,
                                                                 float scale, const float2* __restrict__ table) {
  using P = Plane<N, true>;
  constexpr int L = P::L, TPW = P::TPW, H = P::H;
  __shared__ __attribute__((aligned(16))) float2 W[P::SIZE];
  const int x = blockIdx.x, b = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l = lane % L;
  __shared__ float2 tw_tab[kPlaneTwTab<N> ? N : 1];
  plane_from_global<N>(W, in + ((size_t)b * N + x) * (size_t)N * H);
  PlaneTw<N> tw;
  plane_twiddles<N>(tw, table, tw_tab, l);
  __syncthreads();
  // Columns kz = 0 and kz = N/2: the z C2R below keeps only the real part of
  // both, so they go through one transform of c = h(col0) + i h(colN/2),
  // h(a)(k) = (a(k) + conj a(-k))/2, whose inverse is Re IFFT(col0) +
  // i Re IFFT(colN/2). c is formed in place in column 0 before the y
  // transforms (read, barrier, write, barrier), so that every y transform
  // loads and stores its own column alike.
  static_assert(P::THREADS >= N, "one thread per position of column 0");
  {
    float2 cv = make_float2(0.f, 0.f);
    if (tid < N) {
      const int m = (N - tid) % N;
      const float2 a0 = W[P::yc(tid, 0)], a1 = W[P::yc(m, 0)];
      const float2 b0 = W[P::yc(tid, N / 2)], b1 = W[P::yc(m, N / 2)];
      const float2 ha = make_float2(0.5f * (a0.x + a1.x), 0.5f * (a0.y - a1.y));
      const float2 hb = make_float2(0.5f * (b0.x + b1.x), 0.5f * (b0.y - b1.y));
      cv = make_float2(ha.x - hb.y, ha.y + hb.x);
    }
    __syncthreads();
    if (tid < N) W[P::yc(tid, 0)] = cv;
    __syncthreads();
  }
  // y: columns 0 .. N/2-1 in place (column 0 holds c)
  for (int it = 0; it * P::WAVES * TPW < N / 2; ++it) {
    const int t = (it * P::WAVES + wave) * TPW + lane / L;
    if (t < N / 2) fft_inplace_at<N, +1>(l, tw, [=](int pos) { return W + P::yc(pos, t); });
  }
  __syncthreads();
  float* dst = out + ((size_t)b * N + x) * (size_t)N * N;
  for (int it = 0; it * P::WAVES * TPW < N / 2; ++it) {
    const int t = (it * P::WAVES + wave) * TPW + lane / L;
    if (t < N / 2) {
      auto reg = [=](int pos) { return W + P::zs(t, pos); };
      // Z(k) = A(k) + i B(k), completed by Hermitian symmetry; A, B are the
      // spectra of rows 2t and 2t+1 (imaginary parts dropped at k = 0, N/2).
      // The first stage reads every row value before any lane writes the
      // region in the transform's own layout.
      auto ld = [&](int k) -> float2 {
        if (k < H) {
          // k = N/2 is the imaginary part of column 0 (see above)
          const int kk = (k == N / 2) ? 0 : k;
          float2 a = W[P::yc(2 * t, kk)], bb = W[P::yc(2 * t + 1, kk)];
          if (k == N / 2) {
            a.x = a.y;
            bb.x = bb.y;
          }
          if (k == 0 || k == N / 2) {
            a.y = 0.f;
            bb.y = 0.f;
          }
          return make_float2(a.x - bb.y, a.y + bb.x);
        }
        const float2 a = W[P::yc(2 * t, N - k)], bb = W[P::yc(2 * t + 1, N - k)];
        return make_float2(a.x + bb.y, bb.x - a.y);
      };
      float* r0 = dst + (size_t)(2 * t) * N;
      auto st = [&](int k, float2 v) {
        r0[k] = v.x * scale;
        r0[N + k] = v.y * scale;
      };
      fft_at<N, +1>(l, tw, reg, ld, st);
    }
  }
}

// LDS layout of a strip (N x-values by G columns): element (x, g) at
// x*LD + (g ^ (((x >> SH) & MASK) * MUL)). 8-byte LDS reads are served per
// half-wave on 32 bank pairs (slot mod 32), writes per quarter-wave on 16
// (slot mod 16); the row padding and the x-dependent XOR of the column
// spread both access shapes of the Stockham stages (lanes walking
// consecutive x, and lanes walking x in steps of the first radix) over
// distinct bank pairs. The XOR reads only x bits that are either the same
// for all lanes of an access or fixed per lane, and stays inside aligned
// blocks of G columns, so each row keeps its G slots.
template <int N> struct StripSwz {  // pad, shift, multiplier, mask
  static constexpr int PAD = 1, SH = 0, MUL = 0, MASK = 0;
};
#define GA_STRIP_SWZ(NN, P, S, M, K)                                  \
  template <> struct StripSwz<NN> {                                   \
    static constexpr int PAD = P, SH = S, MUL = M, MASK = K;          \
  };
GA_STRIP_SWZ(16, 4, 2, 4, 3)
GA_STRIP_SWZ(24, 8, 0, 0, 0)
GA_STRIP_SWZ(32, 4, 2, 2, 7)
GA_STRIP_SWZ(48, 4, 0, 0, 0)
GA_STRIP_SWZ(64, 2, 3, 2, 7)
GA_STRIP_SWZ(96, 4, 0, 0, 0)
GA_STRIP_SWZ(128, 2, 3, 2, 7)
GA_STRIP_SWZ(192, 2, 0, 0, 0)
#undef GA_STRIP_SWZ

template <int N, int G, class SH = Shape<N>> struct Strip {
  static constexpr int H = N / 2 + 1;
  static constexpr int C = N * H;  // columns per x-plane
  static constexpr int L = lanes_per_fft<N, SH>();
  static constexpr int TPW = ffts_per_wave<N, SH>();
  static constexpr int WAVES = G / TPW;
  static constexpr int THREADS = 64 * WAVES;
  using Z = StripSwz<N>;
  static constexpr int LD = G + Z::PAD;  // padded LDS row
  static constexpr int SIZE = N * LD;
  static_assert(G % TPW == 0, "strip width must be a whole number of transforms per wave");
  static_assert(Z::MUL * Z::MASK < G && (G & (G - 1)) == 0, "column XOR must stay inside the strip");
  __device__ __forceinline__ static int idx(int x, int g) { return x * LD + (g ^ (((x >> Z::SH) & Z::MASK) * Z::MUL)); }
};

// Loads in flight per thread: the largest divisor of it up to 16.
constexpr int load_batch(int it) {
  for (int b = 16; b > 1; --b)
    if (it % b == 0) return b;
  return 1;
}
template <int N, int G, class SH = Shape<N>>
__device__ __forceinline__ void strip_load(float2* S, const float2* src, int c0, const unsigned* rows = nullptr) {
  using T = Strip<N, G, SH>;
  // rows: a plane mask (kPlaneMaskWords<N> words) or null; rows whose bit is
  // clear are zero and not read. Thread (x0, g) takes rows x0 + XS u of
  // column g, so the word and bit offset of row x0 + XS u are compile-time
  // for each u (XS divides 32 and x0 < XS).
  constexpr int XS = T::THREADS / G, IT = N / XS, B = load_batch(IT), MW = kPlaneMaskWords<N>;
  if constexpr (!(T::THREADS % G == 0 && N % XS == 0 && 32 % XS == 0)) {
    batched_copy<N * G, T::THREADS, float2>(
        [&](int i) {
          const int x = i / G, c = c0 + i % G;
          const bool live = !rows || ((rows[x >> 5] >> (x & 31)) & 1u);
          return (c < T::C && live) ? src[(size_t)x * T::C + c] : make_float2(0.f, 0.f);
        },
        [&](int i, float2 v) { S[T::idx(i / G, i % G)] = v; });
  } else {
    // raw buffer loads: one per-lane offset for all rows, the row step a
    // compile-time scalar offset; a row that is not read gets an offset
    // beyond the buffer, for which the load returns zero without a memory
    // access
    static_assert((size_t)N * T::C * sizeof(float2) < 0x80000000u, "strip offsets below the skip offset");
    constexpr unsigned kSkip = 0x80000000u;
    unsigned rw[MW];
#pragma unroll
    for (int j = 0; j < MW; ++j) rw[j] = rows ? rows[j] : ~0u;
    const int x0 = (int)threadIdx.x / G, g = (int)threadIdx.x % G, c = c0 + g;
    const bool colok = c < T::C;
    const auto rs = buffer_rsrc(const_cast<float2*>(src), (unsigned)((size_t)N * T::C * sizeof(float2)));
    const unsigned vbase = (unsigned)(((size_t)x0 * T::C + c) * sizeof(float2));
#pragma unroll
    for (int u0 = 0; u0 < IT; u0 += B) {
      float2 v[B];
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const int xr = XS * (u0 + u);  // row x0 + xr
        const bool live = colok && ((rw[xr >> 5] >> ((xr & 31) + x0)) & 1u);
        const u32x2 r = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)(live ? vbase : kSkip),
                                                              (int)((size_t)xr * T::C * sizeof(float2)), 0);
        v[u] = make_float2(__uint_as_float(r.x), __uint_as_float(r.y));
      }
#pragma unroll
      for (int u = 0; u < B; ++u) S[T::idx(x0 + XS * (u0 + u), g)] = v[u];
    }
  }
}
template <int N, int G, class SH = Shape<N>>
__device__ __forceinline__ void strip_store(const float2* S, float2* dst, int c0) {
  using T = Strip<N, G, SH>;
  for (int i = threadIdx.x; i < N * G; i += T::THREADS) {
    const int x = i / G, g = i % G, c = c0 + g;
    if (c < T::C) dst[(size_t)x * T::C + c] = S[T::idx(x, g)];
  }
}
template <int N, int G, int DIR, class SH>
__device__ __forceinline__ void strip_fft(float2* S, const Twiddles<N, SH>& tw) {
  using T = Strip<N, G, SH>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = wave * T::TPW + lane / T::L;
  fft_inplace_at<N, DIR>(lane % T::L, tw, [=](int x) { return S + T::idx(x, g); });
}

// x FFT of a strip of columns, in place or out of place.
// grid = (ceil(C/G), batch); element stride between batch members = N*C.
// in and out may be the same buffer (in-place transform), so neither is
// declared __restrict__.
template <int N, int G, int DIR>
__global__ void __launch_bounds__((Strip<N, G>::THREADS)) k_strip_fft(const float2* in, float2* out,
                                                                    const float2* __restrict__ table) {
  using T = Strip<N, G>;
  __shared__ float2 S[T::SIZE];
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
// grid = (nstrips, ceil(batch / K)): a workgroup takes one strip of K batch
// members in turn. With a shared stationary spectrum (a_stride = 0, FWD) each
// thread keeps its elements of A in registers, so A is read once per K
// members. B and out may be the same buffer (the fused path works in place),
// so neither is declared __restrict__. bmask (FWD, or null): the plane masks
// of B's members (SplatParams::pmask); planes whose bit is clear are zero and
// not read.
// xcd_m > 0 selects a one-dimensional, XCD-aware grid: workgroups are
// dispatched round-robin over the 8 XCDs (each with its own L2), so
// workgroup id runs on XCD id % 8; the xcd_m member groups of one strip are
// given consecutive ids on the same XCD (strip (id / 8 / xcd_m) * 8 + id % 8,
// group (id / 8) % xcd_m), and the strip of A they share stays in that L2.
template <int N, int G, bool FWD, int K = 1, class SH = Shape<N>>
__global__ void __launch_bounds__((Strip<N, G, SH>::THREADS)) k_strip_corr(const float2* __restrict__ A,
                                                                         long long a_stride, const float2* B,
                                                                         float2* out, int batch, int xcd_m,
                                                                         const float2* __restrict__ table,
                                                                         const unsigned* __restrict__ bmask) {
  using T = Strip<N, G, SH>;
  constexpr int IT = (N * G + T::THREADS - 1) / T::THREADS;  // strip elements per thread
  constexpr int NSTRIPS = (T::C + G - 1) / G;
  int sx = blockIdx.x, my = blockIdx.y;
  if (xcd_m > 0) {
    const int slot = (int)(blockIdx.x >> 3);
    my = slot % xcd_m;
    sx = (slot / xcd_m) * 8 + (int)(blockIdx.x & 7);
    if (sx >= NSTRIPS) return;  // whole workgroup
  }
  __shared__ float2 S[T::SIZE];
  Twiddles<N, SH> tw;
  const int lane = (int)threadIdx.x & 63, tl = lane % T::L, g = ((int)threadIdx.x >> 6) * T::TPW + lane / T::L;
  load_twiddles<N>(tw, table, tl);  // this thread: lane tl of the x transform of column g
  const int c0 = sx * G;
  auto a_at = [&](const float2* Ab, int i) {
    const int x = i / G, c = c0 + i % G;
    return (c < T::C) ? Ab[(size_t)x * T::C + c] : make_float2(0.f, 0.f);
  };
  // FWD with a shared stationary spectrum (K > 1): that spectrum, held in
  // registers for the K members, in the order the forward x transform hands
  // out its results (element e of this lane is row fft_out_pos(tl, e) of
  // column g), so that the conjugate product is taken in the transform's
  // last stage instead of a pass of its own over the strip
  static_assert(SH::E == IT, "one transform's elements per thread");
  float2 aout[(FWD && K > 1) ? IT : 1];
  if constexpr (FWD && K > 1) {
    const bool colok = c0 + g < T::C;
#pragma unroll
    for (int e = 0; e < IT; ++e)
      aout[e] = colok ? A[(size_t)fft_out_pos<N, SH>(tl, e) * T::C + c0 + g] : make_float2(0.f, 0.f);
  }
#pragma unroll 1
  for (int kk = 0; kk < K; ++kk) {
    const int b = my * K + kk;
    if (b >= batch) break;  // uniform over the workgroup
    const size_t boff = (size_t)b * N * T::C;
    const float2* Ab = A + (size_t)b * (size_t)a_stride;
    if constexpr (FWD) {
      strip_load<N, G, SH>(S, B + boff, c0, bmask ? bmask + (size_t)b * kPlaneMaskWords<N> : nullptr);
      __syncthreads();
      if constexpr (K > 1) {
        auto at = [=](int x) { return S + T::idx(x, g); };
        fft_at<N, -1>(tl, tw, at, [&](int pos) { return *at(pos); },
                      [&](int pos, float2 v, int e) { *at(pos) = cmulc(aout[e], v); });
      } else {
        strip_fft<N, G, -1>(S, tw);
        __syncthreads();
        batched_copy<N * G, T::THREADS, float2>([&](int i) { return a_at(Ab, i); }, [&](int i, float2 a) {
          float2* e = &S[T::idx(i / G, i % G)];
          *e = cmulc(a, *e);
        });
      }
    } else {
      batched_copy<N * G, T::THREADS, float2>(
          [&](int i) {
            const int x = i / G, c = c0 + i % G;
            return (c < T::C) ? cmulc(Ab[(size_t)x * T::C + c], B[boff + (size_t)x * T::C + c]) : make_float2(0.f, 0.f);
          },
          [&](int i, float2 v) { S[T::idx(i / G, i % G)] = v; });
    }
    __syncthreads();
    strip_fft<N, G, +1>(S, tw);
    __syncthreads();
    strip_store<N, G, SH>(S, out + boff, c0);
    __syncthreads();
  }
}

// Score function of complex affinities (eq. 3 and eq. 5 with the reflection
// of the moving part, no conjugate): with rho = a + i b on each side and
// A_a, A_b, B_a, B_b the half spectra of the real channels, the product
// F{rho_1}(k) F{rho_2}(-k) splits into two Hermitian spectra,
//   Re: A_a conj(B_a) - A_b conj(B_b),   Im: A_a conj(B_b) + A_b conj(B_a),
// each followed here by the inverse x FFT. A2 = (A_a, A_b) at a stride of
// a_stride elements per batch member; B2 = batch x (B_a, B_b); out = batch x
// nparts spectra.
// BOTH = false: grid = (nstrips, batch, nparts), one part per workgroup (Re
// when blockIdx.z + first == 0, Im otherwise). BOTH = true: grid = (nstrips,
// batch), a workgroup reads the four spectra once and produces Re and Im:
// the Im products wait in registers while Re is transformed in LDS.
template <int N, int G, bool BOTH>
__global__ void __launch_bounds__((Strip<N, G>::THREADS)) k_strip_score(const float2* __restrict__ A2,
                                                                      long long a_stride,
                                                                      const float2* __restrict__ B2,
                                                                      float2* __restrict__ out, int first,
                                                                      const float2* __restrict__ table) {
  using T = Strip<N, G>;
  constexpr int IT = (N * G + T::THREADS - 1) / T::THREADS;  // strip elements per thread
  __shared__ float2 S[T::SIZE];
  Twiddles<N> tw;
  load_twiddles<N>(tw, table, (threadIdx.x & 63) % T::L);
  const size_t spec = (size_t)N * T::C;
  const int b = blockIdx.y;
  const float2* Aa = A2 + (size_t)b * (size_t)a_stride;
  const float2* Ab = Aa + spec;
  const float2* Ba = B2 + (size_t)b * 2 * spec;
  const float2* Bb = Ba + spec;
  const int c0 = blockIdx.x * G;
  if constexpr (BOTH) {
    float2 ireg[IT];
#pragma unroll
    for (int u = 0; u < IT; ++u) {
      const int i = threadIdx.x + u * T::THREADS;
      const int x = i / G, c = c0 + i % G;
      float2 re = make_float2(0.f, 0.f), im = make_float2(0.f, 0.f);
      if (i < N * G && c < T::C) {
        const size_t e = (size_t)x * T::C + c;
        const float2 aa = Aa[e], ab = Ab[e], ba = Ba[e], bb = Bb[e];
        const float2 p = cmulc(aa, ba), q = cmulc(ab, bb), r = cmulc(aa, bb), t = cmulc(ab, ba);
        re = make_float2(p.x - q.x, p.y - q.y);
        im = make_float2(r.x + t.x, r.y + t.y);
      }
      if (i < N * G) S[T::idx(x, i % G)] = re;
      ireg[u] = im;
    }
    __syncthreads();
    strip_fft<N, G, +1>(S, tw);
    __syncthreads();
    strip_store<N, G>(S, out + (size_t)b * 2 * spec, c0);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < IT; ++u) {
      const int i = threadIdx.x + u * T::THREADS;
      if (i < N * G) S[T::idx(i / G, i % G)] = ireg[u];
    }
    __syncthreads();
    strip_fft<N, G, +1>(S, tw);
    __syncthreads();
    strip_store<N, G>(S, out + ((size_t)b * 2 + 1) * spec, c0);
  } else {
    const bool re = (first + (int)blockIdx.z) == 0;
    batched_copy<N * G, T::THREADS, float2>(
        [&](int i) {
          const int x = i / G, c = c0 + i % G;
          if (c >= T::C) return make_float2(0.f, 0.f);
          const size_t e = (size_t)x * T::C + c;
          const float2 aa = Aa[e], ab = Ab[e], ba = Ba[e], bb = Bb[e];
          const float2 p = cmulc(aa, re ? ba : bb), q = cmulc(ab, re ? bb : ba);
          return re ? make_float2(p.x - q.x, p.y - q.y) : make_float2(p.x + q.x, p.y + q.y);
        },
        [&](int i, float2 v) { S[T::idx(i / G, i % G)] = v; });
    __syncthreads();
    strip_fft<N, G, +1>(S, tw);
    __syncthreads();
    strip_store<N, G>(S, out + ((size_t)b * gridDim.z + blockIdx.z) * spec, c0);
  }
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
  __shared__ float2 S[T::SIZE];
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
    S[T::idx(x, g)] = v;
  }
  __syncthreads();
  strip_fft<N, G, +1>(S, tw);
  __syncthreads();
  strip_store<N, G>(S, out7 + (size_t)o * spec, c0);
}

// The same 7 fields with the spectra read once per strip: grid = (nstrips,
// 2). Workgroup y = 0 keeps P_E = A conj(B_u) of its strip elements in
// registers and produces E, F_x, F_y, F_z (P_E and -2 pi i w_a P_E); y = 1
// keeps Q_b = A conj(M_b) and produces tau = 2 pi i (w x conj M) A, i.e.
// tau_x = 2 pi i (w_y Q_z - w_z Q_y) and cyclic. Each output is transformed
// along x in LDS in turn. Reads 6 spectra per strip instead of 35. The
// products take registers: two wavefronts per SIMD are enough here.
template <int N, int G>
__global__ void __launch_bounds__((Strip<N, G>::THREADS)) __attribute__((amdgpu_waves_per_eu(1, 2))) k_strip_ft_fields2(const float2* __restrict__ A,
                                                                           const float2* __restrict__ B4,
                                                                           float2* __restrict__ out7,
                                                                           const float2* __restrict__ table) {
  using T = Strip<N, G>;
  constexpr int IT = (N * G + T::THREADS - 1) / T::THREADS;
  __shared__ float2 S[T::SIZE];
  Twiddles<N> tw;
  load_twiddles<N>(tw, table, (threadIdx.x & 63) % T::L);
  const size_t spec = (size_t)N * T::C;
  const bool torque = blockIdx.y == 1;
  const int c0 = blockIdx.x * G;
  float2 q0[IT], q1[IT], q2[IT];
#pragma unroll
  for (int u = 0; u < IT; ++u) {
    const int i = threadIdx.x + u * T::THREADS;
    const int x = i / G, c = c0 + i % G;
    q0[u] = q1[u] = q2[u] = make_float2(0.f, 0.f);
    if (i < N * G && c < T::C) {
      const size_t e = (size_t)x * T::C + c;
      const float2 a = A[e];
      if (!torque) {
        q0[u] = cmulc(a, B4[e]);
      } else {
        q0[u] = cmulc(a, B4[spec + e]);
        q1[u] = cmulc(a, B4[2 * spec + e]);
        q2[u] = cmulc(a, B4[3 * spec + e]);
      }
    }
  }
  const int nout = torque ? 3 : 4;
#pragma unroll 1
  for (int k = 0; k < nout; ++k) {
#pragma unroll
    for (int u = 0; u < IT; ++u) {
      const int i = threadIdx.x + u * T::THREADS;
      if (i < N * G) {
        const int x = i / G, c = c0 + i % G;
        const float wx = omega_of<N>(x), wy = omega_of<N>(c / T::H), wz = omega_of<N>(c % T::H);
        float2 v;
        if (!torque) {
          const float2 p = q0[u];
          const float w = (k == 1) ? wx : (k == 2) ? wy : wz;
          // -2 pi i w P = 2 pi w (P.y, -P.x)
          v = (k == 0) ? p : make_float2(kTwoPi * w * p.y, -kTwoPi * w * p.x);
        } else {
          float2 ax;
          if (k == 0) ax = make_float2(wy * q2[u].x - wz * q1[u].x, wy * q2[u].y - wz * q1[u].y);
          else if (k == 1) ax = make_float2(wz * q0[u].x - wx * q2[u].x, wz * q0[u].y - wx * q2[u].y);
          else ax = make_float2(wx * q1[u].x - wy * q0[u].x, wx * q1[u].y - wy * q0[u].y);
          v = make_float2(-kTwoPi * ax.y, kTwoPi * ax.x);  // 2 pi i ax
        }
        S[T::idx(x, i % G)] = v;
      }
    }
    __syncthreads();
    strip_fft<N, G, +1>(S, tw);
    __syncthreads();
    strip_store<N, G>(S, out7 + (size_t)((torque ? 4 : 0) + k) * spec, c0);
    __syncthreads();
  }
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
  bool bad_pose = false;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float tf = poses[p * 3 + a];
    // nearest lattice point, ties away from zero; a translation that is not
    // finite or beyond 2^30 makes the pose's outputs NaN (bad_pose)
    bad_pose |= !(fabsf(tf) < 1073741824.0f);
    const long long ti = bad_pose ? 0 : (long long)roundf(tf) % N;
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
    part[((size_t)p * gridDim.x + blockIdx.x) * 7 + tid] = bad_pose ? __longlong_as_double(0x7ff8000000000000ll) : s;
  }
}

// Spectral gradient spectra of the stationary part: out3[a] = 2 pi i w_a Ahat
// (eq. 6a multiplier; the C2R that follows applies 1/N^3).
template <int N>
__global__ void k_grad_spectra(const float2* __restrict__ A, float2* __restrict__ out3) {
  constexpr int H = N / 2 + 1;
  const size_t spec = (size_t)N * N * H;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= spec) return;
  const int kz = (int)(e % H), ky = (int)((e / H) % N), kx = (int)(e / ((size_t)N * H));
  const float2 a = A[e];
  const float w3[3] = {omega_of<N>(kx), omega_of<N>(ky), omega_of<N>(kz)};
#pragma unroll
  for (int d = 0; d < 3; ++d) out3[d * spec + e] = make_float2(-kTwoPi * w3[d] * a.y, kTwoPi * w3[d] * a.x);
}

// Exact division of small non-negative integers through a float reciprocal
// with one correction step (the estimate is within one for v < 2^24).
__device__ __forceinline__ int divq(int v, int d, float rcp) {
  int q = (int)((float)v * rcp);
  q -= (q * d > v) ? 1 : 0;
  q += ((q + 1) * d <= v) ? 1 : 0;
  return q;
}

// Single-translation energy, force and torque by local sums over the moving
// part's balls (equal to the partial sum of eq. 7b: moving the spectral
// derivative from B to A is summation by parts, the multiplier being
// anti-Hermitian):
//   E = sum_q u_A(q + t) u_B(q),  F = -sum_q grad u_A(q + t) u_B(q),
//   tau = sum_q grad u_A(q + t) x yhat(q) u_B(q),
// u_B(q) = sum_j w_j K(|q - y_j|) on the torus, yhat the minimum-image
// coordinate. Item b = blockIdx.y, samples [blk*SPB, blk*SPB + SPB) of it;
// partials in float64 to part[(b*gridDim.x + blk)*7 + o]. block = 256.
constexpr int kLocalSPB = 64;
template <int N>
__global__ void __launch_bounds__(256) k_local_query(const QueryItem* __restrict__ items, double* __restrict__ part,
                                                     float sig_c, float e0, float inv1me0) {
  // a ball's box holds at most N^3 voxels (rho < N/2): divq needs < 2^24 and
  // the block's 64 boxes must sum below 2^31
  static_assert(N <= 256, "local query box sizes");
  __shared__ float4 sf[kLocalSPB];   // fx, fy, fz, w
  __shared__ int4 sb[kLocalSPB];     // bx, by, bz (B-frame voxel base), ez
  __shared__ int4 sl[kLocalSPB];     // box origin offsets lox, loy, loz, ey
  __shared__ float2 sr[kLocalSPB];   // rho^2, 1/(2 s^2)
  __shared__ int scnt[kLocalSPB + 1];
  __shared__ int sn;
  __shared__ double red[4][7];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const QueryItem& it = items[blockIdx.y];
  const long long s0 = (long long)blockIdx.x * kLocalSPB;
  if (tid == 0) sn = 0;
  __syncthreads();
  if (tid < kLocalSPB && s0 + tid < it.n_pts) {
    const float4 q = it.xyzr[s0 + tid];
    const float w = it.w[s0 + tid];
    const float rho = fmaxf(q.w, 1.0f);
    int cnt = 0;
    float fx = 0.f, fy = 0.f, fz = 0.f;
    int bx = 0, by = 0, bz = 0, lx = 0, ly = 0, lz = 0, ey = 0, ez = 0;
    if (rho < 0.5f * N && isfinite(w) && w != 0.0f) {
      const double dx0 = (double)q.x - (double)it.c[0], dy0 = (double)q.y - (double)it.c[1],
                   dz0 = (double)q.z - (double)it.c[2];
      const double yx = (double)it.R[0] * dx0 + (double)it.R[1] * dy0 + (double)it.R[2] * dz0;
      const double yy = (double)it.R[3] * dx0 + (double)it.R[4] * dy0 + (double)it.R[5] * dz0;
      const double yz = (double)it.R[6] * dx0 + (double)it.R[7] * dy0 + (double)it.R[8] * dz0;
      if (fabs(yx) < 1.0e7 && fabs(yy) < 1.0e7 && fabs(yz) < 1.0e7) {
        const double gx = floor(yx), gy = floor(yy), gz = floor(yz);
        fx = (float)(yx - gx);
        fy = (float)(yy - gy);
        fz = (float)(yz - gz);
        long long ix = (long long)gx % N, iy = (long long)gy % N, iz = (long long)gz % N;
        bx = (int)(ix < 0 ? ix + N : ix);
        by = (int)(iy < 0 ? iy + N : iy);
        bz = (int)(iz < 0 ? iz + N : iz);
        lx = (int)ceilf(fx - rho);
        ly = (int)ceilf(fy - rho);
        lz = (int)ceilf(fz - rho);
        const int ex = (int)floorf(fx + rho) - lx + 1;
        ey = (int)floorf(fy + rho) - ly + 1;
        ez = (int)floorf(fz + rho) - lz + 1;
        cnt = ex * ey * ez;
      }
    }
    sf[tid] = make_float4(fx, fy, fz, w);
    sb[tid] = make_int4(bx, by, bz, ez);
    sl[tid] = make_int4(lx, ly, lz, ey);
    sr[tid] = make_float2(rho * rho, sig_c / (rho * rho));
    scnt[tid] = cnt;
    atomicMax(&sn, tid + 1);
  }
  __syncthreads();
  const int ns = sn;
  if (tid < 64) {  // exclusive scan of the box sizes (ns <= 64)
    const int v = (tid < ns) ? scnt[tid] : 0;
    int incl = v;
    for (int d = 1; d < 64; d <<= 1) {
      const int o = __shfl_up(incl, d, 64);
      if (tid >= d) incl += o;
    }
    if (tid < ns) scnt[tid] = incl - v;
    if (tid == 63) scnt[ns] = incl;
  }
  __syncthreads();
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  const int V = (ns > 0) ? scnt[ns] : 0;
  const int per = (((V + 3) / 4) + 63) & ~63;  // contiguous voxel range per wave
  const int g0 = wave * per, g1 = min(V, g0 + per);
  if (g0 < g1) {
    int lo = 0, hi = ns - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (scnt[mid] <= g0) lo = mid;
      else hi = mid - 1;
    }
    int h = lo;
    for (int gb = g0; gb < g1; gb += 64) {
      const int g = gb + lane;
      if (g < g1) {
        while (scnt[h + 1] <= g) ++h;
        const int v = g - scnt[h];
        const int4 b = sb[h], l = sl[h];
        const int eyz = l.w * b.w;
        const int ox = divq(v, eyz, __builtin_amdgcn_rcpf((float)eyz));
        const int rem = v - ox * eyz;
        const int oy = divq(rem, b.w, __builtin_amdgcn_rcpf((float)b.w));
        const int oz = rem - oy * b.w;
        const float4 f = sf[h];
        const float dx = (float)(l.x + ox) - f.x, dy = (float)(l.y + oy) - f.y, dz = (float)(l.z + oz) - f.z;
        const float2 r = sr[h];
        const float d2 = dx * dx + dy * dy + dz * dz;
        if (d2 < r.x) {
          const float cval = f.w * (__expf(-d2 * r.y) - e0) * inv1me0;  // w K(d): u_B contribution at q
          const int qx = wrapn(b.x + l.x + ox, N), qy = wrapn(b.y + l.y + oy, N), qz = wrapn(b.z + l.z + oz, N);
          const int px = wrapn(qx + it.t[0], N), py = wrapn(qy + it.t[1], N), pz = wrapn(qz + it.t[2], N);
          const float4 fa = it.FA[((size_t)px * N + py) * N + pz];
          const float hx = yhat(qx, N), hy = yhat(qy, N), hz = yhat(qz, N);
          acc[0] += (double)(cval * fa.x);
          acc[1] -= (double)(cval * fa.y);
          acc[2] -= (double)(cval * fa.z);
          acc[3] -= (double)(cval * fa.w);
          acc[4] += (double)(cval * (fa.z * hz - fa.w * hy));
          acc[5] += (double)(cval * (fa.w * hx - fa.y * hz));
          acc[6] += (double)(cval * (fa.y * hy - fa.z * hx));
        }
      }
    }
  }
#pragma unroll
  for (int o = 0; o < 7; ++o) {
    double v = acc[o];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) red[wave][o] = v;
  }
  __syncthreads();
  if (tid < 7) part[((size_t)blockIdx.y * gridDim.x + blockIdx.x) * 7 + tid] = red[0][tid] + red[1][tid] + red[2][tid] +
                                                                              red[3][tid];
}

// ---------------------------------------------------------------------------
// Separate-axis path (grid edges whose x-plane does not fit in LDS, e.g.
// 512^3, and any plan created with GA_PLAN_AXIS_PASSES): splat into a real
// grid, z transforms per row pair, y and x transforms per strip of columns.
// ---------------------------------------------------------------------------

// Splat with global float atomics: one wavefront per sample, its bounding box
// walked 64 voxels at a time. grid = (ceil(n_pts / 4), batch), block = 256.
// out[(b * nch + c) * N^3 + (x * N + y) * N + z] must be zero beforehand;
// channels u, yhat_x u, yhat_y u, yhat_z u.
template <int N>
__global__ void __launch_bounds__(256) k_splat_atomic(SplatParams p, int nch, float* __restrict__ out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long s = (long long)blockIdx.x * 4 + wave;
  const int b = blockIdx.y;
  if (s >= p.n_pts) return;  // uniform over the wavefront
  double R[9];
  load_rotation(p, b, R);
  Placed q;
  if (!place_sample<N>(p, R, s, q)) return;
  const float w = __int_as_float(q.b.w);
  if (w == 0.0f) return;
  const float rho = q.a.w, fx = q.a.x, fy = q.a.y, fz = q.a.z;
  const int lx = (int)ceilf(fx - rho), ly = (int)ceilf(fy - rho), lz = (int)ceilf(fz - rho);
  const int ex = (int)floorf(fx + rho) - lx + 1, ey = (int)floorf(fy + rho) - ly + 1, ez = (int)floorf(fz + rho) - lz + 1;
  const int eyz = ey * ez, V = ex * eyz;
  const float r2 = rho * rho, inv2s2 = p.sig_c / r2;
  const size_t n3 = (size_t)N * N * N;
  float* base = out + (size_t)b * nch * n3;
  for (int v = lane; v < V; v += 64) {
    const int ox = v / eyz, rem = v - ox * eyz, oy = rem / ez, oz = rem - oy * ez;
    const float dx = (float)(lx + ox) - fx, dy = (float)(ly + oy) - fy, dz = (float)(lz + oz) - fz;
    const float d2 = dx * dx + dy * dy + dz * dz;
    if (d2 < r2) {
      const float val = w * (__expf(-d2 * inv2s2) - p.e0) * p.inv1me0;
      const int xx = wrapn(q.b.x + lx + ox, N), yy = wrapn(q.b.y + ly + oy, N), zz = wrapn(q.b.z + lz + oz, N);
      const size_t o = ((size_t)xx * N + yy) * N + zz;
      atomicAdd(base + o, val);
      if (nch == 4) {
        atomicAdd(base + n3 + o, yhat(xx, N) * val);
        atomicAdd(base + 2 * n3 + o, yhat(yy, N) * val);
        atomicAdd(base + 3 * n3 + o, yhat(zz, N) * val);
      }
    }
  }
}

// z transforms of real rows, two rows (y, y+1 of one plane) per complex
// transform: out[(plane * N + y) * H + kz] for kz in [0, N/2]. Transform tr
// of nrp = planes * N/2; 4 wavefronts per workgroup.
template <int N> struct Rows {
  static constexpr int H = N / 2 + 1;
  static constexpr int L = lanes_per_fft<N>();
  static constexpr int TPW = ffts_per_wave<N>();
  static constexpr int PER_WG = 4 * TPW;
  static constexpr int REG = N + 8;  // LDS slots per transform
  // position p of a transform: XOR of the low 3 bits with bits 3-5 spreads
  // the radix-strided stage patterns over bank pairs
  __device__ __forceinline__ static int sw(int p) { return p ^ ((p >> 3) & 7); }
};

template <int N>
__global__ void __launch_bounds__(256) k_rows_fwd(const float* __restrict__ in, float2* __restrict__ out, long long nrp,
                                                  const float2* __restrict__ table) {
  using RW = Rows<N>;
  constexpr int L = RW::L, H = RW::H;
  __shared__ float2 S[RW::PER_WG * RW::REG];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, l = lane % L;
  const int slot = wave * RW::TPW + lane / L;
  const long long tr = (long long)blockIdx.x * RW::PER_WG + slot;
  Twiddles<N> tw;
  load_twiddles<N>(tw, table, l);
  if (tr >= nrp) return;  // whole transforms only: every lane of a transform agrees
  const long long plane = tr / (N / 2);
  const int y0 = 2 * (int)(tr % (N / 2));
  const float* r0 = in + ((size_t)plane * N + y0) * N;
  float2* reg = S + slot * RW::REG;
  auto at = [=](int pos) { return reg + RW::sw(pos); };
  auto ld = [&](int pos) { return make_float2(r0[pos], r0[N + pos]); };
  auto st = [&](int pos, float2 v) { *at(pos) = v; };
  fft_at<N, -1>(l, tw, at, ld, st);
  float2* o0 = out + ((size_t)plane * N + y0) * H;
  for (int k = l; k < H; k += L) {
    const float2 a = *at(k % N);
    const float2 z = *at((N - k) % N);
    o0[k] = make_float2(0.5f * (a.x + z.x), 0.5f * (a.y - z.y));
    o0[H + k] = make_float2(0.5f * (a.y + z.y), -0.5f * (a.x - z.x));
  }
}

// Inverse of k_rows_fwd: out[(plane * N + y) * N + z] = scale * (C2R of
// row y's half spectrum), two rows per complex transform (imaginary parts at
// kz = 0 and kz = N/2 dropped).
template <int N>
__global__ void __launch_bounds__(256) k_rows_inv(const float2* __restrict__ in, float* __restrict__ out, float scale,
                                                  long long nrp, const float2* __restrict__ table) {
  using RW = Rows<N>;
  constexpr int L = RW::L, H = RW::H;
  __shared__ float2 S[RW::PER_WG * RW::REG];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, l = lane % L;
  const int slot = wave * RW::TPW + lane / L;
  const long long tr = (long long)blockIdx.x * RW::PER_WG + slot;
  Twiddles<N> tw;
  load_twiddles<N>(tw, table, l);
  if (tr >= nrp) return;
  const long long plane = tr / (N / 2);
  const int y0 = 2 * (int)(tr % (N / 2));
  const float2* a0 = in + ((size_t)plane * N + y0) * H;
  const float2* b0 = a0 + H;
  float2* reg = S + slot * RW::REG;
  auto at = [=](int pos) { return reg + RW::sw(pos); };
  auto ld = [&](int k) -> float2 {
    if (k < H) {
      float2 a = a0[k], bb = b0[k];
      if (k == 0 || k == N / 2) {
        a.y = 0.f;
        bb.y = 0.f;
      }
      return make_float2(a.x - bb.y, a.y + bb.x);
    }
    const float2 a = a0[N - k], bb = b0[N - k];
    return make_float2(a.x + bb.y, bb.x - a.y);
  };
  float* r0 = out + ((size_t)plane * N + y0) * N;
  auto st = [&](int k, float2 v) {
    r0[k] = v.x * scale;
    r0[N + k] = v.y * scale;
  };
  fft_at<N, +1>(l, tw, at, ld, st);
}

// Transform along a strided axis, G columns per workgroup: element (pos, c)
// of plane pl at pl * plane_stride + pos * stride + c, c < ncols. grid =
// (ceil(ncols / G), planes). In place when in == out (each workgroup reads
// all of its strip before writing it).
template <int N, int G, int DIR>
__global__ void __launch_bounds__((Strip<N, G>::THREADS)) k_pencil_fft(const float2* in, float2* out, long long stride,
                                                                     int ncols, long long plane_stride,
                                                                     const float2* __restrict__ table) {
  using T = Strip<N, G>;
  __shared__ float2 S[T::SIZE];
  Twiddles<N> tw;
  load_twiddles<N>(tw, table, (threadIdx.x & 63) % T::L);
  const size_t off = (size_t)blockIdx.y * (size_t)plane_stride;
  const int c0 = blockIdx.x * G;
  batched_copy<N * G, T::THREADS, float2>(
      [&](int i) {
        const int x = i / G, c = c0 + i % G;
        return (c < ncols) ? in[off + (size_t)x * stride + c] : make_float2(0.f, 0.f);
      },
      [&](int i, float2 v) { S[T::idx(i / G, i % G)] = v; });
  __syncthreads();
  strip_fft<N, G, DIR>(S, tw);
  __syncthreads();
  for (int i = threadIdx.x; i < N * G; i += T::THREADS) {
    const int x = i / G, g = i % G, c = c0 + g;
    if (c < ncols) out[off + (size_t)x * stride + c] = S[T::idx(x, g)];
  }
}

// Kernels without template parameters get internal linkage: the header is
// included by more than one translation unit.
namespace {

// Zero n4 float4 values (grid-stride loop).
__global__ void k_zero4(float4* __restrict__ p, long long n4) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (long long)gridDim.x * blockDim.x)
    p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// The periodic lattice cell of coordinate t: lower corner i0 and upper corner
// i1 = i0 + 1 (both mod n, in [0, n)) and the fraction a = t - floor(t). The
// quotient by n comes from a float division, off by at most one for
// |t| < 2^24 n and then corrected (a 64-bit remainder as the last resort), so
// the corners are always inside the grid.
// A coordinate that is not finite or whose magnitude reaches 2^24 n (beyond
// which float32 holds no fraction) is not converted at all: corners 0 and 1
// and a NaN fraction, so that the interpolated outputs are NaN.
__device__ __forceinline__ void lattice_cell(float t, int n, int& i0, int& i1, float& a) {
  if (!(fabsf(t) < 16777216.0f * (float)n)) {  // also false for NaN
    i0 = 0;
    i1 = 1 % n;
    a = __int_as_float(0x7fc00000);
    return;
  }
  const float fl = floorf(t);
  a = t - fl;
  long long m = (long long)fl - (long long)floorf(fl / (float)n) * n;
  if (m < 0) m += n;
  if (m >= n) m -= n;
  if (m < 0 || m >= n) {
    m = (long long)fl % n;
    if (m < 0) m += n;
  }
  i0 = (int)m;
  i1 = (i0 + 1 == n) ? 0 : i0 + 1;
}

// Queries of precomputed field tables: query q reads the 32-byte records of
// orientation orient[q] (tables + orient * 8 * n^3 floats, [x][y][z][8])
// trilinearly at t[q] (periodic): two 16-byte loads per corner. An
// orientation index outside [0, n_orient) gives NaN outputs. One thread per
// query.
__global__ void k_table_query(const float4* __restrict__ tables, int n, int n_orient, const int* __restrict__ orient,
                              const float* __restrict__ poses, int n_q, float* __restrict__ out7) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_q) return;
  const int ori = orient[q];
  if (ori < 0 || ori >= n_orient) {
    for (int o = 0; o < 7; ++o) out7[q * 7 + o] = __int_as_float(0x7fc00000);
    return;
  }
  const size_t n3 = (size_t)n * n * n;
  const float4* f = tables + (size_t)ori * 2 * n3;
  float a[3];
  int i0[3], i1[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) lattice_cell(poses[q * 3 + d], n, i0[d], i1[d], a[d]);
  float4 lo = make_float4(0.f, 0.f, 0.f, 0.f), hi = lo;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int dx = c >> 2, dy = (c >> 1) & 1, dz = c & 1;
    const float w = (dx ? a[0] : 1.f - a[0]) * (dy ? a[1] : 1.f - a[1]) * (dz ? a[2] : 1.f - a[2]);
    const size_t v = ((size_t)(dx ? i1[0] : i0[0]) * n + (dy ? i1[1] : i0[1])) * n + (dz ? i1[2] : i0[2]);
    const float4 r0 = f[2 * v], r1 = f[2 * v + 1];
    lo.x += w * r0.x;
    lo.y += w * r0.y;
    lo.z += w * r0.z;
    lo.w += w * r0.w;
    hi.x += w * r1.x;
    hi.y += w * r1.y;
    hi.z += w * r1.z;
  }
  float* o = out7 + (size_t)q * 7;
  o[0] = lo.x;
  o[1] = lo.y;
  o[2] = lo.z;
  o[3] = lo.w;
  o[4] = hi.x;
  o[5] = hi.y;
  o[6] = hi.z;
}

// Low-pass filtering of half spectra (Sec. 3.3): modes with |kappa(k_a)| <=
// L/2 - 1 on every axis are kept (times scale), the rest are dropped.
// coarse = 1: out is [batch][L][L][L/2+1] (the kept modes on an L grid);
// coarse = 0: out is [batch][n][n][n/2+1] with the dropped modes zero.
// grid = (runs of one output kx plane, output kx, batch members strided by
// gridDim.z); 32-bit index arithmetic within a plane.
__global__ void k_lowpass(const float2* __restrict__ in, float2* __restrict__ out, int n, int L, int coarse,
                          int batch, float scale) {
  const int hn = n / 2 + 1, m = coarse ? L : n, hm = m / 2 + 1;
  const int lim = L / 2 - 1;
  const int kx = blockIdx.y;
  const int ax = kx < m / 2 ? kx : kx - m;  // signed frequency
  const bool xin = ax <= lim && ax >= -lim;
  const int sx = ax < 0 ? ax + n : ax;
  const int plane = m * hm;
  for (int b = blockIdx.z; b < batch; b += gridDim.z) {
    const float2* src = in + (size_t)b * n * n * hn + (size_t)sx * n * hn;
    float2* dst = out + ((size_t)b * m + kx) * plane;
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < plane; r += gridDim.x * blockDim.x) {
      const int ky = r / hm, kz = r - ky * hm;
      const int ay = ky < m / 2 ? ky : ky - m;
      float2 v = make_float2(0.f, 0.f);
      if (xin && ay <= lim && ay >= -lim && kz <= lim) {
        const float2 a = src[(size_t)(ay < 0 ? ay + n : ay) * hn + kz];
        v = make_float2(a.x * scale, a.y * scale);
      }
      dst[r] = v;
    }
  }
}

// Sum of the per-strip partials of each pose in a fixed order, times scale.
// grid = n_poses, block = 64.
__global__ void __launch_bounds__(64) k_reduce_partials(const double* __restrict__ part, int nblk, float* __restrict__ out7,
                                                        double scale, const QueryItem* __restrict__ items) {
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
    const bool bad = items && items[p].pad != 0;  // a translation that could not be converted
    out7[p * 7 + tid] = bad ? __int_as_float(0x7fc00000) : (float)(s * scale);
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
  float a[3];
  int i0[3], i1[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) lattice_cell(poses[p * 3 + d], n, i0[d], i1[d], a[d]);
  float acc = 0.f;
#pragma unroll
  for (int dx = 0; dx < 2; ++dx)
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
      for (int dz = 0; dz < 2; ++dz) {
        const float wgt = (dx ? a[0] : 1.f - a[0]) * (dy ? a[1] : 1.f - a[1]) * (dz ? a[2] : 1.f - a[2]);
        const int ix = dx ? i1[0] : i0[0], iy = dy ? i1[1] : i0[1], iz = dz ? i1[2] : i0[2];
        acc += wgt * f[((size_t)ix * n + iy) * n + iz];
      }
  out7[p * 7 + o] = acc;
}

// Interleaves u and its three gradient fields into one float4 per voxel.
__global__ void k_pack4(const float* __restrict__ u, const float* __restrict__ g3, float4* __restrict__ FA,
                        long long n3) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n3) FA[i] = make_float4(u[i], g3[i], g3[n3 + i], g3[2 * n3 + i]);
}

// Interleaves 7 real fields [7][n3] into one 32-byte record per voxel
// (E, F_x, F_y, F_z, tau_x, tau_y, tau_z, 0): the field-table layout.
__global__ void k_pack8(const float* __restrict__ f7, float4* __restrict__ out, long long n3) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n3; i += (long long)gridDim.x * blockDim.x) {
    out[2 * i] = make_float4(f7[i], f7[n3 + i], f7[2 * n3 + i], f7[3 * n3 + i]);
    out[2 * i + 1] = make_float4(f7[4 * n3 + i], f7[5 * n3 + i], f7[6 * n3 + i], 0.f);
  }
}

// Query descriptors for a batch of (rotation, translation) poses of one part:
// t rounded to the nearest lattice point (ties away from zero) mod n.
__global__ void k_make_items(QueryItem* __restrict__ items, int batch, const float4* xyzr, const float* w,
                             long long n_pts, const float4* FA, const float2* AX, const float* __restrict__ R,
                             const float* __restrict__ t, float c0, float c1, float c2, int n) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  QueryItem it;
  it.xyzr = xyzr;
  it.w = w;
  it.n_pts = n_pts;
  it.AX = AX;
  it.FA = FA;
  for (int i = 0; i < 9; ++i) it.R[i] = R[b * 9 + i];
  it.c[0] = c0;
  it.c[1] = c1;
  it.c[2] = c2;
  it.pad = 0;
  for (int a = 0; a < 3; ++a) {
    const float tf = t[b * 3 + a];
    const bool ok = fabsf(tf) < 1073741824.0f;  // finite and convertible
    long long v = ok ? (long long)roundf(tf) % n : 0;
    it.t[a] = (int)(v < 0 ? v + n : v);
    if (!ok) it.pad = 1;  // the pose's outputs become NaN (k_reduce_partials)
  }
  items[b] = it;
}

}  // namespace

}  // namespace ga
