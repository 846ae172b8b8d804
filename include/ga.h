/*
 * ga.h -- C ABI of the geometric-energy correlation library (libga.so).
 *
 * The library computes, on one MI355X (gfx950), the hot path of the
 * skeletal-density correlation method for haptic assembly (Behandish & Ilies,
 * "Haptic Assembly Using Skeletal Densities and Fourier Transforms"):
 *
 *   skeleton samples --splat--> real density on an n^3 grid
 *                   --R2C 3D FFT--> half spectrum
 *   conj product with the stationary part's spectrum (+ spectral-gradient
 *   multipliers) --C2R 3D FFT--> energy, force and torque over all
 *   translations, read out at poses.
 *
 * Conventions shared by every call
 *   - Grid: n^3 voxels with centres at integer coordinates (dV = 1), stored
 *     x-major, z fastest: element (x, y, z) at (x*n + y)*n + z. Periodic.
 *   - Half spectrum ("spectrum" below): complex float32 interleaved (re, im),
 *     n x n x (n/2+1), element (kx, ky, kz) at (kx*n + ky)*(n/2+1) + kz.
 *   - Forward transform: X(k) = sum_p x(p) exp(-2 pi i k.p/n), unnormalised
 *     (Sec. 3.2, eq. 7a with dV = 1). Inverse: exp(+2 pi i k.p/n) and 1/n^3
 *     (eq. 7b; the paper leaves the constant to the convention).
 *   - Skeleton samples: float32 (x, y, z, r) per sample, r the ball radius in
 *     voxels, plus a float32 signed weight w. The density is
 *     u(p) = sum_j w_j K(|p - y_j|; r_j) with the truncated Gaussian
 *     K(d) = (exp(-d^2/2s^2) - exp(-rho^2/2s^2)) / (1 - exp(-rho^2/2s^2)) for
 *     d < rho, 0 beyond, rho = max(r, 1), s = sigma*rho (the skeletal density
 *     of Sec. 2.3, modelled on medial-ball samples). Distances are minimum
 *     image on the torus. Every sample needs rho < n/2 and finite values; a
 *     sample that violates this contributes nothing.
 *   - Motion (Sec. 2.4): the moving part B is rotated by R (3x3 row-major,
 *     proper orthogonal) about its reference point c and placed with c at the
 *     grid origin, y_j = R (x_j - c). The translation t is the position of c
 *     in the stationary part's grid frame, in voxels.
 *   - Energy E(t) = sum_p u_A(p) u_B(p - t) (eq. 1/3, computed as eq. 5; for
 *     real densities the reflection is the complex conjugate). Force
 *     F = -dE/dt (eq. 6a). Torque tau = -dE/dtheta about c for a space-frame
 *     rotation of B (eq. 6b with the moment density rho*(p) = rho(p) p).
 *     The spectral derivative multiplies by 2 pi i kappa(k)/n with kappa = 0 on
 *     each axis's Nyquist index.
 *
 * Memory and streams
 *   - Every d_* pointer is device memory owned by the caller; it must stay
 *     valid until the work queued on `stream` has finished. The library never
 *     frees or keeps caller pointers. Host pointers are read before the call
 *     returns.
 *   - Calls that need scratch device memory take a caller-owned workspace
 *     (d_work, work_bytes); ga_workspace_size() returns the bytes needed.
 *   - Every compute call only enqueues work on `stream` (a hipStream_t; 0 is
 *     the null stream) and returns; argument errors are reported
 *     synchronously, launch errors as GA_EDEVICE.
 *
 * Errors: every call returns a ga_status; ga_status_str() gives its text.
 */
#ifndef GA_H
#define GA_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ga_status;

#define GA_OK 0
#define GA_PENDING 1        /* ticket not finished yet */
#define GA_EINVAL (-1)      /* bad argument: null pointer, size, grid edge, mode */
#define GA_ENOMEM (-2)      /* allocation failed, workspace too small or budget exceeded */
#define GA_EAGAIN (-3)      /* queue full, try again */
#define GA_EDEVICE (-4)     /* HIP runtime or launch error */
#define GA_ENOTFOUND (-5)   /* unknown ticket or pair */
#define GA_EUNSUPPORTED (-6) /* grid edge not supported by this build */

/* Transform directions for ga_fft3d. */
#define GA_R2C (-1)
#define GA_C2R (+1)

/* Readout modes for ga_force_torque. */
#define GA_FIELDS 0u /* 7 fields over all translations, trilinear readout at poses */
#define GA_SINGLE 1u /* one partial sum of eq. 7b per pose at the nearest lattice point */

/* Operations for ga_workspace_size. */
#define GA_OP_FFT_C2R 1
#define GA_OP_CORRELATE 2
#define GA_OP_ENERGY 3
#define GA_OP_FORCE_FIELDS 4
#define GA_OP_FORCE_SINGLE 5

typedef struct ga_plan ga_plan;

/* Text for a status code (static storage). */
const char* ga_status_str(ga_status s);

/* Library version string (static storage). */
const char* ga_version(void);

/* Whether grid edge n is supported by this build (1) or not (0). */
int32_t ga_supported_n(int32_t n);

/*
 * Plan for grid edge n on the current HIP device (Sec. 3.2: the transforms of
 * eq. 7a/7b on an n^3 grid). n must be even and of the form 2^a 3^b; see
 * ga_supported_n(). The plan owns the float32 twiddle table, computed in
 * float64 on the host. max_batch bounds the batch of later calls. flags: 0.
 * On success *plan is set; release with ga_plan_destroy.
 */
ga_status ga_plan_create(ga_plan** plan, int32_t n, int32_t max_batch, uint32_t flags);
ga_status ga_plan_destroy(ga_plan* plan);
int32_t ga_plan_n(const ga_plan* plan);

/* Workspace bytes that operation `op` needs for `batch` fields; n_items is
 * the number of skeleton samples for GA_OP_ENERGY and the number of poses
 * for GA_OP_FORCE_SINGLE (ignored otherwise). 0 for an unknown op. */
size_t ga_workspace_size(const ga_plan* plan, int32_t op, int32_t batch, int64_t n_items);

/*
 * Splat (Sec. 2.3 skeletal density, modelled; Sec. 2.4 rotation about c):
 * writes `channels` real n^3 grids to d_grid: channel 0 is u; with
 * channels = 4, channels 1..3 are the moment density yhat_b(q) u(q) of
 * eq. 6b, yhat the minimum-image coordinate of grid index q (q for q < n/2,
 * q - n otherwise). h_R (9 floats, row-major) and h_c (3 floats) are host
 * arrays; pass h_R = NULL and h_c = NULL for the identity placement (grid
 * coordinates used as given, the stationary part). d_xyzr: n_pts x 4 floats,
 * d_w: n_pts floats. sigma > 0. n_pts = 0 gives zero grids.
 */
ga_status ga_splat(const ga_plan* plan, const float* d_xyzr, const float* d_w, int64_t n_pts,
                   const float* h_R, const float* h_c, float sigma, int32_t channels,
                   float* d_grid, hipStream_t stream);

/*
 * 3D FFT of `batch` grids, out of place (eq. 7a / 7b).
 *   GA_R2C: d_in real n^3 grids -> d_out half spectra, unnormalised.
 *   GA_C2R: d_in half spectra -> d_out real grids, exp(+) and 1/n^3. On the
 *           kz = 0 and kz = n/2 planes only the Hermitian part of the input is
 *           used (the real field whose spectrum is closest to the input).
 * GA_C2R needs a workspace of ga_workspace_size(plan, GA_OP_FFT_C2R, batch, 0).
 */
ga_status ga_fft3d(const ga_plan* plan, int32_t dir, const void* d_in, void* d_out, int32_t batch,
                   void* d_work, size_t work_bytes, hipStream_t stream);

/*
 * Energy fields from spectra (eq. 5): E_b = C2R(Ahat_b conj(Bhat_b)), i.e.
 * E_b(t) = sum_p u_A(p) u_B,b(p - t). d_Ahat is read with a stride of
 * a_stride spectrum elements between batch members (0 = one Ahat for all).
 * d_E: batch real n^3 grids. Workspace: GA_OP_CORRELATE.
 */
ga_status ga_correlate(const ga_plan* plan, const float* d_Ahat, int64_t a_stride, const float* d_Bhat,
                       int32_t batch, float* d_E, void* d_work, size_t work_bytes, hipStream_t stream);

/*
 * The whole field path for many rotations of the moving part in one call
 * (Sec. 3.2 real-time sequence with the rotation applied by re-splatting, and
 * eq. 5): for each b < batch, B's samples are rotated by d_R[b] (device,
 * batch x 9 floats) about h_c, splatted, transformed, multiplied by
 * conj with the resident d_Ahat (one spectrum of the stationary part) and
 * transformed back into the energy field d_E[b] (batch x n^3 floats).
 * Workspace: GA_OP_ENERGY with n_items = n_pts.
 */
ga_status ga_energy_fields(const ga_plan* plan, const float* d_Ahat, const float* d_xyzr, const float* d_w,
                           int64_t n_pts, const float* d_R, const float* h_c, float sigma, int32_t batch,
                           float* d_E, void* d_work, size_t work_bytes, hipStream_t stream);

/*
 * Energy, force and torque at poses (eq. 5, 6a, 6b; Sec. 2.4 readout).
 * d_Ahat: spectrum of the stationary part. d_Bhat4: 4 spectra of the placed
 * moving part (u, m_x, m_y, m_z; from ga_splat with channels = 4 and
 * ga_fft3d). d_t: n_poses x 3 floats (translation of c in voxels). d_out7:
 * n_poses x 7 floats (E, F_x, F_y, F_z, tau_x, tau_y, tau_z).
 *   GA_FIELDS: the 7 fields over all translations (7 C2R transforms), then
 *              trilinear interpolation between the 8 periodic lattice
 *              neighbours of t (exact at lattice points).
 *   GA_SINGLE: for each pose, the partial sum of eq. 7b at the single
 *              translation round(t) (nearest lattice point, ties away from
 *              zero, float32 rounding), accumulated in float64 (Sec. 3.3).
 * Workspace: GA_OP_FORCE_FIELDS or GA_OP_FORCE_SINGLE.
 */
ga_status ga_force_torque(const ga_plan* plan, const float* d_Ahat, const float* d_Bhat4, const float* d_t,
                          int32_t n_poses, uint32_t mode, float* d_out7, void* d_work, size_t work_bytes,
                          hipStream_t stream);

/*
 * Per-kernel timing. With profiling enabled, every kernel the plan launches
 * is bracketed by two HIP events recorded on its launch stream.
 * ga_profile_read waits for the recorded events and returns, for one kernel
 * kind, the summed duration in milliseconds and the number of launches since
 * profiling was enabled (enabling again clears the totals). Not thread-safe:
 * use one plan per thread while profiling.
 */
#define GA_K_SPLAT 0     /* density splat (ga_splat) */
#define GA_K_PLANE_FWD 1 /* pass 1: splat or load, z R2C and y FFT per x-plane */
#define GA_K_STRIP 2     /* pass 2: x FFT per column strip (with products) */
#define GA_K_PLANE_INV 3 /* pass 3: inverse y FFT and z C2R per x-plane */
#define GA_K_READOUT 4   /* force/torque products, partial sums, readout */
#define GA_K_BIN 5       /* placement and binning of the moving part's samples */
#define GA_K_COUNT 6

ga_status ga_profile_enable(ga_plan* plan, int32_t enable);
ga_status ga_profile_read(ga_plan* plan, int32_t kind, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* GA_H */
