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
 *   - Grids, spectra, sample arrays (d_xyzr), tables and workspaces are read
 *     and written with 16-byte vector accesses and must be 16-byte aligned
 *     (hipMalloc and torch allocations are); a misaligned one gives
 *     GA_EINVAL. Weights, rotations, poses and pose outputs need only float
 *     alignment.
 *   - Calls that need scratch device memory take a caller-owned workspace
 *     (d_work, work_bytes); ga_workspace_size() returns the bytes needed.
 *   - Every compute call only enqueues work on `stream` (a hipStream_t; 0 is
 *     the null stream) and returns; argument errors are reported
 *     synchronously, launch errors as GA_EDEVICE.
 *   - A plan holds no per-call device state except the events of its
 *     overlapped execution (ga_plan_set_overlap) and its profiling records:
 *     with either in use, one host thread at a time calls with a given plan.
 *     Otherwise compute calls on one plan from several threads are safe.
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
#define GA_EUNSUPPORTED (-6) /* grid edge not compiled into the library */

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
#define GA_OP_FIELD_GRAD 6
#define GA_OP_POSE_LOCAL 7
#define GA_OP_SCORE 8
#define GA_OP_POSE_SPECTRAL 9

/* Plan flags. */
#define GA_PLAN_AXIS_PASSES 1u /* separate-axis path at every grid edge */

typedef struct ga_plan ga_plan;

/* Text for a status code (static storage). */
const char* ga_status_str(ga_status s);

/* Library version string (static storage). */
const char* ga_version(void);

/* Whether grid edge n is compiled into the library (1) or not (0). */
int32_t ga_supported_n(int32_t n);

/*
 * Plan for grid edge n on the current HIP device (Sec. 3.2: the transforms of
 * eq. 7a/7b on an n^3 grid). n must be even and of the form 2^a 3^b; see
 * ga_supported_n(). The plan owns the float32 twiddle table, computed in
 * float64 on the host. max_batch bounds the batch of later calls.
 *
 * Execution paths. For n <= 192 one x-plane of the spectrum fits in LDS and
 * the transforms run in three HBM passes (splat + z + y per plane, x per
 * strip of columns, y + z per plane). For n = 256, 384, 512, or with flags =
 * GA_PLAN_AXIS_PASSES at any n, the separate-axis path runs instead: splat
 * into real grids with float atomics, z transforms per row pair, y and x
 * transforms per strip of columns (same results, more HBM passes; the C-ABI
 * calls are unchanged, but ga_pose_local needs n <= 256 and the serving loop
 * the plane path). flags: 0 or GA_PLAN_AXIS_PASSES.
 * On success *plan is set; release with ga_plan_destroy.
 */
ga_status ga_plan_create(ga_plan** plan, int32_t n, int32_t max_batch, uint32_t flags);
ga_status ga_plan_destroy(ga_plan* plan);
int32_t ga_plan_n(const ga_plan* plan);

/* Workspace bytes that operation `op` needs for `batch` fields (or poses for
 * GA_OP_POSE_LOCAL); n_items is the number of skeleton samples for
 * GA_OP_ENERGY and GA_OP_POSE_LOCAL and the number of poses for
 * GA_OP_FORCE_SINGLE, and the number of parts (1 or 2) for GA_OP_SCORE
 * (ignored otherwise). 0 for an unknown op. */
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

/* Parts of the complex score (ga_score). */
#define GA_SCORE_RE 1u
#define GA_SCORE_IM 2u

/*
 * Score function of complex affinities (Sec. 2.3: complex kernel with signed
 * coefficients for interior and exterior query points; eq. 3 and eq. 5 with
 * the reflection of the moving part). For rho_1 = a_1 + i b_1 and
 * rho_2,b = a_2 + i b_2 (each channel a real density, e.g. from ga_splat
 * with its own weights), f_b(t) = sum_p rho_1(p) rho_2,b(p - t), with no
 * conjugate. From the half spectra of the four real channels:
 *   Re f = C2R(A_a conj(B_a) - A_b conj(B_b)),
 *   Im f = C2R(A_a conj(B_b) + A_b conj(B_a)).
 * d_A2: the two half spectra (A_a, then A_b) of the stationary affinity,
 * read with a stride of a_stride spectrum elements between batch members
 * (0 = one pair for the whole batch). d_B2: batch x 2 half spectra (B_a,
 * B_b). parts: GA_SCORE_RE, GA_SCORE_IM, or both (Re before Im). d_out:
 * batch x nparts real n^3 grids. Workspace: GA_OP_SCORE with
 * n_items = nparts. GA_EINVAL for parts outside 1..3, a negative stride or
 * overlapping buffers; GA_ENOMEM for a short workspace.
 */
ga_status ga_score(const ga_plan* plan, const float* d_A2, int64_t a_stride, const float* d_B2, int32_t batch,
                   uint32_t parts, float* d_out, void* d_work, size_t work_bytes, hipStream_t stream);

/*
 * The whole field path for many rotations of the moving part in one call
 * (Sec. 3.2 real-time sequence with the rotation applied by re-splatting, and
 * eq. 5): for each b < batch, B's samples are rotated by d_R[b] (device,
 * batch x 9 floats) about h_c, splatted, transformed, multiplied by
 * conj with the resident d_Ahat (one spectrum of the stationary part) and
 * transformed back into the energy field d_E[b] (batch x n^3 floats).
 * The moving part's densities are accumulated in fixed point, each x-plane
 * scaled by a power of two from the sum of |w| over the samples that reach
 * it. That sum must lie within about 2^-96 .. 2^96, where the rounding per
 * sample is at most 2^-31 of that sum; scaling every weight by a power of
 * two scales d_E by exactly that power.
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
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight haptic or serving loops, harnesses that forbid hipMalloc):
 * ga_force_torque in GA_SINGLE mode with no workspace argument. Same
 * arguments, kernels and results as ga_force_torque(..., GA_SINGLE, ...);
 * the per-strip float64 partial sums live in a static device array of the
 * library, GA_NOALLOC_SCRATCH_BYTES per device, held until the process ends.
 * The call allocates nothing (no hipMalloc, hipFree or allocating library
 * routine). It needs n_poses * ceil(n (n/2+1) / 64) * 56 bytes of that array
 * (2304 poses at n = 128, 145 at n = 512) and returns GA_ENOMEM beyond it,
 * before enqueueing anything. Every partial sum is written before it is read,
 * so nothing has to be cleared between calls. All calls on one device share
 * its array: calls that may overlap on one device (several streams or host
 * threads) race and must be serialised by the caller; d_out7 must not alias
 * the inputs.
 */
#define GA_NOALLOC_SCRATCH_BYTES (16u << 20)
ga_status ga_force_torque_noalloc(const ga_plan* plan, const float* d_Ahat, const float* d_Bhat4, const float* d_t,
                                  int32_t n_poses, float* d_out7, hipStream_t stream);

/*
 * Resident field of the stationary part for single-translation queries:
 * d_FA4[v] = (u_A, d_x u_A, d_y u_A, d_z u_A) at voxel v (float4 per voxel,
 * n^3 of them), the gradient being the spectral derivative of eq. 6a,
 * Re IFFT(2 pi i omega_a Ahat). d_uA: the density (ga_splat), d_Ahat: its
 * spectrum (ga_fft3d). Workspace: GA_OP_FIELD_GRAD.
 */
ga_status ga_field_grad(const ga_plan* plan, const float* d_uA, const float* d_Ahat, float* d_FA4, void* d_work,
                        size_t work_bytes, hipStream_t stream);

/*
 * Energy, force and torque at n_poses single poses, pose b being rotation
 * d_R[b] (9 floats) of the moving part about h_c and translation d_t[b]
 * (rounded to the nearest lattice point like GA_SINGLE), by local sums over
 * the moving part's balls only:
 *   E = sum_q u_A(q + t) u_B(q),   F = -sum_q grad u_A(q + t) u_B(q),
 *   tau = sum_q grad u_A(q + t) x yhat(q) u_B(q),
 * which equal the partial sums of eq. 7b that GA_SINGLE computes (the
 * spectral derivative moves from B to A by summation by parts), with
 * O(support of B) work and no transform of the moving part. d_FA4 from
 * ga_field_grad. d_out7: n_poses x 7 floats. Workspace: GA_OP_POSE_LOCAL
 * with batch = n_poses and n_items = n_pts.
 */
ga_status ga_pose_local(const ga_plan* plan, const float* d_FA4, const float* d_xyzr, const float* d_w, int64_t n_pts,
                        const float* d_R, const float* h_c, float sigma, const float* d_t, int32_t n_poses,
                        float* d_out7, void* d_work, size_t work_bytes, hipStream_t stream);

/*
 * Resident data of the stationary part for re-correlated single-translation
 * queries (ga_pose_spectral): d_AX2 = 2 half-spectrum-sized arrays,
 * AX(x, k_y, k_z) = sum_kx Ahat(k) exp(+2 pi i kx x / n) and DX, the same
 * transform of 2 pi i omega(kx) Ahat (the x-derivative multiplier of eq. 6a),
 * both unnormalised, [2][x][k_y][k_z] in the half-spectrum layout. d_Ahat:
 * the stationary part's spectrum (ga_fft3d). Needs the plane path (n <= 192,
 * else GA_EUNSUPPORTED). d_Ahat and d_AX2 must not overlap.
 */
ga_status ga_pose_prepare(const ga_plan* plan, const float* d_Ahat, float* d_AX2, hipStream_t stream);

/*
 * Energy, force and torque at n_poses single poses by re-correlation (Sec.
 * 3.2 real-time sequence for a new rotation; Sec. 3.3 single translation):
 * pose b rotates the moving part by d_R[b] about h_c and splats its 4
 * channels (u and the moment densities of eq. 6b), transforms each x-plane
 * along z and y, and adds that plane's share of the partial sum of eq. 7b at
 * translation round(d_t[b]) (nearest lattice point, as GA_SINGLE) for all 7
 * products of eq. 5, 6a, 6b: with the x transform folded into d_AX2
 * (ga_pose_prepare), sum_kx Ahat conj(Bhat) e^{2 pi i kx tx/n} =
 * sum_x conj(B(x)) AX(x + tx). Same values as ga_force_torque GA_SINGLE on
 * the re-splatted part's spectra (and as ga_pose_local), without writing any
 * spectrum of the moving part. Partial sums in float64. d_out7: n_poses x 7
 * floats; n_poses <= 65535. Workspace GA_OP_POSE_SPECTRAL with batch =
 * n_poses and n_items = n_pts. Needs the plane path (n <= 192).
 */
ga_status ga_pose_spectral(const ga_plan* plan, const float* d_AX2, const float* d_xyzr, const float* d_w,
                           int64_t n_pts, const float* d_R, const float* h_c, float sigma, const float* d_t,
                           int32_t n_poses, float* d_out7, void* d_work, size_t work_bytes, hipStream_t stream);

/*
 * Field tables for motion restricted to a set of orientations (Sec. 4.2,
 * "Restricted Motion DOF": with the orientation fixed the correlation is
 * precomputed once and read at every frame; the experiment of Sec. 4.3 runs
 * translation-only). ga_field_table writes, for each orientation o, the 7
 * fields (E, F_x, F_y, F_z, tau_x, tau_y, tau_z over all translations, as
 * ga_force_torque GA_FIELDS) to d_tables + o * 8 * n^3 as one 32-byte record
 * per voxel (float32 [o][x][y][z][8]: the 7 fields, then 0; 32 n^3 bytes per
 * orientation), so that a query reads one record per trilinear corner.
 * d_Bhat4: n_orient x 4 half spectra of the moving part at each orientation
 * (ga_splat + ga_fft3d, or ga_spectral_rotate); workspace
 * 7 * n^2 (n/2+1) * 8 + 7 * n^3 * 4 bytes.
 * ga_field_table_query reads query q's fields trilinearly at d_t[q]
 * (periodic, voxel units) in the table of orientation d_orient[q] (int32,
 * device): d_out7 = n_q x 7. An orientation index outside [0, n_orient)
 * gives NaN for that query. Errors: GA_EINVAL, GA_ENOMEM (workspace).
 */
ga_status ga_field_table(const ga_plan* plan, const float* d_Ahat, const float* d_Bhat4, int32_t n_orient,
                         float* d_tables, void* d_work, size_t work_bytes, hipStream_t stream);
ga_status ga_field_table_query(const ga_plan* plan, const float* d_tables, int32_t n_orient, const int32_t* d_orient,
                               const float* d_t, int32_t n_q, float* d_out7, hipStream_t stream);

/*
 * Spectral rotation (Sec. 3.2, step 1): instead of re-splatting the rotated
 * part, its resident spectra are interpolated trilinearly over the rotated
 * frequency grid: out_b(k) = X(R_b^T kappa(k)), kappa the signed frequency
 * (the Nyquist index n/2 taken as -n/2 on every axis),
 * X(-k) = conj X(k) for negative kz, zero beyond |component| = n/2. With
 * channels = 4 (u, yhat_x u, yhat_y u, yhat_z u of the part about the grid
 * origin, e.g. ga_splat with R = I and c = its reference point) the moment
 * channels rotate as a vector: M_R(k) = R_b M(R_b^T kappa). d_in: channels
 * half spectra; d_R: batch x 9 rotations (device, row-major); d_out: batch x
 * channels half spectra, usable by ga_correlate and ga_force_torque. An
 * approximation of the re-splatted spectra (exact for R = I and the 24
 * rotations of the cube). Errors: GA_EINVAL (channels not 1 or 4, overlaps).
 */
ga_status ga_spectral_rotate(const ga_plan* plan, const float* d_in, int32_t channels, const float* d_R, int32_t batch,
                             float* d_out, hipStream_t stream);

/*
 * Packed resident spectra for repeated spectral rotation (Sec. 3.2, step 1:
 * the moving part's spectra stay resident and are rotated every frame).
 * ga_spectral_pack4 writes the 4 half spectra d_in4 (u, yhat_x u, yhat_y u,
 * yhat_z u, as ga_spectral_rotate with channels = 4 takes them) as one
 * 32-byte record per frequency: d_packed[8 e .. 8 e + 7] = Re, Im of the 4
 * channels at element e of the half-spectrum layout (4 n^2 (n/2+1) float2,
 * the same size as d_in4; owned by the caller). ga_spectral_rotate_packed
 * then gives the outputs of ga_spectral_rotate with channels = 4 (batch x 4
 * half spectra in d_out, the same definition and arithmetic) reading one
 * record per interpolation corner for all 4 channels. Errors: GA_EINVAL
 * (overlapping or misaligned buffers, batch < 1).
 */
ga_status ga_spectral_pack4(const ga_plan* plan, const float* d_in4, float* d_packed, hipStream_t stream);
ga_status ga_spectral_rotate_packed(const ga_plan* plan, const float* d_packed, const float* d_R, int32_t batch,
                                    float* d_out, hipStream_t stream);

/*
 * Low-pass filtering (Sec. 3.3): of the n-grid half spectra only the modes
 * of the symmetric low-frequency box |kappa(k_a)| <= L/2 - 1 (kappa the signed
 * frequency index, every axis) are kept, times `scale`; L even, 4 <= L <= n.
 *   GA_LOWPASS_COARSE:  d_out = batch x [L][L][L/2+1], the kept modes on an L
 *     grid (index L/2 of each axis zero). Correlated with a plan for edge L
 *     (ga_correlate, ga_force_torque), with scale (L/n)^3 applied to one
 *     operand, it gives the filtered energy at the coarse translations
 *     t = t' n / L: E_L(t) = n^-3 sum_box Ahat conj(Bhat) exp(+2 pi i k.t/n);
 *     forces and torques from the L plan are per coarse voxel, i.e. times
 *     n / L of their per-voxel values, so multiply them by L / n.
 *   GA_LOWPASS_ZEROPAD: d_out = batch x [n][n][n/2+1] with the dropped modes
 *     zero (the zero padding of Sec. 4.3); any n-plan call then yields the
 *     filtered fields at full resolution.
 * d_in and d_out must not overlap. Errors: GA_EINVAL.
 */
#define GA_LOWPASS_COARSE 0u
#define GA_LOWPASS_ZEROPAD 1u
ga_status ga_lowpass(const ga_plan* plan, int32_t L, uint32_t mode, const float* d_in, float* d_out, int32_t batch,
                     float scale, hipStream_t stream);

/*
 * Autotuning of the fused correlation pass of ga_energy_fields (the x
 * transform, product with the stationary spectrum and inverse x transform).
 * Knobs: the strip width (groups = 4 or 8 groups of transforms per
 * wavefront, i.e. 4 or 8 wavefronts per workgroup), the number of batch
 * members k a workgroup takes in turn while keeping its stationary-spectrum
 * elements in registers (1, 2, 4, 8), and the grid mapping xcd: 1 =
 * XCD-aware (the member groups of one strip run back to back on one XCD,
 * whose L2 then serves the shared spectrum), 2 = plain; and the radix
 * schedule of the x transforms: 0 = the edge's default order of radices, 1 =
 * its alternative (n = 32: 4 x 8 instead of 8 x 4; 64: 4 x 16 instead of
 * 8 x 8; 96: 3 x 8 x 4 instead of 3 x 4 x 8; 128: 16 x 8 instead of 8 x 16;
 * 192: 8 x 8 x 3 instead of 3 x 8 x 8; other edges have none).
 * ga_plan_autotune times the plain-grid candidates, radix (0, 1) x groups
 * (4, 8) x k (1, 2, 4, 8) (the XCD-aware grid measured slower at every
 * setting on the 128^3 x 64 workload; ga_plan_tune can include it), each once
 * plus three timed launches on d_work (zeroed first; at least
 * batch * n^2 (n/2+1) * 8 bytes, the first part of a GA_OP_ENERGY workspace)
 * against d_Ahat; the fastest is kept in the plan and used by later
 * ga_energy_fields calls. The call synchronises `stream`. h_us (may be null
 * when n_us = 0) receives up to n_us = 16 per-launch times in microseconds
 * in that order, k fastest (0 for the radix-1 slots of an edge without an
 * alternative). ga_plan_set_tuning sets groups, k and xcd (0 = default: 4
 * groups, 4 members, plain grid) and ga_plan_set_radix the schedule
 * (GA_EINVAL for 1 on an edge without an alternative; ga_plan_has_alt_radix
 * says which); ga_plan_get_tuning and ga_plan_get_radix report the ones in
 * use. Not for graph capture.
 */
ga_status ga_plan_autotune(ga_plan* plan, const float* d_Ahat, int32_t batch, void* d_work, size_t work_bytes,
                           hipStream_t stream, float* h_us, int32_t n_us);
ga_status ga_plan_set_tuning(ga_plan* plan, int32_t groups, int32_t k, int32_t xcd);
ga_status ga_plan_get_tuning(const ga_plan* plan, int32_t* groups, int32_t* k, int32_t* xcd);
ga_status ga_plan_set_radix(ga_plan* plan, int32_t radix);
int32_t ga_plan_get_radix(const ga_plan* plan);
int32_t ga_plan_has_alt_radix(const ga_plan* plan);

/*
 * Tuning of a whole ga_energy_fields call for one (architecture, n, batch)
 * with a persisted cache (the real-time sequence of Sec. 3.2 repeats the
 * same call shape every frame, so a choice made once is reused). The key is
 * "<arch>/<n>/<batch>/1" (arch: the device's architecture name up to its
 * first ':', e.g. gfx950; 1 channel: the energy field). With cache_path set
 * and the key present in that file, the stored choice is applied without
 * timing (result->from_cache = 1). Otherwise the fused x pass's candidates
 * (radix, groups, k) are timed as by ga_plan_autotune (with flags &
 * GA_TUNE_XCD also on the XCD-aware grid), then, with flags & GA_TUNE_OVERLAP, whole calls on the
 * caller's inputs in 1, 2 and 4 parts over two streams (ga_plan_set_overlap;
 * two rounds of 2 warm-up and 5 timed calls each, the best time kept); the
 * fastest is applied to the plan, reported in *result (us = time per call)
 * and, with cache_path set, written to the file (other keys kept; written to
 * a temporary file and renamed over it). The arguments d_Ahat .. stream are
 * those of ga_energy_fields (d_E is overwritten). The file is a JSON object
 * with one line per key, {"groups": g, "k": k, "xcd": x, "radix": r,
 * "overlap": p, "us": t}. Errors: GA_EINVAL (arguments; a cache file that cannot be read,
 * is not in that layout, or cannot be written: it is left as it was),
 * GA_ENOMEM (workspace), GA_EUNSUPPORTED (separate-axis plans: their knobs
 * are not tuned), GA_EDEVICE. The call synchronises `stream`; not for graph
 * capture.
 */
#define GA_TUNE_XCD 1u
#define GA_TUNE_OVERLAP 2u
typedef struct ga_tuning {
  int32_t groups;     /* wavefronts of transforms per workgroup of the fused x pass */
  int32_t k;          /* batch members per workgroup */
  int32_t xcd;        /* 1 XCD-aware grid, 2 plain */
  int32_t radix;      /* 0 default radix schedule, 1 the alternative */
  int32_t overlap;    /* parts of the batch over two streams */
  float us;           /* time per ga_energy_fields call of this choice, microseconds */
  int32_t from_cache; /* 1 when read from the cache file */
} ga_tuning;
ga_status ga_plan_tune(ga_plan* plan, const float* d_Ahat, const float* d_xyzr, const float* d_w, int64_t n_pts,
                       const float* d_R, const float* h_c, float sigma, int32_t batch, float* d_E, void* d_work,
                       size_t work_bytes, uint32_t flags, const char* cache_path, hipStream_t stream,
                       ga_tuning* result);

/*
 * Overlapped execution of ga_energy_fields on the plane path (grid edges up
 * to 192). chunks = 1 (the default): every pass on the caller's stream.
 * chunks = 2 or 4: the batch is split into that many parts (whole workgroups
 * of the fused x pass), and each part's whole pipeline (binning, pass 1,
 * fused x pass, pass 3) runs on the caller's stream or on a second stream
 * owned by the plan (default priority), alternately. The parts on the two
 * streams run side by side: each stream fills the other's kernel tails and
 * launch gaps (measured faster than holding pass 1 of a part back until
 * pass 1 of the previous part is done). The second stream starts after an event on the caller's
 * stream and the call ends with the caller's stream waiting on it: results
 * and workspace reuse keep the caller's stream order. Calls on a capturing stream run with one
 * stream. The first call with chunks > 1 creates the plan's stream and
 * events on the plan's device. The fields are those of chunks = 1 up to the
 * order of float atomic additions in the splat. GA_EINVAL for other values;
 * GA_EDEVICE if the stream or events cannot be created.
 */
ga_status ga_plan_set_overlap(ga_plan* plan, int32_t chunks);
int32_t ga_plan_get_overlap(const ga_plan* plan);

/*
 * Batched execution as one graph launch (Sec. 3.2: the energy field of many
 * relative rotations per frame). A batch is a list of items, each one
 * stationary spectrum against `batch` rotations of one moving part on the
 * item's own grid edge, i.e. one ga_energy_fields call; items may use
 * different plans (grid edges). ga_batch_create records all items into one
 * HIP graph, each item on its own parallel branch, and instantiates it;
 * ga_batch_launch replays it on `stream` with a single graph launch. An item
 * whose plan is set to 2 or 4 parts (ga_plan_set_overlap, plane path) is
 * recorded as that many parts of its batch on parallel branches, each in a
 * 256-byte aligned slice of the item's d_work, when the slices fit in
 * work_bytes (otherwise as one branch).
 *
 * Every pointer of an item is captured by the graph: a replay reads the
 * current contents of d_Ahat, d_xyzr, d_w and d_R and overwrites d_E and
 * d_work, so callers update inputs in place between launches. Items must not
 * share d_E or d_work, and each d_work holds GA_OP_ENERGY bytes for the
 * item's batch and n_pts. The plans and all buffers must outlive the batch.
 * Errors: GA_EINVAL (an item fails the ga_energy_fields checks, overlapping
 * outputs or workspaces between items, n_items < 1), GA_ENOMEM (workspace too
 * small), GA_EDEVICE (graph capture or instantiation failed). Replays run
 * without per-kernel timing.
 */
typedef struct ga_batch ga_batch;

typedef struct {
  const ga_plan* plan;
  const float* d_Ahat;  /* stationary half spectrum (complex64 as float pairs) */
  const float* d_xyzr;  /* moving part: n_pts x (x, y, z, r) */
  const float* d_w;     /* n_pts weights */
  int64_t n_pts;
  const float* d_R;     /* batch x 9 rotations, row-major */
  float c[3];           /* rotation centre of the moving part */
  float sigma;
  int32_t batch;
  float* d_E;           /* batch x n^3 energy fields */
  void* d_work;
  size_t work_bytes;
} ga_batch_item;

ga_status ga_batch_create(ga_batch** out, const ga_batch_item* items, int32_t n_items);
ga_status ga_batch_launch(const ga_batch* b, hipStream_t stream);
ga_status ga_batch_destroy(ga_batch* b);

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

/*
 * Serving loop (Sec. 4.2: the haptic loop has a budget t0 of about 1 ms per
 * frame; Sec. 3.3: one translation per query). A server keeps, for every
 * registered part pair, the stationary part's spectrum and the moving part's
 * samples resident in device memory, and answers pose queries: each query is
 * a new rotation R of the moving part about its reference point and a
 * translation t; its answer is (E, F, tau) at round(t) for that rotation:
 * the GA_SINGLE readout of ga_force_torque after a 4-channel splat and
 * R2C of the rotated part (GA_SERVE_SPECTRAL), or the equal local sums of
 * ga_pose_local (GA_SERVE_LOCAL).
 *
 * Continuous batching: queries wait in a queue per grid size; a scheduler
 * thread moves up to max_slots of them into a free execution slot group
 * (two per grid size, sharing the size's stream) as soon as one is free, so
 * queries that arrive while others run are admitted as slots free up and
 * the groups of different sizes run concurrently on the device. Every query
 * is computed independently of the others in its group: its result does not
 * depend on the mix, up to float32 rounding of the splat's accumulation.
 * All device memory the server holds (spectra, samples, slot scratch) is
 * charged to hbm_budget_bytes; registration fails with GA_ENOMEM beyond it.
 * Calls are thread-safe. A device error is sticky: later calls return
 * GA_EDEVICE.
 */
typedef struct ga_server ga_server;

#define GA_SERVE_LOCAL 0u    /* queries by ga_pose_local sums (resident u_A and grad u_A) */
#define GA_SERVE_SPECTRAL 1u /* queries by splat, R2C and the GA_SINGLE partial sum (resident Ahat) */

/*
 * Test executor (for host-side tests of the scheduler, no device): with
 * mock_fn set, the server schedules exactly as it does on the GPU (queues,
 * launch groups, continuous batching, admission by budget and queue depth,
 * the byte accounting of the device data it would hold, sticky errors) but
 * holds no device memory and launches nothing: a launch group calls
 * mock_fn(mock_user, pair_id, n, R, t, out7) for each of its queries on the
 * scheduler thread (t: the lattice translation the kernels would use) and
 * reports completion mock_launch_us microseconds after its launch. A
 * nonzero return acts as a device error: the group fails and the server
 * turns sticky (GA_EDEVICE). device is then not used. Null mock_fn: the GPU.
 */
typedef int32_t (*ga_mock_query_fn)(void* user, uint32_t pair_id, int32_t n, const float* R, const int32_t* t,
                                    float* out7);

typedef struct {
  int32_t device;            /* HIP device ordinal */
  uint64_t hbm_budget_bytes; /* device memory the server may hold */
  int32_t max_slots;         /* queries per launch group (1 .. 256) */
  int32_t queue_depth;       /* queued queries before ga_submit returns GA_EAGAIN */
  uint32_t mode;             /* GA_SERVE_LOCAL or GA_SERVE_SPECTRAL; both give the same values */
  ga_mock_query_fn mock_fn;  /* test executor; null for the GPU */
  void* mock_user;           /* passed to mock_fn */
  uint32_t mock_launch_us;   /* simulated duration of one launch group */
} ga_server_cfg;

typedef struct {
  const float* xyzr; /* host, n_pts x 4 floats (x, y, z, r) */
  const float* w;    /* host, n_pts floats */
  int64_t n_pts;
} ga_part;

typedef struct {
  float E;
  float F[3];
  float tau[3];
  uint64_t t_submit_ns; /* steady clock, when ga_submit accepted the query */
  uint64_t t_start_ns;  /* when its group was launched */
  uint64_t t_done_ns;   /* when the scheduler saw its group complete */
} ga_result;

typedef struct {
  uint64_t submitted, completed, launches, rejected_full;
  uint64_t bytes_in_use;
  int32_t pairs;
} ga_server_stats;

ga_status ga_server_create(ga_server** server, const ga_server_cfg* cfg);
ga_status ga_server_destroy(ga_server* server); /* waits for queued queries */

/* Registers a part pair on an n^3 grid with thickness sigma: A (stationary,
 * grid coordinates) and B (moving, rotated about cB). The host arrays are
 * copied. Computes A's spectrum on the device before returning. */
ga_status ga_pair_register(ga_server* server, const ga_part* A, const ga_part* B, const float cB[3], int32_t n,
                           float sigma, uint32_t* pair_id);
/* Releases a pair once its queued queries have completed. */
ga_status ga_pair_release(ga_server* server, uint32_t pair_id);

/* Queues one query. R: 9 floats row-major, proper orthogonal within 1e-4; t:
 * 3 finite floats (voxels). Non-blocking; GA_EAGAIN when the queue is full,
 * GA_ENOTFOUND for an unknown pair. */
ga_status ga_submit(ga_server* server, uint32_t pair_id, const float R[9], const float t[3], uint64_t* ticket);

/* GA_OK with the result (once per ticket; the ticket is then forgotten),
 * GA_PENDING while queued or running, GA_ENOTFOUND for an unknown ticket. */
ga_status ga_poll(ga_server* server, uint64_t ticket, ga_result* out);

ga_status ga_server_get_stats(ga_server* server, ga_server_stats* out);

#ifdef __cplusplus
}
#endif

#endif /* GA_H */
