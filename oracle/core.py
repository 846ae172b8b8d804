"""FP64 oracle: plain definitions of the geometric-energy correlation path.

TEST INFRASTRUCTURE ONLY (see the package docstring). Every routine here is
written for a reader to check against the paper by eye; none is blocked,
fused or reordered for speed beyond what its definition states.

Conventions (readings of the paper, each listed with its reason in the design
notes of the repository):

* Grid: N^3 voxels, voxel centres at integer coordinates, dV = 1, array
  index [x, y, z] (z fastest). Everything is periodic on the N^3 torus
  (the discrete transforms of Sec. 3.2, eq. 7a/7b, are circular).
* Density (Sec. 2.3, skeletal density; modelled): each skeleton sample j is a
  ball (centre y_j, radius r_j, weight w_j) that contributes
  w_j K(d; r_j) with a truncated, shifted Gaussian in the distance d to the
  centre, K(d) = [exp(-d^2/2s^2) - exp(-rho^2/2s^2)] / [1 - exp(-rho^2/2s^2)]
  for d < rho and 0 beyond, rho = max(r, 1), s = sigma * rho. Its thickness is
  proportional to sigma * r like the paper's angular criterion, which is
  scale-free. d is the minimum-image distance on the torus.
* Motion (Sec. 2.4, motion decomposition): the moving part B is rotated about
  its reference point c_B and placed with c_B at the grid origin,
  y_j = R (x_j - c_B); the translation t is the position of c_B in A's frame.
* Transforms (eq. 4a/4b and 7a/7b): forward sum with exp(-2 pi i k.p/N),
  unnormalised; inverse with exp(+2 pi i k.p/N) and the factor N^-3.
* Energy (eq. 1 and 3, with eq. 5 as the fast route): for real densities the
  reflection of eq. 3 is the complex conjugate in frequency, so
  E(t) = sum_p u_A(p) u_B(p - t) = Re IFFT(FFT(u_A) conj FFT(u_B))(t).
* Force (eq. 6a): F = -dE/dt. With the spectral derivative of multiplier
  2 pi i omega_a, omega_a = kappa(k_a)/N and kappa zero on the Nyquist plane,
  F_a(t) = sum_p u_A(p) (d_a u_B)(p - t) = Re IFFT(-2 pi i omega_a A conj B)(t).
* Torque (eq. 6b, read with the moment density rho*_2(p) = rho_2(p) p): the
  space-frame torque about c_B, tau = -dE/dtheta, equals
  sum_p u_A(p) (yhat x grad u_B)(p - t) and spectrally
  Re IFFT(2 pi i (omega x conj M) A)(t) with M_b = FFT(yhat_b u_B), yhat the
  minimum-image coordinate of the grid point.
"""

from __future__ import annotations

import math

import numpy as np

__all__ = []

TWO_PI = 2.0 * math.pi


# ---------------------------------------------------------------------------
# Motion (Sec. 2.4, "Motion Decomposition")
# ---------------------------------------------------------------------------

def place(xyz, R, c):
    """Sample centres of a part rotated by R about c, with c moved to the
    origin: y_j = R (x_j - c). With R = I and c = 0 the centres are unchanged.

    Sec. 2.4: rho(T^-1 p; S) = rho(R^T (p - t); S) = rho(p - t; R S), so the
    rotated part's density is the density of the rotated samples (the kernel
    is isotropic)."""
    x = np.asarray(xyz, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64).reshape(3, 3)
    c = np.asarray(c, dtype=np.float64).reshape(3)
    return (x - c) @ R.T


# ---------------------------------------------------------------------------
# Density (Sec. 2.3, "Skeletal Density"; modelled, see module docstring)
# ---------------------------------------------------------------------------

def kernel_value(d2, r, sigma):
    """K(d; r) for squared distance d2: truncated, shifted Gaussian of
    width s = sigma * rho on the ball of radius rho = max(r, 1); peak 1 at the
    centre, continuous and zero at d = rho."""
    rho = max(float(r), 1.0)
    s2 = (sigma * rho) ** 2
    e0 = math.exp(-rho * rho / (2.0 * s2))
    d2 = np.asarray(d2, dtype=np.float64)
    val = (np.exp(-d2 / (2.0 * s2)) - e0) / (1.0 - e0)
    return np.where(d2 < rho * rho, val, 0.0)


def splat(y, r, w, n, sigma=0.5):
    """Density u(p) = sum_j w_j K(||p - y_j||_N; r_j) on the n^3 torus.

    One sample at a time: the voxels whose minimum-image distance to y_j is
    below rho_j are the integer points of the box (y_j - rho_j, y_j + rho_j)
    taken mod n (requires rho_j < n/2 so that no voxel is reached twice)."""
    y = np.asarray(y, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    u = np.zeros((n, n, n), dtype=np.float64)
    for j in range(y.shape[0]):
        rho = max(r[j], 1.0)
        if not rho < n / 2.0:
            raise ValueError("ball radius must be below n/2")
        lo = np.ceil(y[j] - rho).astype(np.int64)
        hi = np.floor(y[j] + rho).astype(np.int64)
        ax = [np.arange(lo[a], hi[a] + 1) for a in range(3)]
        px, py, pz = np.meshgrid(ax[0], ax[1], ax[2], indexing="ij")
        d2 = (px - y[j, 0]) ** 2 + (py - y[j, 1]) ** 2 + (pz - y[j, 2]) ** 2
        val = w[j] * kernel_value(d2, rho, sigma)
        np.add.at(u, (px % n, py % n, pz % n), val)
    return u


def min_image_coord(n):
    """yhat(q) = q for q < n/2 and q - n otherwise (position of grid index q
    relative to the origin, on the torus)."""
    q = np.arange(n)
    return np.where(q < n / 2.0, q, q - n).astype(np.float64)


def moment_channels(u):
    """Moment density rho*(p) = rho(p) p of eq. 6b on the grid:
    m_b(q) = yhat_b(q) u(q), b = x, y, z. Returns [3, n, n, n]."""
    n = u.shape[0]
    yh = min_image_coord(n)
    return np.stack([
        yh[:, None, None] * u,
        yh[None, :, None] * u,
        yh[None, None, :] * u,
    ])


# ---------------------------------------------------------------------------
# Discrete Fourier transforms (eq. 7a/7b; Cooley-Tukey 1965 for the fast form)
# ---------------------------------------------------------------------------

def _unit_root(n, idx, sign):
    """exp(sign * 2 pi i idx / n) with the integer phase index reduced mod n
    before the trigonometric call."""
    a = TWO_PI * (np.asarray(idx, dtype=np.int64) % n) / n
    return np.cos(a) + sign * 1j * np.sin(a)


def dft_direct3(x, sign=-1):
    """Direct O(N^6) sum X(k) = sum_p x(p) exp(sign 2 pi i k.p / N) (eq. 7a
    with dV = 1; sign +1 without the 1/N^3 factor). For tiny grids only."""
    x = np.asarray(x, dtype=np.complex128)
    n = x.shape[0]
    g = np.arange(n)
    P = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    phase = (P @ P.T) % n  # k.p for every (k, p) pair
    X = _unit_root(n, phase, sign) @ x.reshape(-1)
    return X.reshape(n, n, n)


def dft_axis(x, axis, sign=-1):
    """Separable direct DFT along one axis (a DFT matrix, O(N^2) per line)."""
    x = np.asarray(x, dtype=np.complex128)
    n = x.shape[axis]
    k = np.arange(n)
    D = _unit_root(n, np.outer(k, k), sign)
    return np.moveaxis(np.tensordot(D, np.moveaxis(x, axis, 0), axes=(1, 0)), 0, axis)


def _fft_last(x, sign):
    """Recursive decimation-in-time Cooley-Tukey along the last axis, radix 2
    or 3 (whichever divides first), direct DFT for other lengths."""
    n = x.shape[-1]
    if n == 1:
        return x.copy()
    p = 2 if n % 2 == 0 else (3 if n % 3 == 0 else 0)
    if p == 0:
        k = np.arange(n)
        return x @ _unit_root(n, np.outer(k, k), sign).T
    m = n // p
    k = np.arange(n)
    out = np.zeros(x.shape, dtype=np.complex128)
    for q in range(p):
        sub = _fft_last(x[..., q::p], sign)  # length-m transform of x[p j + q]
        out += _unit_root(n, q * k, sign) * sub[..., k % m]
    return out


def fft_axis(x, axis, sign=-1):
    """Fast DFT along one axis (same sums as dft_axis)."""
    x = np.moveaxis(np.asarray(x, dtype=np.complex128), axis, -1)
    return np.moveaxis(_fft_last(np.ascontiguousarray(x), sign), -1, axis)


def fft3(x, sign=-1, method="fft"):
    """3D DFT, unnormalised: X(k) = sum_p x(p) exp(sign 2 pi i k.p / N)."""
    if method == "direct":
        return dft_direct3(x, sign)
    f = fft_axis if method == "fft" else dft_axis
    X = np.asarray(x, dtype=np.complex128)
    for a in range(3):
        X = f(X, a, sign)
    return X


def ifft3(X, method="fft"):
    """Inverse 3D DFT: x(p) = N^-3 sum_k X(k) exp(+2 pi i k.p / N)."""
    n = X.shape[0]
    return fft3(X, +1, method) / float(n) ** 3


def rfft3(x, method="fft"):
    """Forward transform of a real grid, half spectrum k_z = 0..N/2."""
    n = x.shape[0]
    return fft3(x, -1, method)[:, :, : n // 2 + 1]


def irfft3(H, method="fft"):
    """Real inverse of a half spectrum [N, N, N/2+1].

    The full spectrum is completed by X(-k) = conj X(k); on the k_z = 0 and
    k_z = N/2 planes, where the half spectrum holds both members of a pair,
    the Hermitian part (X(k) + conj X(-k))/2 is used, so that the result is
    the real field whose spectrum is closest to the input."""
    n = H.shape[0]
    X = np.zeros((n, n, n), dtype=np.complex128)
    X[:, :, : n // 2 + 1] = H
    neg = (-np.arange(n)) % n
    for kz in range(n // 2 + 1, n):
        X[:, :, kz] = np.conj(H[np.ix_(neg, neg, [n - kz])][:, :, 0])
    for kz in (0, n // 2):
        plane = H[:, :, kz]
        X[:, :, kz] = 0.5 * (plane + np.conj(plane[np.ix_(neg, neg)]))
    return np.real(ifft3(X, method))


# ---------------------------------------------------------------------------
# Spectral derivative (eq. 6a multiplier)
# ---------------------------------------------------------------------------

def omega(n):
    """omega(k) = kappa(k)/N with kappa(k) = k (k < N/2), k - N (k > N/2) and
    0 on the Nyquist index k = N/2 (its +/- pair has no odd part)."""
    k = np.arange(n)
    kap = np.where(k < n / 2.0, k, k - n).astype(np.float64)
    if n % 2 == 0:
        kap[n // 2] = 0.0
    return kap / n


def _omega_axes(n):
    w = omega(n)
    return (w[:, None, None], w[None, :, None], w[None, None, :])


def grad_spectral(u, method="fft"):
    """Gradient of the trigonometric interpolant of u on the lattice:
    d_a u = Re IFFT(2 pi i omega_a FFT(u)). Returns [3, n, n, n]."""
    U = fft3(u, -1, method)
    oms = _omega_axes(u.shape[0])
    return np.stack([np.real(ifft3(2j * math.pi * oms[a] * U, method)) for a in range(3)])


# ---------------------------------------------------------------------------
# Correlation (eq. 1 / eq. 3 by definition, eq. 5 by the convolution theorem)
# ---------------------------------------------------------------------------

def correlate_direct(a, b, ts):
    """C(t) = sum_p a(p) b((p - t) mod N) at the given integer translations."""
    ts = np.asarray(np.rint(ts), dtype=np.int64).reshape(-1, 3)
    out = np.empty(ts.shape[0])
    for i, t in enumerate(ts):
        out[i] = np.sum(a * np.roll(b, tuple(int(v) for v in t), axis=(0, 1, 2)))
    return out


def correlate_brute_field(a, b):
    """C(t) for every t on the lattice, straight from the definition."""
    n = a.shape[0]
    g = np.arange(n)
    T = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    return correlate_direct(a, b, T).reshape(n, n, n)


def correlate_fft(a, b, method="fft"):
    """C = Re IFFT(FFT(a) conj FFT(b)) (eq. 5 for real densities)."""
    return np.real(ifft3(fft3(a, -1, method) * np.conj(fft3(b, -1, method)), method))


def energy_field(uA, uB, method="fft"):
    """Geometric energy E(t) over all lattice translations (eq. 3 / eq. 5)."""
    return correlate_fft(uA, uB, method)


def force_field_spectral(Ahat, Bhat):
    """F_a = Re IFFT(-2 pi i omega_a A conj B) for a = x, y, z (eq. 6a, with
    F = -dE/dt). Full spectra in, [3, n, n, n] out."""
    P = Ahat * np.conj(Bhat)
    oms = _omega_axes(Ahat.shape[0])
    return np.stack([np.real(ifft3(-2j * math.pi * oms[a] * P)) for a in range(3)])


def force_field_physical(uA, uB, method="fft", brute=False):
    """F_a(t) = sum_p u_A(p) (d_a u_B)(p - t): the force as the correlation of
    A with the gradient of B (F = -dE/dt of eq. 3)."""
    g = grad_spectral(uB, method)
    corr = correlate_brute_field if brute else (lambda x, y: correlate_fft(x, y, method))
    return np.stack([corr(uA, g[a]) for a in range(3)])


def torque_field_moment(Ahat, Mhat):
    """tau_a = Re IFFT(2 pi i (omega x conj M)_a A) with M_b = FFT(yhat_b u_B)
    (eq. 6b with the moment density)."""
    oms = _omega_axes(Ahat.shape[0])
    Mc = [np.conj(Mhat[b]) for b in range(3)]
    cross = [
        oms[1] * Mc[2] - oms[2] * Mc[1],
        oms[2] * Mc[0] - oms[0] * Mc[2],
        oms[0] * Mc[1] - oms[1] * Mc[0],
    ]
    return np.stack([np.real(ifft3(2j * math.pi * cross[a] * Ahat)) for a in range(3)])


def torque_field_cross(uA, uB, method="fft", brute=False):
    """tau(t) = sum_p u_A(p) G(p - t) with G = yhat x grad u_B: minus the
    derivative of E under a rotation of B about c_B (space frame)."""
    n = uA.shape[0]
    g = grad_spectral(uB, method)
    yh = min_image_coord(n)
    Y = (yh[:, None, None], yh[None, :, None], yh[None, None, :])
    G = [
        Y[1] * g[2] - Y[2] * g[1],
        Y[2] * g[0] - Y[0] * g[2],
        Y[0] * g[1] - Y[1] * g[0],
    ]
    corr = correlate_brute_field if brute else (lambda x, y: correlate_fft(x, y, method))
    return np.stack([corr(uA, G[a]) for a in range(3)])


def single_pose_sum(Ahat, Bhat, Mhat, t):
    """(E, F, tau) at one integer translation t by the partial sum of eq. 7b
    over all modes (the cascade for a single translation, Sec. 3.3):
    value = N^-3 Re sum_k P(k) exp(+2 pi i (k.t mod N)/N)."""
    n = Ahat.shape[0]
    t = np.asarray(np.rint(t), dtype=np.int64).reshape(3)
    g = np.arange(n)
    idx = (g[:, None, None] * t[0] + g[None, :, None] * t[1] + g[None, None, :] * t[2]) % n
    ph = _unit_root(n, idx, +1)
    oms = _omega_axes(n)
    P = Ahat * np.conj(Bhat)
    out = [np.real(np.sum(P * ph))]
    for a in range(3):
        out.append(np.real(np.sum(-2j * math.pi * oms[a] * P * ph)))
    Mc = [np.conj(Mhat[b]) for b in range(3)]
    cross = [
        oms[1] * Mc[2] - oms[2] * Mc[1],
        oms[2] * Mc[0] - oms[0] * Mc[2],
        oms[0] * Mc[1] - oms[1] * Mc[0],
    ]
    for a in range(3):
        out.append(np.real(np.sum(2j * math.pi * cross[a] * Ahat * ph)))
    return np.array(out) / float(n) ** 3


def local_pose_sum(uA, uB, t, grad=None):
    """(E, F, tau) at one integer translation t by sums over the lattice in
    physical space, with the gradient on the stationary part:
    E = sum_q u_A(q + t) u_B(q), F = -sum_q grad u_A(q + t) u_B(q),
    tau = sum_q (grad u_A(q + t) x yhat(q)) u_B(q).
    Equal to single_pose_sum: the correlation of eq. 3 with q = p - t, and the
    spectral derivative of eq. 6a/6b moved from B to A by summation by parts
    (its multiplier 2 pi i omega is odd, the Nyquist mode being zero).
    grad: grad_spectral(uA) when the caller already has it (several poses)."""
    n = uA.shape[0]
    t = np.asarray(np.rint(t), dtype=np.int64).reshape(3)
    shift = tuple(int(-v) for v in t)
    a = np.roll(uA, shift, axis=(0, 1, 2))  # a[q] = u_A(q + t)
    g = np.roll(grad_spectral(uA) if grad is None else grad, shift, axis=(1, 2, 3))
    yh = min_image_coord(n)
    Y = (yh[:, None, None], yh[None, :, None], yh[None, None, :])
    cross = [g[1] * Y[2] - g[2] * Y[1], g[2] * Y[0] - g[0] * Y[2], g[0] * Y[1] - g[1] * Y[0]]
    out = [np.sum(a * uB)]
    out += [-np.sum(g[k] * uB) for k in range(3)]
    out += [np.sum(cross[k] * uB) for k in range(3)]
    return np.array(out)


# ---------------------------------------------------------------------------
# Spectral rotation (Sec. 3.2, step 1: the moving part's spectra interpolated
# trilinearly over the rotated frequency grid R^T omega)
# ---------------------------------------------------------------------------

def spectral_rotate(X, R):
    """X_R(k) = X(R^T kappa(k)) by trilinear interpolation over the full
    spectrum X [n, n, n] (signed frequencies kappa; corners with a component
    beyond n/2 in magnitude contribute zero). For a density u about the grid
    origin, X_R approximates the spectrum of u o R^T."""
    n = X.shape[0]
    R = np.asarray(R, dtype=np.float64).reshape(3, 3)
    kap = np.where(np.arange(n) < n / 2.0, np.arange(n), np.arange(n) - n).astype(np.float64)
    K = np.stack(np.meshgrid(kap, kap, kap, indexing="ij"), -1)  # [n, n, n, 3]
    Q = K @ R  # rows: (R^T kappa)^T = kappa^T R
    f = np.floor(Q)
    a = Q - f
    f = f.astype(np.int64)
    out = np.zeros(X.shape, dtype=np.complex128)
    for dx in (0, 1):
        for dy in (0, 1):
            for dz in (0, 1):
                c = f + np.array([dx, dy, dz])
                w = (np.where(dx, a[..., 0], 1 - a[..., 0]) * np.where(dy, a[..., 1], 1 - a[..., 1]) *
                     np.where(dz, a[..., 2], 1 - a[..., 2]))
                inside = np.all(np.abs(c) <= n // 2, axis=-1)
                v = X[c[..., 0] % n, c[..., 1] % n, c[..., 2] % n]
                out += np.where(inside, w * v, 0)
    return out


def spectral_rotate4(X4, R):
    """The 4 channels (u, yhat_x u, yhat_y u, yhat_z u) of the moving part: the
    density spectrum is interpolated at R^T kappa, the moment spectra as a
    vector, M_R(k) = R M(R^T kappa(k)) (the moment density of the rotated part
    is p u(R^T p) = R (R^T p) u(R^T p))."""
    R = np.asarray(R, dtype=np.float64).reshape(3, 3)
    I = [spectral_rotate(X4[c], R) for c in range(4)]
    M = [sum(R[a, b] * I[1 + b] for b in range(3)) for a in range(3)]
    return np.stack([I[0], *M])


# ---------------------------------------------------------------------------
# Low-pass filtering (Sec. 3.3: only m' << m low-frequency modes are kept)
# ---------------------------------------------------------------------------

def lowpass_mask(n, L):
    """Half-spectrum mask [n, n, n/2+1] of the symmetric low-frequency box
    |kappa(k_a)| <= L/2 - 1 on every axis (kappa = signed frequency index), a
    set closed under k -> -k, so the kept modes stay Hermitian."""
    kap = np.where(np.arange(n) < n / 2.0, np.arange(n), np.arange(n) - n)
    keep = np.abs(kap) <= L // 2 - 1
    kz = np.arange(n // 2 + 1) <= L // 2 - 1
    return keep[:, None, None] & keep[None, :, None] & kz[None, None, :]


def lowpass_coarse(H, L):
    """The kept modes of an n-grid half spectrum H as an L-grid half spectrum
    [L, L, L/2+1] (index L/2 on each axis and kz = L/2 are zero)."""
    n = H.shape[0]
    out = np.zeros((L, L, L // 2 + 1), dtype=np.complex128)
    kp = np.arange(L)
    kap = np.where(kp < L / 2.0, kp, kp - L)
    ok = np.abs(kap) <= L // 2 - 1
    src = kap % n
    for i in np.nonzero(ok)[0]:
        for j in np.nonzero(ok)[0]:
            out[i, j, : L // 2] = H[src[i], src[j], : L // 2]
    return out


def lowpass_energy(Ahat, Bhat, L, ts):
    """E_L(t) = n^-3 sum over the kept box of Ahat(k) conj(Bhat(k))
    exp(+2 pi i k.t / n) at integer translations t (full spectra in)."""
    n = Ahat.shape[0]
    kap = np.where(np.arange(n) < n / 2.0, np.arange(n), np.arange(n) - n)
    keep1 = np.abs(kap) <= L // 2 - 1
    keep = keep1[:, None, None] & keep1[None, :, None] & keep1[None, None, :]
    P = np.where(keep, Ahat * np.conj(Bhat), 0)
    g = np.arange(n)
    out = []
    for t in np.asarray(np.rint(ts), dtype=np.int64).reshape(-1, 3):
        idx = (g[:, None, None] * t[0] + g[None, :, None] * t[1] + g[None, None, :] * t[2]) % n
        out.append(np.real(np.sum(P * _unit_root(n, idx, +1))) / float(n) ** 3)
    return np.array(out)


# ---------------------------------------------------------------------------
# Complex affinities (Sec. 2.3: complex kernel with signed coefficients for
# interior and exterior query points; eq. 3 and eq. 5 with the reflection of
# the moving part, which for complex functions is not a conjugation)
# ---------------------------------------------------------------------------

def affinity_weights(exterior, penalty):
    """Imaginary-channel weight of each skeleton sample: +lambda1 = +1 on the
    interior skeleton, -lambda2 = -penalty on the exterior one (penalty factor
    lambda2/lambda1). Near the skeleton the complex kernel's value is close to
    purely imaginary with the sign of the side, so the affinity is
    i (u_int - penalty u_ext)."""
    exterior = np.asarray(exterior, dtype=bool)
    return np.where(exterior, -float(penalty), 1.0)


def reflect_spectrum(X):
    """X(-k) on the torus: the spectrum of the reflection x(-p) (the reflection
    commutes with the transform, eq. 4a)."""
    n = X.shape[0]
    neg = (-np.arange(n)) % n
    return X[np.ix_(neg, neg, neg)]


def score_direct(rho1, rho2, ts):
    """f_SC(t) = sum_p rho1(p) rho2((p - t) mod N) at the given integer
    translations: eq. 3, the convolution of rho1 with the reflection of rho2,
    for complex affinities (no conjugate anywhere)."""
    ts = np.asarray(np.rint(ts), dtype=np.int64).reshape(-1, 3)
    out = np.empty(ts.shape[0], dtype=np.complex128)
    for i, t in enumerate(ts):
        out[i] = np.sum(rho1 * np.roll(rho2, tuple(int(v) for v in t), axis=(0, 1, 2)))
    return out


def score_fft(rho1, rho2, method="fft"):
    """f_SC = IFFT(FFT(rho1)(k) FFT(rho2)(-k)) with complex transforms
    (eq. 5: the spectrum of the reflected part is the reflected spectrum)."""
    return ifft3(fft3(rho1, -1, method) * reflect_spectrum(fft3(rho2, -1, method)), method)


# ---------------------------------------------------------------------------
# Pose readout (Sec. 2.4, force/torque at the current configuration)
# ---------------------------------------------------------------------------

def lattice_read(field, ts):
    """field[t mod N] at integer translations t (fields [..., n, n, n])."""
    n = field.shape[-1]
    ts = np.asarray(np.rint(ts), dtype=np.int64).reshape(-1, 3) % n
    return field[..., ts[:, 0], ts[:, 1], ts[:, 2]]


def trilinear_read(field, ts):
    """Trilinear interpolation between the 8 periodic lattice neighbours."""
    n = field.shape[-1]
    ts = np.asarray(ts, dtype=np.float64).reshape(-1, 3)
    f = np.floor(ts)
    a = ts - f
    i0 = f.astype(np.int64)
    out = 0.0
    for dx in (0, 1):
        for dy in (0, 1):
            for dz in (0, 1):
                wgt = ((a[:, 0] if dx else 1 - a[:, 0]) * (a[:, 1] if dy else 1 - a[:, 1])
                       * (a[:, 2] if dz else 1 - a[:, 2]))
                ix = (i0[:, 0] + dx) % n
                iy = (i0[:, 1] + dy) % n
                iz = (i0[:, 2] + dz) % n
                out = out + wgt * field[..., ix, iy, iz]
    return out


# ---------------------------------------------------------------------------
# Whole path for one pair at one rotation
# ---------------------------------------------------------------------------

def pair_fields(A_xyzr, A_w, B_xyzr, B_w, R, cB, n, sigma=0.5, want_torque=True, method="fft"):
    """Densities, spectra and the 7 fields (E, F_xyz, tau_xyz) for stationary
    part A (grid coordinates as given) and moving part B rotated by R about cB.
    Returns a dict of float64 arrays."""
    A_xyzr = np.asarray(A_xyzr, dtype=np.float32).astype(np.float64)
    B_xyzr = np.asarray(B_xyzr, dtype=np.float32).astype(np.float64)
    uA = splat(A_xyzr[:, :3], A_xyzr[:, 3], np.asarray(A_w, np.float64), n, sigma)
    yB = place(B_xyzr[:, :3], np.asarray(R, np.float32), np.asarray(cB, np.float32))
    uB = splat(yB, B_xyzr[:, 3], np.asarray(B_w, np.float64), n, sigma)
    Ah = fft3(uA, -1, method)
    Bh = fft3(uB, -1, method)
    E = np.real(ifft3(Ah * np.conj(Bh), method))
    out = {"uA": uA, "uB": uB, "Ahat": Ah, "Bhat": Bh, "E": E,
           "F": force_field_spectral(Ah, Bh)}
    if want_torque:
        M = moment_channels(uB)
        Mh = np.stack([fft3(M[b], -1, method) for b in range(3)])
        out["Mhat"] = Mh
        out["tau"] = torque_field_moment(Ah, Mh)
    return out


def rel_l2(got, ref):
    """||got - ref||_2 / ||ref||_2 over all elements (complex values compared
    as complex numbers)."""
    cplx = np.iscomplexobj(got) or np.iscomplexobj(ref)
    got = np.asarray(got, dtype=np.complex128 if cplx else np.float64)
    ref = np.asarray(ref, dtype=np.complex128 if cplx else np.float64)
    den = np.linalg.norm(ref.ravel())
    return float(np.linalg.norm((got - ref).ravel()) / (den if den > 0 else 1.0))
