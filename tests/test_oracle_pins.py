"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these compares the oracle with itself by retyping a formula: each
checks a closed form, an invariant, brute force on tiny inputs, a textbook
routine, or a third-party library (numpy.fft) as an outside cross-check.
CPU only.
"""

import itertools
import math

import numpy as np
import pytest

import oracle as O
import synth


def _small_pair(n=16, seed=11, npts=60, conf=4.0, rlo=1.0, rhi=2.5):
    A = synth.random_part(seed, n, npts, rlo, rhi, conf_radius=conf)
    B = synth.random_part(seed + 1, n, npts, rlo, rhi, conf_radius=conf)
    return A, B


def _fields(A, B, n, R=None, cB=None, **kw):
    R = np.eye(3, dtype=np.float32) if R is None else R
    cB = B.ref_point() if cB is None else cB
    return O.pair_fields(A.xyzr, A.w, B.xyzr, B.w, R, cB, n, **kw)


# ---------------------------------------------------------------------------
# P14 -- transforms against the direct DFT, numpy.fft and textbook identities
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [4, 6, 8, 12])
def test_p14_fast_and_separable_equal_direct_sum(n):
    x = np.random.default_rng(n).standard_normal((n, n, n)) + 1j * np.random.default_rng(n + 1).standard_normal((n, n, n))
    Xd = O.fft3(x, method="direct")
    assert np.abs(O.fft3(x, method="dft") - Xd).max() < 1e-11 * n ** 3
    assert np.abs(O.fft3(x, method="fft") - Xd).max() < 1e-11 * n ** 3
    Xi = O.fft3(x, +1, method="direct")
    assert np.abs(O.fft3(x, +1, method="fft") - Xi).max() < 1e-11 * n ** 3


@pytest.mark.parametrize("n", [16, 24, 32, 48, 64, 96])
def test_p14_fft_matches_numpy_third_party(n):
    x = np.random.default_rng(n).standard_normal((n, n, n))
    X = O.fft3(x)
    ref = np.fft.fftn(x)
    assert np.abs(X - ref).max() / np.abs(ref).max() < 1e-13
    if n <= 48:
        assert np.abs(O.fft3(x, method="dft") - ref).max() / np.abs(ref).max() < 1e-12


@pytest.mark.parametrize("n", [8, 12, 32])
def test_p14_roundtrip_hermitian_delta_planewave(n):
    rng = np.random.default_rng(5)
    x = rng.standard_normal((n, n, n))
    X = O.fft3(x)
    # inverse of forward is the identity
    assert np.abs(O.ifft3(X).real - x).max() < 1e-12
    # real input: X(-k) = conj X(k)
    neg = (-np.arange(n)) % n
    assert np.abs(X[np.ix_(neg, neg, neg)] - np.conj(X)).max() < 1e-10
    # a delta at p0 gives the pure phase exp(-2 pi i k.p0 / n); at 0 a constant
    d = np.zeros((n, n, n))
    d[0, 0, 0] = 1.0
    assert np.abs(O.fft3(d) - 1.0).max() < 1e-13
    p0 = (1, 2, n - 1)
    d = np.zeros((n, n, n))
    d[p0] = 1.0
    g = np.arange(n)
    ph = np.exp(-2j * np.pi * (g[:, None, None] * p0[0] + g[None, :, None] * p0[1] + g[None, None, :] * p0[2]) / n)
    assert np.abs(O.fft3(d) - ph).max() < 1e-12
    # a plane wave exp(2 pi i k0.p / n) gives n^3 at k0 and 0 elsewhere
    k0 = (2, n - 3, 1)
    wave = np.exp(2j * np.pi * (g[:, None, None] * k0[0] + g[None, :, None] * k0[1] + g[None, None, :] * k0[2]) / n)
    W = O.fft3(wave)
    expect = np.zeros((n, n, n), complex)
    expect[k0] = n ** 3
    assert np.abs(W - expect).max() < 1e-9


@pytest.mark.parametrize("n", [8, 12, 16])
def test_p14_half_spectrum_inverse_matches_numpy(n):
    rng = np.random.default_rng(9)
    x = rng.standard_normal((n, n, n))
    H = O.rfft3(x)
    assert np.abs(H - np.fft.rfftn(x)).max() < 1e-11
    assert np.abs(O.irfft3(H) - x).max() < 1e-12
    # arbitrary (non-Hermitian) half spectrum: same convention as numpy's irfftn
    H2 = rng.standard_normal(H.shape) + 1j * rng.standard_normal(H.shape)
    assert np.abs(O.irfft3(H2) - np.fft.irfftn(H2, s=(n, n, n), axes=(0, 1, 2))).max() < 1e-12


# ---------------------------------------------------------------------------
# P15 -- the splat kernel
# ---------------------------------------------------------------------------

def test_p15_single_sample_on_lattice_point():
    n = 16
    u = O.splat(np.array([[5.0, 6.0, 7.0]]), np.array([2.5]), np.array([0.75]), n)
    assert u[5, 6, 7] == pytest.approx(0.75, abs=1e-15)
    assert u.max() == pytest.approx(0.75, abs=1e-15)
    # support is the open ball of radius rho (2.5): (5+2, 6, 7) in, (5+3, 6, 7) out
    assert u[7, 6, 7] > 0 and u[8, 6, 7] == 0.0
    # radial symmetry: equal distance, equal value (all 48 signed permutations)
    ref = u[5 + 1, 6 + 2, 7 + 0]
    for perm in itertools.permutations((1, 2, 0)):
        for sg in itertools.product((1, -1), repeat=3):
            assert u[5 + sg[0] * perm[0], 6 + sg[1] * perm[1], 7 + sg[2] * perm[2]] == pytest.approx(ref, rel=1e-14)


def test_p15_kernel_profile_and_small_radius_floor():
    # sigma = 0.5: K(d) = (exp(-2 d^2/rho^2) - e^-2) / (1 - e^-2) inside the ball
    for r, d in [(3.0, 0.0), (3.0, 1.5), (4.0, 3.9), (0.5, 0.5)]:
        rho = max(r, 1.0)
        expect = (math.exp(-2 * d * d / rho ** 2) - math.exp(-2)) / (1 - math.exp(-2)) if d < rho else 0.0
        assert float(O.kernel_value(d * d, r, 0.5)) == pytest.approx(expect, rel=1e-14, abs=1e-15)
    assert float(O.kernel_value(1.0, 1.0, 0.5)) == 0.0  # d == rho is outside


def test_p15_integer_shift_equivariance_and_wrap():
    n = 16
    rng = np.random.default_rng(3)
    y = rng.uniform(0, n, (20, 3))
    r = rng.uniform(1, 3, 20)
    w = rng.uniform(-1, 1, 20)
    u = O.splat(y, r, w, n)
    s = np.array([3, -5, 17])
    u2 = O.splat(y + s, r, w, n)
    assert np.abs(u2 - np.roll(u, tuple(s), axis=(0, 1, 2))).max() < 1e-13


def test_p15_lattice_sum_matches_closed_form_integral():
    n = 32
    sig = 0.5
    rho = 6.0
    s = sig * rho
    e0 = math.exp(-rho * rho / (2 * s * s))
    radial = s ** 3 * (math.sqrt(math.pi / 2) * math.erf(rho / (math.sqrt(2) * s))
                       - (rho / s) * math.exp(-rho * rho / (2 * s * s)))
    integral = 4 * math.pi * (radial - e0 * rho ** 3 / 3) / (1 - e0)
    u = O.splat(np.array([[10.3, 11.7, 12.1]]), np.array([rho]), np.array([1.0]), n, sig)
    assert u.sum() == pytest.approx(integral, rel=2e-3)


# ---------------------------------------------------------------------------
# P1, P2, P3 -- correlation against brute force and closed forms
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [8, 12, 16])
def test_p1_fft_correlation_equals_brute_force(n):
    A, B = _small_pair(n, seed=20 + n, npts=40, conf=n / 4)
    d = _fields(A, B, n)
    Eb = O.correlate_brute_field(d["uA"], d["uB"])
    assert O.rel_l2(d["E"], Eb) < 1e-13
    # and the definition straight from the samples at a few translations
    assert np.allclose(O.correlate_direct(d["uA"], d["uB"], [[0, 0, 0], [1, 2, 3], [n - 1, 0, 5]]),
                       O.lattice_read(Eb, [[0, 0, 0], [1, 2, 3], [n - 1, 0, 5]]), rtol=1e-13, atol=1e-12)


def test_p2_indicator_boxes_give_intersection_volume():
    n = 12
    a0, La = np.array([1, 2, 3]), np.array([4, 3, 5])
    b0, Lb = np.array([6, 0, 2]), np.array([3, 5, 2])
    a = np.zeros((n, n, n))
    b = np.zeros((n, n, n))
    a[a0[0]:a0[0] + La[0], a0[1]:a0[1] + La[1], a0[2]:a0[2] + La[2]] = 1.0
    b[b0[0]:b0[0] + Lb[0], b0[1]:b0[1] + Lb[1], b0[2]:b0[2] + Lb[2]] = 1.0
    E = O.correlate_fft(a, b)

    def overlap(ax, t):
        tot = 0
        for s in (-n, 0, n):
            lo = max(a0[ax], b0[ax] + t + s)
            hi = min(a0[ax] + La[ax], b0[ax] + t + Lb[ax] + s)
            tot += max(0, hi - lo)
        return tot

    for t in itertools.product(range(n), repeat=3):
        vol = overlap(0, t[0]) * overlap(1, t[1]) * overlap(2, t[2])
        assert E[t] == pytest.approx(vol, abs=1e-9)


@pytest.mark.parametrize("n,k0,phi", [(12, (1, 2, 0), 0.3), (16, (3, -2, 5), 1.1), (24, (0, 0, 7), -0.4)])
def test_p3_cosine_waves_closed_form_energy_and_force(n, k0, phi):
    g = np.arange(n)
    th = 2 * np.pi * (g[:, None, None] * k0[0] + g[None, :, None] * k0[1] + g[None, None, :] * k0[2]) / n
    a = np.cos(th)
    b = np.cos(th + phi)
    Ah, Bh = O.fft3(a), O.fft3(b)
    E = np.real(O.ifft3(Ah * np.conj(Bh)))
    F = O.force_field_spectral(Ah, Bh)
    # E(t) = n^3/2 cos(theta_t - phi); F = -grad_t E = n^3/2 sin(theta_t - phi) 2 pi k0/n
    assert np.abs(E - 0.5 * n ** 3 * np.cos(th - phi)).max() < 1e-9 * n ** 3
    for ax in range(3):
        expect = 0.5 * n ** 3 * np.sin(th - phi) * 2 * np.pi * k0[ax] / n
        assert np.abs(F[ax] - expect).max() < 1e-9 * n ** 3


# ---------------------------------------------------------------------------
# P4-P7 -- invariants
# ---------------------------------------------------------------------------

def test_p4_parseval_and_p5_sums():
    n = 16
    A, B = _small_pair(n)
    d = _fields(A, B, n, want_torque=False)
    E = d["E"]
    assert np.sum(E ** 2) == pytest.approx(np.sum(np.abs(d["Ahat"]) ** 2 * np.abs(d["Bhat"]) ** 2) / n ** 3, rel=1e-12)
    assert np.sum(E) == pytest.approx(d["uA"].sum() * d["uB"].sum(), rel=1e-12)
    assert E[0, 0, 0] == pytest.approx(np.sum(d["uA"] * d["uB"]), rel=1e-12)


def test_p6_action_reaction_symmetry():
    n = 16
    A, B = _small_pair(n)
    uA = O.splat(A.xyzr[:, :3].astype(np.float64), A.xyzr[:, 3], A.w, n)
    uB = O.splat(B.xyzr[:, :3].astype(np.float64), B.xyzr[:, 3], B.w, n)
    Ah, Bh = O.fft3(uA), O.fft3(uB)
    Eab = np.real(O.ifft3(Ah * np.conj(Bh)))
    Eba = np.real(O.ifft3(Bh * np.conj(Ah)))
    neg = (-np.arange(n)) % n
    assert np.abs(Eab - Eba[np.ix_(neg, neg, neg)]).max() < 1e-10 * np.abs(Eab).max()
    Fab = O.force_field_spectral(Ah, Bh)
    Fba = O.force_field_spectral(Bh, Ah)
    for ax in range(3):
        assert np.abs(Fab[ax] + Fba[ax][np.ix_(neg, neg, neg)]).max() < 1e-10 * np.abs(Fab).max()


def test_p7_shift_equivariance_of_samples():
    n = 16
    A, B = _small_pair(n)
    xa = A.xyzr[:, :3].astype(np.float64)
    xb = B.xyzr[:, :3].astype(np.float64)
    cB = B.ref_point().astype(np.float64)
    I = np.eye(3)

    def energy(xa_, xb_):
        uA = O.splat(O.place(xa_, I, np.zeros(3)), A.xyzr[:, 3], A.w, n)
        uB = O.splat(O.place(xb_, I, cB), B.xyzr[:, 3], B.w, n)
        return O.correlate_fft(uA, uB)

    E = energy(xa, xb)
    s = np.array([2, -3, 5])
    tol = 1e-10 * np.abs(E).max()
    # A shifted by s: E'(t) = E(t - s)
    assert np.abs(energy(xa + s, xb) - np.roll(E, tuple(s), axis=(0, 1, 2))).max() < tol
    # B shifted by s with c_B held fixed: E'(t) = E(t + s)
    assert np.abs(energy(xa, xb + s) - np.roll(E, tuple(-s), axis=(0, 1, 2))).max() < tol


# ---------------------------------------------------------------------------
# P8 -- the 24 proper cube rotations act exactly on the lattice
# ---------------------------------------------------------------------------

def _cube_rotations():
    out = []
    for perm in itertools.permutations(range(3)):
        for sg in itertools.product((1, -1), repeat=3):
            Q = np.zeros((3, 3))
            for i in range(3):
                Q[i, perm[i]] = sg[i]
            if np.linalg.det(Q) > 0:
                out.append(Q)
    return out


def test_p8_cube_rotation_equivariance():
    n = 16
    A = synth.random_part(41, n, 50, 1.0, 2.0, conf_radius=4.0)
    B = synth.random_part(42, n, 50, 1.0, 2.0, conf_radius=3.0)
    cB = B.ref_point()
    base = _fields(A, B, n, cB=cB)
    rots = _cube_rotations()
    assert len(rots) == 24
    g = np.arange(n)
    T = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    for Q in rots[1::5]:
        # A rotated about the grid origin, B rotated about c_B
        A2 = synth.Part(np.concatenate([(A.xyzr[:, :3].astype(np.float64) @ Q.T), A.xyzr[:, 3:]], 1).astype(np.float32), A.w)
        d2 = _fields(A2, B, n, R=Q.astype(np.float32), cB=cB)
        QT = (T @ Q.T.astype(np.int64)) % n
        assert np.abs(d2["E"][QT[:, 0], QT[:, 1], QT[:, 2]] - base["E"].reshape(-1)).max() < 1e-9 * np.abs(base["E"]).max()
        for key in ("F", "tau"):
            v = base[key].reshape(3, -1)
            Qv = Q @ v
            got = d2[key][:, QT[:, 0], QT[:, 1], QT[:, 2]]
            assert np.abs(got - Qv).max() < 1e-9 * np.abs(v).max(), key


# ---------------------------------------------------------------------------
# P9 -- force = -gradient of the trigonometric interpolant of E
# ---------------------------------------------------------------------------

def _trig_interp(Ehat, t):
    """Real trigonometric interpolant of a lattice field through its spectrum
    (numpy.fft), with the Nyquist term taken as cos(pi t)."""
    n = Ehat.shape[0]
    k = np.arange(n)
    kap = np.where(k < n / 2, k, k - n)
    phis = []
    for a in range(3):
        ph = np.exp(2j * np.pi * kap * t[a] / n)
        ph[n // 2] = np.cos(np.pi * t[a])
        phis.append(ph)
    return float(np.real(np.einsum("ijk,i,j,k->", Ehat, phis[0], phis[1], phis[2]))) / n ** 3


def test_p9_force_is_minus_gradient_of_interpolated_energy():
    n = 12
    A, B = _small_pair(n, seed=5, npts=40, conf=3.0)
    d = _fields(A, B, n, want_torque=False)
    Ehat = np.fft.fftn(d["E"])
    h = 1e-5
    for t in [(0, 0, 0), (3, 7, 1), (11, 5, 6)]:
        assert _trig_interp(Ehat, t) == pytest.approx(d["E"][t], rel=1e-10, abs=1e-10)
        for a in range(3):
            tp = np.array(t, float)
            tm = np.array(t, float)
            tp[a] += h
            tm[a] -= h
            fd = -(_trig_interp(Ehat, tp) - _trig_interp(Ehat, tm)) / (2 * h)
            assert d["F"][a][t] == pytest.approx(fd, rel=1e-6, abs=1e-6 * np.abs(d["F"]).max())


# ---------------------------------------------------------------------------
# P10, P11, P13 -- torque
# ---------------------------------------------------------------------------

def test_p10_torque_routes_agree_and_physical_force():
    n = 16
    A, B = _small_pair(n)
    d = _fields(A, B, n)
    T1 = O.torque_field_cross(d["uA"], d["uB"], brute=True)
    assert O.rel_l2(d["tau"], T1) < 1e-12
    F1 = O.force_field_physical(d["uA"], d["uB"], brute=True)
    assert O.rel_l2(d["F"], F1) < 1e-12


def _rot(axis, ang):
    c, s = math.cos(ang), math.sin(ang)
    x, y, z = axis
    return np.array([[c + x * x * (1 - c), x * y * (1 - c) - z * s, x * z * (1 - c) + y * s],
                     [y * x * (1 - c) + z * s, c + y * y * (1 - c), y * z * (1 - c) - x * s],
                     [z * x * (1 - c) - y * s, z * y * (1 - c) + x * s, c + z * z * (1 - c)]])


def _analytic_gradient(y, r, w, n, sigma=0.5):
    """Exact gradient of the continuous splat density at the lattice points
    (derivative of the truncated Gaussian, written out independently)."""
    g = np.zeros((3, n, n, n))
    for j in range(y.shape[0]):
        rho = max(r[j], 1.0)
        s2 = (sigma * rho) ** 2
        e0 = math.exp(-rho * rho / (2 * s2))
        lo = np.ceil(y[j] - rho).astype(int)
        hi = np.floor(y[j] + rho).astype(int)
        P = np.meshgrid(*[np.arange(lo[a], hi[a] + 1) for a in range(3)], indexing="ij")
        d = [P[a] - y[j, a] for a in range(3)]
        d2 = d[0] ** 2 + d[1] ** 2 + d[2] ** 2
        dk = np.where(d2 < rho * rho, -np.exp(-d2 / (2 * s2)) / s2 / (1 - e0), 0.0)
        for a in range(3):
            np.add.at(g[a], (P[0] % n, P[1] % n, P[2] % n), w[j] * dk * d[a])
    return g


def _rotational_fd(A, B, cB, n, ts, h=1e-4):
    """-dE/dtheta at translations ts by re-splatting B rotated by +-h about
    c_B (space-frame axes x, y, z)."""
    uA = O.splat(A.xyzr[:, :3].astype(np.float64), A.xyzr[:, 3], A.w, n)
    fd = np.zeros((len(ts), 3))
    for a in range(3):
        e = np.zeros(3)
        e[a] = 1.0
        vals = []
        for sgn in (+1, -1):
            yB = O.place(B.xyzr[:, :3], _rot(e, sgn * h), cB)
            uB = O.splat(yB, B.xyzr[:, 3], B.w, n)
            vals.append(O.correlate_direct(uA, uB, ts))
        fd[:, a] = -(vals[0] - vals[1]) / (2 * h)
    return uA, fd


def test_p11_torque_formula_is_minus_rotational_derivative():
    """tau = sum_p u_A(p) (yhat x grad u_B)(p - t) is -dE/dtheta: with the exact
    gradient of the continuous density it matches a finite difference of
    re-splatted rotations to FD accuracy (sign, axis order, centre)."""
    n = 32
    A = synth.random_part(61, n, 120, 3.0, 3.5, conf_radius=6.0)
    B = synth.random_part(62, n, 120, 3.0, 3.5, conf_radius=5.0)
    cB = B.ref_point()
    ts = [(16, 16, 16), (17, 15, 18), (14, 18, 15), (18, 17, 13)]
    uA, fd = _rotational_fd(A, B, cB, n, ts)
    yB = O.place(B.xyzr[:, :3], np.eye(3), cB)
    g = _analytic_gradient(yB, B.xyzr[:, 3].astype(np.float64), B.w.astype(np.float64), n)
    yh = O.min_image_coord(n)
    Y = (yh[:, None, None], yh[None, :, None], yh[None, None, :])
    G = [Y[1] * g[2] - Y[2] * g[1], Y[2] * g[0] - Y[0] * g[2], Y[0] * g[1] - Y[1] * g[0]]
    tau = np.stack([O.correlate_direct(uA, G[a], ts) for a in range(3)], 1)
    assert O.rel_l2(tau, fd) < 1e-6


def test_p11_spectral_torque_tracks_rotational_derivative_loose():
    """The method's torque uses the spectral gradient of the sampled density
    (eq. 6b), which differs from the continuous gradient by discretisation
    error (the kernel is only C0 at its cut-off); sign and scale must still
    follow -dE/dtheta."""
    n = 32
    A = synth.random_part(61, n, 120, 3.0, 3.5, conf_radius=6.0)
    B = synth.random_part(62, n, 120, 3.0, 3.5, conf_radius=5.0)
    cB = B.ref_point()
    ts = [(16, 16, 16), (17, 15, 18), (14, 18, 15), (18, 17, 13)]
    _, fd = _rotational_fd(A, B, cB, n, ts)
    got = O.lattice_read(_fields(A, B, n, cB=cB)["tau"], ts).T
    assert O.rel_l2(got, fd) < 0.35
    assert np.all(np.sign(got[np.abs(fd) > 0.3 * np.abs(fd).max()]) == np.sign(fd[np.abs(fd) > 0.3 * np.abs(fd).max()]))


def test_force_formula_is_minus_translational_derivative():
    """F = sum_p u_A(p) grad u_B(p - t) is -dE/dt: exact gradient vs a finite
    difference of re-splatted translations; the spectral force within the
    discretisation error."""
    n = 32
    A = synth.random_part(61, n, 120, 3.0, 3.5, conf_radius=6.0)
    B = synth.random_part(62, n, 120, 3.0, 3.5, conf_radius=5.0)
    cB = B.ref_point().astype(np.float64)
    ts = [(16, 16, 16), (17, 15, 18), (14, 18, 15)]
    uA = O.splat(A.xyzr[:, :3].astype(np.float64), A.xyzr[:, 3], A.w, n)
    y0 = O.place(B.xyzr[:, :3], np.eye(3), cB)
    h = 1e-4
    fd = np.zeros((len(ts), 3))
    for a in range(3):
        vals = []
        for sgn in (+1, -1):
            y = y0.copy()
            y[:, a] += sgn * h  # E'(t) = E(t + h e_a)
            vals.append(O.correlate_direct(uA, O.splat(y, B.xyzr[:, 3], B.w, n), ts))
        fd[:, a] = -(vals[0] - vals[1]) / (2 * h)
    g = _analytic_gradient(y0, B.xyzr[:, 3].astype(np.float64), B.w.astype(np.float64), n)
    F = np.stack([O.correlate_direct(uA, g[a], ts) for a in range(3)], 1)
    assert O.rel_l2(F, fd) < 1e-6
    Fs = O.lattice_read(_fields(A, B, n, cB=B.ref_point(), want_torque=False)["F"], ts).T
    assert O.rel_l2(Fs, fd) < 0.03


def test_p13_centred_single_sample_has_small_torque():
    n = 32
    A = synth.random_part(71, n, 150, 1.5, 3.0, conf_radius=8.0)
    cB = np.array([16.0, 16.0, 16.0], np.float32)
    one = synth.Part(np.array([[16.0, 16.0, 16.0, 3.0]], np.float32), np.ones(1, np.float32))
    off = synth.Part(np.array([[19.0, 16.0, 16.0, 3.0]], np.float32), np.ones(1, np.float32))
    d0 = _fields(A, one, n, cB=cB)
    d1 = _fields(A, off, n, cB=cB)
    # the same blob 3 voxels off the rotation centre has torque ~ |r x F|
    assert np.abs(d0["tau"]).max() < 1e-2 * np.abs(d1["tau"]).max()


# ---------------------------------------------------------------------------
# P12 -- zero-mode of the gradient fields; single-pose sum vs the fields
# ---------------------------------------------------------------------------

def test_p12_gradient_fields_sum_to_zero():
    n = 16
    A, B = _small_pair(n)
    d = _fields(A, B, n)
    for key in ("F", "tau"):
        for a in range(3):
            assert abs(d[key][a].sum()) < 1e-10 * np.abs(d[key]).sum()


def test_single_pose_sum_equals_lattice_fields():
    n = 12
    A, B = _small_pair(n, seed=31, npts=40, conf=3.0)
    d = _fields(A, B, n)
    for t in [(0, 0, 0), (1, 5, 11), (6, 6, 6), (5, 7, 6)]:
        s = O.single_pose_sum(d["Ahat"], d["Bhat"], d["Mhat"], t)
        ref = np.concatenate([[d["E"][t]], d["F"][:, t[0], t[1], t[2]], d["tau"][:, t[0], t[1], t[2]]])
        scale = max(np.abs(d["E"]).max(), np.abs(d["F"]).max(), np.abs(d["tau"]).max())
        assert np.abs(s - ref).max() < 1e-10 * scale


@pytest.mark.parametrize("n", [12, 15])
def test_local_pose_sum_equals_lattice_fields(n):
    """The physical-space sums with the gradient on A reproduce the spectral
    fields at every sampled lattice translation (odd and even n, rotated B)."""
    A, B = _small_pair(n, seed=41 + n, npts=40, conf=3.0)
    R = synth.shoemake_rotations(7, 1)[0]
    d = _fields(A, B, n, R=R)
    scale = max(np.abs(d["E"]).max(), np.abs(d["F"]).max(), np.abs(d["tau"]).max())
    for t in [(0, 0, 0), (1, 5, 11), (6, 6, 6), (n - 1, 2, 9), (-3, 4, 20)]:
        s = O.local_pose_sum(d["uA"], d["uB"], t)
        tl = tuple(int(v) % n for v in t)
        ref = np.concatenate([[d["E"][tl]], d["F"][(slice(None), *tl)], d["tau"][(slice(None), *tl)]])
        assert np.abs(s - ref).max() < 1e-10 * scale


def _cube_rotations():
    mats = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            Q = np.zeros((3, 3))
            for i in range(3):
                Q[i, perm[i]] = signs[i]
            if np.linalg.det(Q) > 0:
                mats.append(Q)
    return mats


def _rotate_grid(u, Q):
    """u'(p) = u(Q^T p) on the lattice (signed coordinates mod n), exact for
    a cube rotation Q."""
    n = u.shape[0]
    s = np.where(np.arange(n) < n / 2.0, np.arange(n), np.arange(n) - n)
    P = np.stack(np.meshgrid(s, s, s, indexing="ij"), -1)
    src = (P @ Q).astype(np.int64) % n  # Q^T p as rows
    return u[src[..., 0], src[..., 1], src[..., 2]]


def test_spectral_rotation_identity_and_cube_rotations_are_exact():
    """Sec. 3.2 step 1. R = I returns the spectrum; for each of the 24 cube
    rotations Q, R^T kappa is a lattice point, so the interpolated spectra are
    exactly the spectra of the rotated grid (density and moment channels)."""
    n = 12
    A, B = _small_pair(n, seed=71, npts=30, conf=2.5)
    u = O.splat(O.place(B.xyzr[:, :3], np.eye(3), B.ref_point()), B.xyzr[:, 3], B.w, n)
    X4 = np.stack([O.fft3(u)] + [O.fft3(m) for m in O.moment_channels(u)])
    assert np.allclose(O.spectral_rotate(X4[0], np.eye(3)), X4[0], atol=1e-12 * np.abs(X4[0]).max())
    for Q in _cube_rotations()[1::3]:
        ur = _rotate_grid(u, Q)
        ref = np.stack([O.fft3(ur)] + [O.fft3(m) for m in O.moment_channels(ur)])
        got = O.spectral_rotate4(X4, Q)
        assert np.abs(got - ref).max() < 1e-9 * np.abs(ref).max(), Q


def test_spectral_rotation_approximates_resplat():
    """For a general rotation the interpolated spectrum approximates the
    spectrum of the re-splatted rotated part (loose: trilinear interpolation
    of a spectrum whose support is a few voxels wide)."""
    n = 24
    B = synth.random_part(81, n, 30, 2.0, 3.0, conf_radius=2.0)
    c = B.ref_point()
    u0 = O.splat(O.place(B.xyzr[:, :3], np.eye(3), c), B.xyzr[:, 3], B.w, n)
    R = synth.shoemake_rotations(82, 1)[0]
    uR = O.splat(O.place(B.xyzr[:, :3], R, c), B.xyzr[:, 3], B.w, n)
    got = O.spectral_rotate(O.fft3(u0), R)
    assert O.rel_l2(got, O.fft3(uR)) < 0.25


@pytest.mark.parametrize("k0,inside", [((1, 2, 1), True), ((3, -2, 1), True), ((4, 1, 1), False), ((1, 1, 6), False)])
def test_lowpass_of_band_limited_waves(k0, inside):
    """Sec. 3.3 low-pass filtering. Two waves cos(2 pi k0.p/n) and
    cos(2 pi k0.p/n + phi): inside the box (|k0_a| <= L/2 - 1) the filtered
    energy is the full closed form (n^3/2) cos(2 pi k0.t/n - phi); outside it
    vanishes. On the coarse grid the kept modes give the same values at
    t = t' n / L, and the mask is Hermitian-closed."""
    n, L, phi = 16, 8, 0.7
    g = np.arange(n, dtype=np.float64)
    ph = 2 * np.pi * ((k0[0] * g[:, None, None] + k0[1] * g[None, :, None] + k0[2] * g[None, None, :]) % n) / n
    a, b = np.cos(ph), np.cos(ph + phi)
    Ah, Bh = O.fft3(a), O.fft3(b)
    ts = [(0, 0, 0), (2, 4, 6), (6, 2, 10), (14, 8, 4)]
    got = O.lowpass_energy(Ah, Bh, L, ts)
    full = np.array([(n ** 3 / 2) * np.cos(2 * np.pi * np.dot(k0, t) / n - phi) for t in ts])
    assert np.allclose(got, full if inside else 0 * full, atol=1e-9 * n ** 3)
    # coarse grid: L^-3 IDFT_L of the kept product, times (L/n)^3, at t' = t L / n
    PL = O.lowpass_coarse(O.rfft3(a), L) * np.conj(O.lowpass_coarse(O.rfft3(b), L))
    EL = O.irfft3(PL) * (L / n) ** 3
    coarse = [EL[t[0] * L // n, t[1] * L // n, t[2] * L // n] for t in ts]
    assert np.allclose(coarse, got, atol=1e-9 * n ** 3)
    m = O.lowpass_mask(n, L)
    assert m[1, 2, 1] and not m[4, 0, 0] and not m[0, 0, 4] and m[n - 3, 3, 3] == m[3, n - 3, 3]


def test_trilinear_read_is_exact_on_lattice_and_linear_between():
    n = 8
    f = np.random.default_rng(2).standard_normal((n, n, n))
    assert np.allclose(O.trilinear_read(f, [[1, 2, 3]]), f[1, 2, 3])
    mid = O.trilinear_read(f, [[1.5, 2.0, 7.0]])
    assert mid[0] == pytest.approx(0.5 * (f[1, 2, 7] + f[2, 2, 7]))
    wrap = O.trilinear_read(f, [[7.25, 0.0, 0.0]])
    assert wrap[0] == pytest.approx(0.75 * f[7, 0, 0] + 0.25 * f[0, 0, 0])


def test_rel_l2_compares_complex_values():
    """A mismatch only in imaginary parts must show."""
    a = np.array([1 + 1j, 2 - 1j])
    assert O.rel_l2(a, a) == 0.0
    assert O.rel_l2(a.real + 0j, a) > 0.4


# ---------------------------------------------------------------------------
# Complex affinities: the score function with the reflection of the moving
# part (eq. 3, eq. 5), and the signs of interior/exterior overlaps (Sec. 2.3)
# ---------------------------------------------------------------------------

def _complex_grid(rng, n):
    return rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n))


def _all_translations(n):
    g = np.arange(n)
    return np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)


@pytest.mark.parametrize("n", [4, 6])
def test_score_fft_equals_direct_sum_for_complex_affinities(n):
    rng = np.random.default_rng(40 + n)
    r1, r2 = _complex_grid(rng, n), _complex_grid(rng, n)
    brute = O.score_direct(r1, r2, _all_translations(n)).reshape(n, n, n)
    assert O.rel_l2(O.score_fft(r1, r2), brute) < 1e-13
    assert O.rel_l2(O.score_fft(r1, r2, method="direct"), brute) < 1e-13
    # conjugating the complex partner's spectrum instead of reflecting it is
    # a different function
    conj_route = O.ifft3(O.fft3(r1) * np.conj(O.fft3(r2)))
    assert O.rel_l2(conj_route, brute) > 0.1


def test_score_splits_into_real_correlations():
    """rho = a + i b on each side: Re f = a1*a2 - b1*b2, Im f = a1*b2 + b1*a2
    with * the real correlation, computed here by brute force."""
    n = 6
    rng = np.random.default_rng(7)
    a1, b1, a2, b2 = (rng.standard_normal((n, n, n)) for _ in range(4))
    f = O.score_fft(a1 + 1j * b1, a2 + 1j * b2)
    C = O.correlate_brute_field
    assert O.rel_l2(f.real, C(a1, a2) - C(b1, b2)) < 1e-13
    assert O.rel_l2(f.imag, C(a1, b2) + C(b1, a2)) < 1e-13


def test_score_of_real_and_imaginary_affinities():
    """Real affinities: the reflection is the conjugate, f = the real
    correlation. Purely imaginary ones (the skeleton reading): Re f is minus
    the correlation of the imaginary parts and Im f vanishes."""
    n = 8
    rng = np.random.default_rng(9)
    u1, u2 = rng.standard_normal((n, n, n)), rng.standard_normal((n, n, n))
    E = O.correlate_fft(u1, u2)
    f = O.score_fft(u1 + 0j, u2 + 0j)
    assert O.rel_l2(f.real, E) < 1e-13 and np.abs(f.imag).max() < 1e-12 * np.abs(E).max()
    g = O.score_fft(1j * u1, 1j * u2)
    assert O.rel_l2(g.real, -E) < 1e-13 and np.abs(g.imag).max() < 1e-12 * np.abs(E).max()


def test_interior_exterior_overlaps_reward_fit_and_penalise_collision():
    """One skeleton sample per part, overlapping at t = (8, 8, 8): interior
    against exterior scores positive, interior against interior and exterior
    against exterior negative, the latter penalty^2 times stronger."""
    n, pen = 16, 3.0
    yA = np.array([[8.0, 8.0, 8.0]])
    yB = np.zeros((1, 3))
    r = np.array([2.0])
    t = [[8, 8, 8]]

    def rho(y, ext):
        return 1j * O.splat(y, r, O.affinity_weights([ext], pen), n, 0.5)

    s = {(ea, eb): O.score_direct(rho(yA, ea), rho(yB, eb), t)[0] for ea in (False, True) for eb in (False, True)}
    assert s[(False, True)].real > 0 and s[(True, False)].real > 0
    assert s[(False, False)].real < 0 and s[(True, True)].real < 0
    assert s[(True, True)].real == pytest.approx(pen ** 2 * s[(False, False)].real, rel=1e-12)
    assert s[(False, True)].real == pytest.approx(-pen * s[(False, False)].real, rel=1e-12)
    assert all(abs(v.imag) < 1e-12 * abs(v.real) for v in s.values())
    assert list(O.affinity_weights([False, True, False], pen)) == [1.0, -pen, 1.0]


def test_generator_weights_follow_the_affinity_reading():
    a = synth.config_c2(4, exterior=True)
    assert np.array_equal(a.A.w, O.affinity_weights(a.A.exterior, synth.PENALTY).astype(np.float32))


def test_hole_axis_exterior_skeleton_makes_the_inserted_pose_the_unique_best_score():
    """Peg-in-hole at 128^3 (zero-clearance kernels: the peg's balls end 0.5
    voxel short of the rods'). With interior skeletons only, Re f is 0 on a
    flat plateau of millions of translations around the insertion; with the
    hole's axis as an exterior skeleton, the inserted pose (peg axis on the
    hole axis, c_B at the centre) is the strict maximum."""
    a = synth.config_c2(4, exterior=True)
    n = a.n
    yB = O.place(a.B.xyzr[:, :3], np.eye(3, dtype=np.float32), a.cB)
    rhoB = 1j * O.splat(yB, a.B.xyzr[:, 3], a.B.w, n, a.sigma)
    f = O.score_fft(1j * O.splat(a.A.xyzr[:, :3], a.A.xyzr[:, 3], a.A.w, n, a.sigma), rhoB).real
    best = np.unravel_index(np.argmax(f), f.shape)
    assert best == (64, 64, 64)
    others = f.copy()
    others[best] = -np.inf
    assert f[best] > others.max() > 0
    m = ~a.A.exterior
    f0 = O.score_fft(1j * O.splat(a.A.xyzr[m, :3], a.A.xyzr[m, 3], a.A.w[m], n, a.sigma), rhoB).real
    assert abs(f0[64, 64, 64]) < 1e-9 and f0.max() < 1e-9 and (f0 > -1e-9).sum() > 10 ** 6
