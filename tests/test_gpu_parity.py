"""GPU parity: every C-ABI call against the FP64 oracle on the same seeded inputs.

Tolerances (relative L2 over all compared elements): 1e-5 for densities,
spectra and energy fields, 1e-4 for forces and torques. Small grids are
compared element by element; the full-size workloads (128^3) on sampled
outputs that the oracle evaluates one by one.
"""

import numpy as np
import pytest
import torch

import oracle as O
import synth

pytestmark = pytest.mark.gpu

FIELD_TOL = 1e-5
FORCE_TOL = 1e-4


@pytest.fixture(scope="module")
def G():
    import paper_1711_05017_amd as pkg

    pkg.lib()
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    return pkg


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _part(n, seed, npts, rlo=1.0, rhi=3.0, conf=None):
    return synth.random_part(seed, n, npts, rlo, rhi, conf_radius=conf)


# ---------------------------------------------------------------------------
# splat
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,npts,rot", [(16, 30, False), (32, 200, False), (48, 333, True), (96, 700, True),
                                        (128, 2000, True), (192, 1500, True)])
def test_splat_matches_oracle(G, n, npts, rot):
    p = _part(n, 1000 + n, npts, 0.5, 4.0)
    plan = G.Plan(n)
    if rot:
        R = synth.shoemake_rotations(7 + n, 1)[0]
        c = p.ref_point()
    else:
        R, c = None, None
    got = G.ga_splat(plan, _dev(p.xyzr), _dev(p.w), R=R, c=c, channels=4).cpu().numpy()
    if rot:
        y = O.place(p.xyzr[:, :3], R, c)
    else:
        y = p.xyzr[:, :3].astype(np.float64)
    u = O.splat(y, p.xyzr[:, 3], p.w, n)
    ref = np.concatenate([u[None], O.moment_channels(u)])
    assert O.rel_l2(got[0], ref[0]) < FIELD_TOL
    for ch in range(1, 4):
        assert O.rel_l2(got[ch], ref[ch]) < FIELD_TOL


def test_splat_edge_cases(G):
    n = 16
    plan = G.Plan(n)
    # empty input gives zeros
    z = G.ga_splat(plan, torch.zeros((0, 4), device="cuda"), torch.zeros(0, device="cuda"))
    assert float(z.abs().max()) == 0.0
    # radius below one voxel is raised to one; a radius reaching n/2 is dropped;
    # negative weights and coordinates outside [0, n) wrap
    xyzr = np.array([[3.0, 4.0, 5.0, 0.3], [-1.25, 17.5, 8.0, 2.5], [8.0, 8.0, 8.0, 8.0], [15.9, 0.1, 7.7, 3.0]],
                    np.float32)
    w = np.array([1.0, -0.5, 1.0, 2.0], np.float32)
    got = G.ga_splat(plan, _dev(xyzr), _dev(w)).cpu().numpy()[0]
    keep = [0, 1, 3]
    ref = O.splat(xyzr[keep, :3].astype(np.float64), xyzr[keep, 3], w[keep], n)
    assert O.rel_l2(got, ref) < FIELD_TOL
    # invalid arguments are rejected synchronously
    with pytest.raises(G.GaError):
        G.ga_splat(plan, _dev(xyzr), _dev(w), sigma=0.0)
    with pytest.raises(G.GaError):
        G.ga_splat(plan, _dev(xyzr), _dev(w), channels=2)
    with pytest.raises(G.GaError):
        G.ga_splat(plan, _dev(xyzr), _dev(w), R=np.diag([1.0, 1.0, -1.0]), c=[0, 0, 0])


# ---------------------------------------------------------------------------
# 3D FFT
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [16, 24, 32, 48, 64, 96, 128, 192])
def test_fft3d_r2c_and_c2r_match_oracle(G, n):
    rng = np.random.default_rng(n)
    batch = 2
    x = rng.standard_normal((batch, n, n, n)).astype(np.float32)
    plan = G.Plan(n, max_batch=batch)
    X = G.ga_fft3d(plan, G.GA_R2C, _dev(x)).cpu().numpy()
    for b in range(batch):
        ref = O.rfft3(x[b].astype(np.float64))
        assert O.rel_l2(X[b], ref) < FIELD_TOL
    # C2R of an arbitrary (not Hermitian) half spectrum
    H = (rng.standard_normal((batch, n, n, n // 2 + 1)) + 1j * rng.standard_normal((batch, n, n, n // 2 + 1)))
    H = H.astype(np.complex64)
    y = G.ga_fft3d(plan, G.GA_C2R, _dev(H)).cpu().numpy()
    for b in range(batch):
        ref = O.irfft3(H[b].astype(np.complex128))
        assert O.rel_l2(y[b], ref) < FIELD_TOL


def test_fft3d_roundtrip_and_batch_limit(G):
    n = 32
    plan = G.Plan(n, max_batch=3)
    x = np.random.default_rng(1).standard_normal((3, n, n, n)).astype(np.float32)
    y = G.ga_fft3d(plan, G.GA_C2R, G.ga_fft3d(plan, G.GA_R2C, _dev(x))).cpu().numpy()
    assert np.abs(y - x).max() < 1e-5 * np.abs(x).max()
    with pytest.raises(G.GaError):
        G.ga_fft3d(plan, G.GA_R2C, _dev(np.zeros((4, n, n, n), np.float32)))


# ---------------------------------------------------------------------------
# correlation
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [16, 32, 48, 96])
def test_correlate_from_oracle_spectra(G, n):
    A = _part(n, 2000 + n, 8 * n)
    B = _part(n, 3000 + n, 8 * n)
    d = O.pair_fields(A.xyzr, A.w, B.xyzr, B.w, np.eye(3, dtype=np.float32), B.ref_point(), n,
                      want_torque=False)
    h = n // 2 + 1
    Ah = _dev(d["Ahat"][:, :, :h].astype(np.complex64))
    Bh = _dev(np.stack([d["Bhat"][:, :, :h], np.conj(d["Bhat"][:, :, :h])]).astype(np.complex64))
    plan = G.Plan(n, max_batch=2)
    E = G.ga_correlate(plan, Ah, Bh).cpu().numpy()
    assert O.rel_l2(E[0], d["E"]) < FIELD_TOL
    # second member: conj(B) correlates with the reflected density
    ref2 = np.real(O.ifft3(d["Ahat"] * d["Bhat"]))
    assert O.rel_l2(E[1], ref2) < FIELD_TOL


@pytest.mark.parametrize("n,npts,nrot", [(32, 200, 3), (48, 300, 5), (96, 900, 3), (192, 1200, 2)])
def test_energy_fields_fused_path(G, n, npts, nrot):
    A = _part(n, 4000 + n, npts, 1.0, 4.0)
    B = _part(n, 5000 + n, npts, 1.0, 4.0)
    R = synth.shoemake_rotations(6000 + n, nrot)
    cB = B.ref_point()
    plan = G.Plan(n, max_batch=nrot)
    uA = G.ga_splat(plan, _dev(A.xyzr), _dev(A.w))
    Ahat = G.ga_fft3d(plan, G.GA_R2C, uA)[0]
    E = G.ga_energy_fields(plan, Ahat, _dev(B.xyzr), _dev(B.w), _dev(R), cB).cpu().numpy()
    uA_ref = O.splat(A.xyzr[:, :3].astype(np.float64), A.xyzr[:, 3], A.w, n)
    for r in range(nrot):
        uB_ref = O.splat(O.place(B.xyzr[:, :3], R[r], cB), B.xyzr[:, 3], B.w, n)
        assert O.rel_l2(E[r], O.energy_field(uA_ref, uB_ref)) < FIELD_TOL, r


@pytest.mark.parametrize("n,npts,nrot", [(64, 500, 2), (96, 800, 2), (128, 1500, 2)])
def test_energy_fields_fixed_point_splat(G, n, npts, nrot):
    """The batched path splats the moving part in fixed point with a per-plane
    power-of-two scale (sum of |w| over the plane's candidates): weights over
    six decades still match the oracle, scaling every weight by 2^40 or 2^-40
    scales the field by exactly that power (the integer sums are unchanged),
    and repeated calls give the same bits."""
    A = _part(n, 7100 + n, npts, 1.0, 3.0)
    B = _part(n, 7200 + n, npts, 1.0, 3.0, conf=n / 6)
    wB = (B.w * 10.0 ** np.random.default_rng(7300 + n).uniform(-3, 3, B.n)).astype(np.float32)
    R = synth.shoemake_rotations(7400 + n, nrot)
    cB = B.ref_point()
    plan = G.Plan(n, max_batch=nrot)
    Ahat = G.ga_fft3d(plan, G.GA_R2C, G.ga_splat(plan, _dev(A.xyzr), _dev(A.w)))[0].contiguous()
    xb, Rd = _dev(B.xyzr), _dev(R)
    E = G.ga_energy_fields(plan, Ahat, xb, _dev(wB), Rd, cB).cpu().numpy()
    uA_ref = O.splat(A.xyzr[:, :3].astype(np.float64), A.xyzr[:, 3], A.w, n)
    for r in range(nrot):
        uB_ref = O.splat(O.place(B.xyzr[:, :3], R[r], cB), B.xyzr[:, 3], wB.astype(np.float64), n)
        assert O.rel_l2(E[r], O.energy_field(uA_ref, uB_ref)) < FIELD_TOL, r
    again = G.ga_energy_fields(plan, Ahat, xb, _dev(wB), Rd, cB).cpu().numpy()
    assert np.array_equal(again, E)
    for k in (40, -40):
        Ek = G.ga_energy_fields(plan, Ahat, xb, _dev(np.ldexp(wB, k).astype(np.float32)), Rd, cB).cpu().numpy()
        assert np.array_equal(Ek, np.ldexp(E, k)), k


@pytest.mark.parametrize("n,npts,nrot", [(64, 400, 3), (128, 1200, 5), (192, 1500, 2)])
def test_energy_fields_skip_empty_planes(G, n, npts, nrot):
    """Pass 1 stores no x-plane that no sample reaches and the x pass reads
    only the planes pass 1 marked: a workspace full of NaN bits beforehand
    (stale spectra in every plane) must not reach the fields."""
    A = _part(n, 7600 + n, npts, 1.0, 3.0)
    B = _part(n, 7700 + n, npts, 1.0, 3.0, conf=n / 6)  # most x-planes of B stay empty
    R = synth.shoemake_rotations(7800 + n, nrot)
    cB = B.ref_point()
    plan = G.Plan(n, max_batch=nrot)
    Ahat = G.ga_fft3d(plan, G.GA_R2C, G.ga_splat(plan, _dev(A.xyzr), _dev(A.w)))[0].contiguous()
    work = plan.workspace(G.ga.GA_OP_ENERGY, nrot, B.n)
    work.fill_(255)
    E = G.ga_energy_fields(plan, Ahat, _dev(B.xyzr), _dev(B.w), _dev(R), cB, work=work).cpu().numpy()
    assert np.isfinite(E).all()
    uA_ref = O.splat(A.xyzr[:, :3].astype(np.float64), A.xyzr[:, 3], A.w, n)
    for r in range(nrot):
        uB_ref = O.splat(O.place(B.xyzr[:, :3], R[r], cB), B.xyzr[:, 3], B.w, n)
        assert O.rel_l2(E[r], O.energy_field(uA_ref, uB_ref)) < FIELD_TOL, r


@pytest.mark.parametrize("n,npts,nrot", [(32, 6000, 2), (64, 12000, 2), (128, 25000, 2)])
def test_energy_fields_dense_part_many_candidate_rounds(G, n, npts, nrot):
    """A dense moving part: every x-plane has several rounds of candidates
    (more than one per lane of the workgroup) and wavefronts hold more hits
    than their LDS batch, so the splat's later rounds, its batches and the
    plane bound over all rounds are exercised against the oracle."""
    A = _part(n, 8000 + n, 400, 1.0, 3.0)
    B = _part(n, 8100 + n, npts, 1.0, 3.0, conf=n / 6)
    R = synth.shoemake_rotations(8200 + n, nrot)
    cB = B.ref_point()
    plan = G.Plan(n, max_batch=nrot)
    Ahat = G.ga_fft3d(plan, G.GA_R2C, G.ga_splat(plan, _dev(A.xyzr), _dev(A.w)))[0].contiguous()
    E = G.ga_energy_fields(plan, Ahat, _dev(B.xyzr), _dev(B.w), _dev(R), cB).cpu().numpy()
    uA_ref = O.splat(A.xyzr[:, :3].astype(np.float64), A.xyzr[:, 3], A.w, n)
    for r in range(nrot):
        uB_ref = O.splat(O.place(B.xyzr[:, :3], R[r], cB), B.xyzr[:, 3], B.w, n)
        assert O.rel_l2(E[r], O.energy_field(uA_ref, uB_ref)) < FIELD_TOL, r


def test_c1_workload_end_to_end(G):
    a = synth.config_c1()
    n = a.n
    plan = G.Plan(n, max_batch=4)
    uA = G.ga_splat(plan, _dev(a.A.xyzr), _dev(a.A.w), sigma=a.sigma)
    Ahat = G.ga_fft3d(plan, G.GA_R2C, uA)[0]
    E = G.ga_energy_fields(plan, Ahat, _dev(a.B.xyzr), _dev(a.B.w), _dev(a.rotations), a.cB, a.sigma).cpu().numpy()
    d = O.pair_fields(a.A.xyzr, a.A.w, a.B.xyzr, a.B.w, a.rotations[0], a.cB, n, a.sigma)
    assert O.rel_l2(E[0], d["E"]) < FIELD_TOL
    uB4 = G.ga_splat(plan, _dev(a.B.xyzr), _dev(a.B.w), R=a.rotations[0], c=a.cB, sigma=a.sigma, channels=4)
    Bhat4 = G.ga_fft3d(plan, G.GA_R2C, uB4)
    t = _dev(a.poses)
    ref = np.concatenate([O.lattice_read(d["E"], a.poses)[:, None], O.lattice_read(d["F"], a.poses).T,
                          O.lattice_read(d["tau"], a.poses).T], 1)
    for mode in (G.GA_FIELDS, G.GA_SINGLE):
        got = G.ga_force_torque(plan, Ahat, Bhat4, t, mode).cpu().numpy()
        assert O.rel_l2(got[:, 0], ref[:, 0]) < FIELD_TOL
        assert O.rel_l2(got[:, 1:4], ref[:, 1:4]) < FORCE_TOL
        assert O.rel_l2(got[:, 4:7], ref[:, 4:7]) < FORCE_TOL


# ---------------------------------------------------------------------------
# force / torque
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,npts", [(24, 120), (48, 400), (96, 1000)])
def test_force_torque_fields_and_single(G, n, npts):
    A = _part(n, 7000 + n, npts, 1.0, 4.0)
    B = _part(n, 8000 + n, npts, 1.0, 4.0, conf=n / 6)
    R = synth.shoemake_rotations(9000 + n, 1)[0]
    cB = B.ref_point()
    d = O.pair_fields(A.xyzr, A.w, B.xyzr, B.w, R, cB, n)
    plan = G.Plan(n, max_batch=4)
    Ahat = G.ga_fft3d(plan, G.GA_R2C, G.ga_splat(plan, _dev(A.xyzr), _dev(A.w)))[0]
    Bhat4 = G.ga_fft3d(plan, G.GA_R2C, G.ga_splat(plan, _dev(B.xyzr), _dev(B.w), R=R, c=cB, channels=4))
    rng = np.random.default_rng(n)
    lat = (n // 2 + rng.integers(-n // 4, n // 4, (40, 3))).astype(np.float32)
    lat[0] = [0, 0, 0]
    lat[1] = [n - 1, n - 1, n - 1]
    frac = (lat[:20] + rng.random((20, 3))).astype(np.float32)
    fields = np.concatenate([d["E"][None], d["F"], d["tau"]])
    for mode, poses in ((G.GA_FIELDS, lat), (G.GA_FIELDS, frac), (G.GA_SINGLE, lat)):
        got = G.ga_force_torque(plan, Ahat, Bhat4, _dev(poses), mode).cpu().numpy()
        if np.all(poses == np.round(poses)):
            ref = O.lattice_read(fields, poses).T
        else:
            ref = O.trilinear_read(fields, poses).T
        assert O.rel_l2(got[:, 0], ref[:, 0]) < FIELD_TOL
        assert O.rel_l2(got[:, 1:4], ref[:, 1:4]) < FORCE_TOL
        assert O.rel_l2(got[:, 4:7], ref[:, 4:7]) < FORCE_TOL


def test_single_pose_rounds_to_nearest_lattice_point(G):
    n = 16
    A = _part(n, 11, 60, 1.0, 3.0)
    B = _part(n, 12, 60, 1.0, 3.0, conf=3.0)
    d = O.pair_fields(A.xyzr, A.w, B.xyzr, B.w, np.eye(3, dtype=np.float32), B.ref_point(), n)
    plan = G.Plan(n, max_batch=4)
    Ahat = G.ga_fft3d(plan, G.GA_R2C, G.ga_splat(plan, _dev(A.xyzr), _dev(A.w)))[0]
    Bhat4 = G.ga_fft3d(plan, G.GA_R2C, G.ga_splat(plan, _dev(B.xyzr), _dev(B.w), R=np.eye(3), c=B.ref_point(),
                                                   channels=4))
    poses = np.array([[7.4, 8.5, 9.6], [-0.5, 16.2, 31.49]], np.float32)
    got = G.ga_force_torque(plan, Ahat, Bhat4, _dev(poses), G.GA_SINGLE).cpu().numpy()
    lat = np.array([[7, 9, 10], [-1, 16, 31]], np.float32)  # round half away from zero
    fields = np.concatenate([d["E"][None], d["F"], d["tau"]])
    ref = O.lattice_read(fields, lat).T
    assert O.rel_l2(got, ref) < FORCE_TOL


# ---------------------------------------------------------------------------
# resident field (u_A, grad u_A) and single poses by local sums
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,npts", [(16, 40), (48, 300), (96, 900)])
def test_field_grad_matches_oracle(G, n, npts):
    A = _part(n, 500 + n, npts, 1.0, 4.0)
    uA = O.splat(A.xyzr[:, :3].astype(np.float64), A.xyzr[:, 3].astype(np.float64), A.w.astype(np.float64), n)
    g = O.grad_spectral(uA)
    plan = G.Plan(n)
    u = G.ga_splat(plan, _dev(A.xyzr), _dev(A.w))
    Ahat = G.ga_fft3d(plan, G.GA_R2C, u)[0]
    FA = G.ga_field_grad(plan, u[0], Ahat).cpu().numpy().astype(np.float64)
    assert O.rel_l2(FA[..., 0], uA) < FIELD_TOL
    assert O.rel_l2(np.moveaxis(FA[..., 1:], -1, 0), g) < FIELD_TOL


@pytest.mark.parametrize("n,npts,nrot", [(16, 40, 2), (24, 120, 3), (48, 400, 3), (96, 1000, 2)])
def test_pose_local_matches_oracle(G, n, npts, nrot):
    """Every pose has its own rotation; translations include both ends of
    the lattice, negative and non-integer values (rounded half away from
    zero), so that the gathers wrap on the torus."""
    A = _part(n, 600 + n, npts, 1.0, 4.0)
    B = _part(n, 700 + n, npts // 2 + 1, 1.0, 4.0, conf=n / 6)
    cB = B.ref_point()
    rots = synth.shoemake_rotations(800 + n, nrot)
    rng = np.random.default_rng(n)
    plan = G.Plan(n)
    u = G.ga_splat(plan, _dev(A.xyzr), _dev(A.w))
    FA = G.ga_field_grad(plan, u[0], G.ga_fft3d(plan, G.GA_R2C, u)[0])
    Rs, ts, refs = [], [], []
    for r in range(nrot):
        d = O.pair_fields(A.xyzr, A.w, B.xyzr, B.w, rots[r], cB, n)
        fields = np.concatenate([d["E"][None], d["F"], d["tau"]])
        t = (n // 2 + rng.integers(-n // 4, n // 4 + 1, (12, 3))).astype(np.float32)
        t[0] = [0, 0, 0]
        t[1] = [n - 1, n - 1, 0]
        t[2] = [-2, n + 3, 2 * n - 1]
        t[3] = [n / 2 + 0.5, n / 2 - 0.5, n / 2 + 0.4]
        lat = np.array([[np.floor(abs(v) + 0.5) * np.sign(v) for v in row] for row in t])
        refs.append(O.lattice_read(fields, lat).T)
        Rs.append(np.repeat(rots[r][None], len(t), 0))
        ts.append(t)
    got = G.ga_pose_local(plan, FA, _dev(B.xyzr), _dev(B.w), _dev(np.concatenate(Rs).astype(np.float32)), cB,
                          _dev(np.concatenate(ts))).cpu().numpy()
    ref = np.concatenate(refs)
    assert np.abs(ref[:, 0]).max() > 0
    assert O.rel_l2(got[:, 0], ref[:, 0]) < FIELD_TOL
    assert O.rel_l2(got[:, 1:4], ref[:, 1:4]) < FORCE_TOL
    assert O.rel_l2(got[:, 4:7], ref[:, 4:7]) < FORCE_TOL


@pytest.mark.timeout(600)
@pytest.mark.parametrize("n,npts,nrot", [(16, 40, 2), (24, 120, 3), (48, 400, 3), (64, 600, 2), (96, 1000, 2),
                                         (128, 2500, 3), (192, 1500, 2)])
def test_pose_spectral_matches_oracle(G, n, npts, nrot):
    """Re-correlated single poses (splat and z/y transforms of the rotated
    part per pose, each x-plane's share of the single-translation sums
    against the resident AX, DX): every pose its own rotation, translations
    at both ends of the lattice, negative and fractional (rounded half away
    from zero); against the oracle's single-pose sums and the local-sum
    entry point. 128 runs the two-stage kernel, the other edges the general
    one (with its radix-3 schedules at 24, 48, 96, 192)."""
    A = _part(n, 1600 + n, npts, 1.0, 4.0)
    B = _part(n, 1700 + n, npts // 2 + 1, 1.0, 4.0, conf=n / 6)
    cB = B.ref_point()
    rots = synth.shoemake_rotations(1800 + n, nrot)
    rng = np.random.default_rng(n + 1)
    ts = np.array([n / 2 + rng.uniform(-3, 3, 3) for _ in range(nrot)], np.float32)
    ts[0] = [n / 2 - 0.5, n / 2 + 1.5, -n + n / 2]  # ties and a negative translation
    plan = G.Plan(n, max_batch=4)
    u = G.ga_splat(plan, _dev(A.xyzr), _dev(A.w))
    Ahat = G.ga_fft3d(plan, G.GA_R2C, u)[0].contiguous()
    AX = G.ga_pose_prepare(plan, Ahat)
    R = _dev(rots.reshape(nrot, 9).astype(np.float32))
    got = G.ga_pose_spectral(plan, AX, _dev(B.xyzr), _dev(B.w), R, cB, _dev(ts)).cpu().numpy().astype(np.float64)
    FA = G.ga_field_grad(plan, u[0], Ahat)
    loc = G.ga_pose_local(plan, FA, _dev(B.xyzr), _dev(B.w), R, cB, _dev(ts)).cpu().numpy().astype(np.float64)
    uA = O.splat(A.xyzr[:, :3].astype(np.float64), A.xyzr[:, 3], A.w, n)
    g = O.grad_spectral(uA)
    ref = []
    for r in range(nrot):
        uB = O.splat(O.place(B.xyzr[:, :3], rots[r], cB), B.xyzr[:, 3], B.w, n)
        t_lat = [np.floor(abs(v) + 0.5) * np.sign(v) for v in ts[r]]
        ref.append(O.local_pose_sum(uA, uB, t_lat, grad=g))
    ref = np.array(ref)
    assert np.abs(ref[:, 0]).max() > 0
    for out in (got, loc):
        assert O.rel_l2(out[:, 0], ref[:, 0]) < FIELD_TOL
        assert O.rel_l2(out[:, 1:4], ref[:, 1:4]) < FORCE_TOL
        assert O.rel_l2(out[:, 4:7], ref[:, 4:7]) < FORCE_TOL


def test_pose_spectral_rejects_bad_arguments(G):
    n = 32
    plan = G.Plan(n)
    AX = torch.zeros((2, n, n, n // 2 + 1), dtype=torch.complex64, device="cuda")
    x = torch.zeros((4, 4), device="cuda")
    w = torch.ones(4, device="cuda")
    R = torch.eye(3, device="cuda").reshape(1, 9)
    t = torch.zeros((1, 3), device="cuda")
    with pytest.raises(G.GaError):  # sigma <= 0
        G.ga_pose_spectral(plan, AX, x, w, R, [0, 0, 0], t, sigma=0.0)
    with pytest.raises(G.GaError):  # workspace too small
        G.ga_pose_spectral(plan, AX, x, w, R, [0, 0, 0], t, work=torch.empty(16, dtype=torch.uint8, device="cuda"))
    big = G.Plan(256)
    with pytest.raises(G.GaError):  # the separate-axis edges have no fused pass
        G.ga_pose_prepare(big, torch.zeros((256, 256, 129), dtype=torch.complex64, device="cuda"))
    # no poses: nothing to do
    out = G.ga_pose_spectral(plan, AX, x, w, R[:0], [0, 0, 0], t[:0])
    assert out.shape == (0, 7)


def test_pose_local_edge_cases(G):
    n = 32
    A = _part(n, 31, 80, 1.0, 3.0)
    plan = G.Plan(n)
    u = G.ga_splat(plan, _dev(A.xyzr), _dev(A.w))
    FA = G.ga_field_grad(plan, u[0], G.ga_fft3d(plan, G.GA_R2C, u)[0])
    R = _dev(np.eye(3, dtype=np.float32)[None].repeat(2, 0))
    t = _dev(np.full((2, 3), 16.0, np.float32))
    # no samples: zero energy, force and torque
    empty = torch.zeros((0, 4), dtype=torch.float32, device="cuda")
    out = G.ga_pose_local(plan, FA, empty, torch.zeros(0, dtype=torch.float32, device="cuda"), R, [0, 0, 0], t)
    assert torch.count_nonzero(out).item() == 0
    # zero poses is a no-op; 65 samples span two sample blocks; zero weights add nothing
    B = _part(n, 32, 65, 1.0, 3.0, conf=5.0)
    G.ga_pose_local(plan, FA, _dev(B.xyzr), _dev(B.w), R[:0], B.ref_point(), t[:0])
    w0 = B.w.copy()
    w0[64] = 0.0
    full = G.ga_pose_local(plan, FA, _dev(B.xyzr), _dev(w0), R, B.ref_point(), t).cpu().numpy()
    first = G.ga_pose_local(plan, FA, _dev(np.ascontiguousarray(B.xyzr[:64])), _dev(np.ascontiguousarray(B.w[:64])),
                            R, B.ref_point(), t).cpu().numpy()
    assert np.array_equal(full[:, 0] != 0, first[:, 0] != 0)
    assert np.allclose(full, first, rtol=1e-6, atol=1e-12)
    # argument errors
    with pytest.raises(G.GaError):
        G.ga_pose_local(plan, FA, _dev(B.xyzr), _dev(B.w), R, B.ref_point(), t, sigma=0.0)
    with pytest.raises(G.GaError):
        G.ga_pose_local(plan, FA, _dev(B.xyzr), _dev(B.w), R, [np.nan, 0, 0], t)


def test_translations_that_are_not_finite_give_nan_outputs(G):
    """Device-resident translations are never converted to integers when they
    are NaN, infinite or beyond the float32 lattice: every readout gives NaN
    for such a pose and the usual values for the others."""
    n = 32
    A = _part(n, 41, 80, 1.0, 3.0)
    B = _part(n, 42, 60, 1.0, 3.0, conf=5.0)
    cB = B.ref_point()
    plan = G.Plan(n, max_batch=4)
    u = G.ga_splat(plan, _dev(A.xyzr), _dev(A.w))
    Ahat = G.ga_fft3d(plan, G.GA_R2C, u)[0].contiguous()
    Bhat4 = G.ga_fft3d(plan, G.GA_R2C, G.ga_splat(plan, _dev(B.xyzr), _dev(B.w), R=np.eye(3), c=cB, channels=4))
    poses = np.array([[16, 16, 16], [np.nan, 16, 16], [16, np.inf, 16], [16, 16, -np.inf], [3e38, 0, 0],
                      [15, 17, 16]], np.float32)
    good = [0, 5]
    bad = [1, 2, 3, 4]
    R = _dev(np.eye(3, dtype=np.float32)[None].repeat(len(poses), 0).reshape(-1, 9))
    FA = G.ga_field_grad(plan, u[0], Ahat)
    outs = {
        "fields": G.ga_force_torque(plan, Ahat, Bhat4, _dev(poses), G.GA_FIELDS),
        "single": G.ga_force_torque(plan, Ahat, Bhat4, _dev(poses), G.GA_SINGLE),
        "local": G.ga_pose_local(plan, FA, _dev(B.xyzr), _dev(B.w), R, cB, _dev(poses)),
        "spectral": G.ga_pose_spectral(plan, G.ga_pose_prepare(plan, Ahat), _dev(B.xyzr), _dev(B.w), R, cB,
                                       _dev(poses)),
    }
    ref = outs["single"].cpu().numpy()[good]
    for name, o in outs.items():
        o = o.cpu().numpy()
        assert np.all(np.isnan(o[bad])), name
        assert np.all(np.isfinite(o[good])), name
        assert O.rel_l2(o[good, 0], ref[:, 0]) < FIELD_TOL, name
        assert O.rel_l2(o[good, 1:], ref[:, 1:]) < FORCE_TOL, name


# ---------------------------------------------------------------------------
# full-size workloads
# ---------------------------------------------------------------------------

def test_c2_peg_in_hole_1000_poses(G):
    a = synth.config_c2()
    n = a.n
    plan = G.Plan(n, max_batch=4)
    Ahat = G.ga_fft3d(plan, G.GA_R2C, G.ga_splat(plan, _dev(a.A.xyzr), _dev(a.A.w), sigma=a.sigma))[0]
    Bhat4 = G.ga_fft3d(plan, G.GA_R2C, G.ga_splat(plan, _dev(a.B.xyzr), _dev(a.B.w), R=a.rotations[0], c=a.cB,
                                                   sigma=a.sigma, channels=4))
    got = G.ga_force_torque(plan, Ahat, Bhat4, _dev(a.poses), G.GA_FIELDS).cpu().numpy()
    d = O.pair_fields(a.A.xyzr, a.A.w, a.B.xyzr, a.B.w, a.rotations[0], a.cB, n, a.sigma)
    fields = np.concatenate([d["E"][None], d["F"], d["tau"]])
    ref = O.lattice_read(fields, a.poses).T
    assert np.abs(ref[:, 0]).max() > 0
    assert O.rel_l2(got[:, 0], ref[:, 0]) < FIELD_TOL
    assert O.rel_l2(got[:, 1:4], ref[:, 1:4]) < FORCE_TOL
    assert O.rel_l2(got[:, 4:7], ref[:, 4:7]) < FORCE_TOL
    # the same 1000 poses by local sums over the peg's balls
    u = G.ga_splat(plan, _dev(a.A.xyzr), _dev(a.A.w), sigma=a.sigma)
    FA = G.ga_field_grad(plan, u[0], Ahat)
    Rk = _dev(np.repeat(a.rotations[:1], len(a.poses), 0).astype(np.float32))
    loc = G.ga_pose_local(plan, FA, _dev(a.B.xyzr), _dev(a.B.w), Rk, a.cB, _dev(a.poses), a.sigma).cpu().numpy()
    assert O.rel_l2(loc[:, 0], ref[:, 0]) < FIELD_TOL
    assert O.rel_l2(loc[:, 1:4], ref[:, 1:4]) < FORCE_TOL
    assert O.rel_l2(loc[:, 4:7], ref[:, 4:7]) < FORCE_TOL


def test_c3_batched_rotations_full_size_sampled(G):
    """128^3, one stationary part against 64 rotations in one call (the
    benchmark's launch configuration); each field sampled at 16 translations
    where the oracle evaluates E(t) = sum_p u_A(p) u_B(p - t) directly."""
    a = synth.config_c3()
    n = a.n
    nrot = a.rotations.shape[0]
    plan = G.Plan(n, max_batch=nrot)
    Ahat = G.ga_fft3d(plan, G.GA_R2C, G.ga_splat(plan, _dev(a.A.xyzr), _dev(a.A.w), sigma=a.sigma))[0]
    E = G.ga_energy_fields(plan, Ahat, _dev(a.B.xyzr), _dev(a.B.w), _dev(a.rotations), a.cB, a.sigma)
    plan.set_overlap(2)  # the benchmark's timed configuration: two parts over two streams
    E2 = G.ga_energy_fields(plan, Ahat, _dev(a.B.xyzr), _dev(a.B.w), _dev(a.rotations), a.cB, a.sigma)
    torch.cuda.synchronize()
    uA = O.splat(a.A.xyzr[:, :3].astype(np.float64), a.A.xyzr[:, 3], a.A.w, n)
    ts = a.poses
    got_all, got2_all, ref_all = [], [], []
    for r in range(nrot):
        uB = O.splat(O.place(a.B.xyzr[:, :3], a.rotations[r], a.cB), a.B.xyzr[:, 3], a.B.w, n)
        ref_all.append(O.correlate_direct(uA, uB, ts))
        got_all.append(O.lattice_read(E[r].cpu().numpy(), ts))
        got2_all.append(O.lattice_read(E2[r].cpu().numpy(), ts))
    got_all, got2_all, ref_all = np.array(got_all), np.array(got2_all), np.array(ref_all)
    assert np.abs(ref_all).max() > 0
    assert O.rel_l2(got_all, ref_all) < FIELD_TOL
    assert O.rel_l2(got2_all, ref_all) < FIELD_TOL


# ---------------------------------------------------------------------------
# autotuned fused pass: every candidate gives the oracle's fields
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,npts,nrot", [(32, 200, 5), (64, 400, 3), (96, 700, 3), (48, 300, 2)])
def test_every_tuning_candidate_matches_oracle(G, n, npts, nrot):
    """Every strip width, member count, grid mapping and radix schedule of
    the fused x pass gives the oracle's fields (48 has no alternative
    schedule: radix 1 is refused there)."""
    A = _part(n, 900 + n, npts, 1.0, 3.0)
    B = _part(n, 950 + n, npts, 1.0, 3.0, conf=n / 6)
    rots = synth.shoemake_rotations(990 + n, nrot)
    cB = B.ref_point()
    plan = G.Plan(n, max_batch=nrot)
    Ahat = G.ga_fft3d(plan, G.GA_R2C, G.ga_splat(plan, _dev(A.xyzr), _dev(A.w)))[0].contiguous()
    refs = [O.pair_fields(A.xyzr, A.w, B.xyzr, B.w, rots[r], cB, n, want_torque=False)["E"] for r in range(nrot)]
    R = _dev(rots.reshape(nrot, 9).astype(np.float32))
    alt = plan.has_alt_radix()
    assert alt == (n != 48)
    for g, k, x, rx in G.Plan.TUNE_CANDIDATES:
        if rx == 1 and not alt:
            with pytest.raises(G.GaError):
                plan.set_radix(1)
            continue
        plan.set_tuning(g, k, x)
        plan.set_radix(rx)
        assert plan.tuning() == (g, k, x) and plan.radix() == rx
        E = G.ga_energy_fields(plan, Ahat, _dev(B.xyzr), _dev(B.w), R, cB).cpu().numpy()
        for r in range(nrot):
            assert O.rel_l2(E[r], refs[r]) < FIELD_TOL, (g, k, x, rx, r)
    choice, times = plan.autotune(Ahat, nrot)
    assert choice in G.Plan.AUTOTUNE_CANDIDATES and len(times) == (16 if alt else 8)
    assert all(t > 0 for t in times.values())
    E = G.ga_energy_fields(plan, Ahat, _dev(B.xyzr), _dev(B.w), R, cB).cpu().numpy()
    assert O.rel_l2(E[0], refs[0]) < FIELD_TOL
    with pytest.raises(G.GaError):
        plan.set_tuning(3, 4)
    with pytest.raises(G.GaError):
        plan.set_tuning(4, 3)
    with pytest.raises(G.GaError):
        plan.set_tuning(4, 4, 3)


def test_whole_call_tuning_is_cached_per_shape(G, tmp_path):
    """ga_plan_tune times the fused x pass (with the XCD-aware grid) and the
    part counts of whole calls, applies the fastest and stores it under
    "<arch>/<n>/<batch>/1"; a second plan of the same shape takes the stored
    choice without timing; the fields after tuning match the oracle; a cache
    file in another layout is refused and left as it was."""
    import json

    n, npts, nrot = 64, 600, 4
    A = _part(n, 1270, npts, 1.0, 3.0)
    B = _part(n, 1271, npts, 1.0, 3.0, conf=n / 6)
    rots = synth.shoemake_rotations(1272, nrot)
    cB = B.ref_point()
    R = _dev(rots.reshape(nrot, 9).astype(np.float32))
    path = str(tmp_path / "tune.json")
    plan = G.Plan(n, max_batch=nrot)
    Ahat = G.ga_fft3d(plan, G.GA_R2C, G.ga_splat(plan, _dev(A.xyzr), _dev(A.w)))[0].contiguous()
    got = plan.tune(Ahat, _dev(B.xyzr), _dev(B.w), R, cB, flags=G.ga.GA_TUNE_XCD | G.ga.GA_TUNE_OVERLAP,
                    cache_path=path)
    assert got["from_cache"] == 0 and got["us"] > 0
    assert (got["groups"], got["k"], got["xcd"], got["radix"]) in G.Plan.TUNE_CANDIDATES and got["overlap"] in (1, 2, 4)
    assert plan.tuning() == (got["groups"], got["k"], got["xcd"]) and plan.overlap() == got["overlap"]
    assert plan.radix() == got["radix"]
    stored = json.load(open(path))
    (key, entry), = stored.items()
    assert key.endswith(f"/{n}/{nrot}/1") and key.split("/")[0].startswith("gfx")
    keys = ("groups", "k", "xcd", "radix", "overlap")
    assert {k: entry[k] for k in keys} == {k: got[k] for k in keys}
    E = G.ga_energy_fields(plan, Ahat, _dev(B.xyzr), _dev(B.w), R, cB).cpu().numpy()
    for r in range(nrot):
        ref = O.pair_fields(A.xyzr, A.w, B.xyzr, B.w, rots[r], cB, n, want_torque=False)["E"]
        assert O.rel_l2(E[r], ref) < FIELD_TOL, r
    plan2 = G.Plan(n, max_batch=nrot)
    again = plan2.tune(Ahat, _dev(B.xyzr), _dev(B.w), R, cB, cache_path=path)
    assert again["from_cache"] == 1 and {k: again[k] for k in keys} == {k: got[k] for k in keys}
    assert plan2.tuning() == plan.tuning() and plan2.overlap() == plan.overlap() and plan2.radix() == plan.radix()
    # another batch size is another key: both kept
    plan3 = G.Plan(n, max_batch=nrot)
    plan3.tune(Ahat, _dev(B.xyzr), _dev(B.w), R[:2].contiguous(), cB, cache_path=path)
    assert len(json.load(open(path))) == 2
    bad = tmp_path / "bad.json"
    bad.write_text('{"gfx950/64/4/1": {"groups": 5}}\n')
    with pytest.raises(G.GaError):
        plan.tune(Ahat, _dev(B.xyzr), _dev(B.w), R, cB, cache_path=str(bad))
    assert bad.read_text() == '{"gfx950/64/4/1": {"groups": 5}}\n'


# ---------------------------------------------------------------------------
# overlapped execution: chunks of the batch over two streams
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,npts,nrot,chunks,k", [(32, 200, 7, 4, 4), (96, 700, 6, 2, 1), (128, 1500, 9, 4, 2)])
def test_overlapped_energy_fields_match_oracle(G, n, npts, nrot, chunks, k):
    A = _part(n, 1200 + n, npts, 1.0, 3.0)
    B = _part(n, 1250 + n, npts, 1.0, 3.0, conf=n / 6)
    rots = synth.shoemake_rotations(1290 + n, 2 * nrot)
    cB = B.ref_point()
    plan = G.Plan(n, max_batch=nrot)
    plan.set_tuning(4, k)
    Ahat = G.ga_fft3d(plan, G.GA_R2C, G.ga_splat(plan, _dev(A.xyzr), _dev(A.w)))[0].contiguous()
    R1 = _dev(rots[:nrot].reshape(nrot, 9).astype(np.float32))
    R2 = _dev(rots[nrot:].reshape(nrot, 9).astype(np.float32))
    xb, wb = _dev(B.xyzr), _dev(B.w)
    seq1 = G.ga_energy_fields(plan, Ahat, xb, wb, R1, cB).cpu().numpy()
    seq2 = G.ga_energy_fields(plan, Ahat, xb, wb, R2, cB).cpu().numpy()
    plan.set_overlap(chunks)
    assert plan.overlap() == chunks
    # two calls back to back on a side stream, sharing one workspace, read on
    # that stream right after: the second call's binning must wait for the
    # first call's second-stream work, and the reads for both
    s = torch.cuda.Stream()
    work = plan.workspace(G.ga.GA_OP_ENERGY, nrot, B.n)
    with torch.cuda.stream(s):
        E1 = G.ga_energy_fields(plan, Ahat, xb, wb, R1, cB, work=work, stream=s)
        E2 = G.ga_energy_fields(plan, Ahat, xb, wb, R2, cB, work=work, stream=s)
        sums = torch.stack([E1.double().sum(), E2.double().sum()])
    s.synchronize()
    E1, E2, sums = E1.cpu().numpy(), E2.cpu().numpy(), sums.cpu().numpy()
    assert O.rel_l2(E1, seq1) < 1e-6 and O.rel_l2(E2, seq2) < 1e-6
    assert sums[0] == pytest.approx(E1.astype(np.float64).sum(), rel=1e-12)
    assert sums[1] == pytest.approx(E2.astype(np.float64).sum(), rel=1e-12)
    for r in (0, nrot - 1):
        ref = O.pair_fields(A.xyzr, A.w, B.xyzr, B.w, rots[r], cB, n, want_torque=False)["E"]
        assert O.rel_l2(E1[r], ref) < FIELD_TOL, r
    plan.set_overlap(1)
    with pytest.raises(G.GaError):
        plan.set_overlap(3)


def test_misaligned_buffers_are_rejected(G):
    n = 32
    plan = G.Plan(n)
    p = _part(n, 77, 20)
    buf = torch.zeros(n ** 3 + 4, dtype=torch.float32, device="cuda")
    with pytest.raises(G.GaError):
        G.ga_splat(plan, _dev(p.xyzr), _dev(p.w), out=buf[1:1 + n ** 3].view(1, n, n, n))
    xyzr = torch.zeros(4 * p.n + 4, dtype=torch.float32, device="cuda")
    with pytest.raises(G.GaError):
        G.ga_splat(plan, xyzr[2:2 + 4 * p.n].view(p.n, 4), _dev(p.w))
    u = G.ga_splat(plan, _dev(p.xyzr), _dev(p.w), out=buf[4:4 + n ** 3].view(1, n, n, n))  # 16 bytes in: fine
    assert float(u.abs().sum()) > 0
