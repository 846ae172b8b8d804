"""GPU parity of the separate-axis path (splat into real grids, z transforms
per row pair, y and x transforms per strip of columns). At small grid edges
the path is forced with GA_PLAN_AXIS_PASSES and every entry point is compared
with the FP64 oracle element by element; 256^3 and 384^3 are checked against
closed forms (256^3, 384^3 and 512^3); the 512^3 workload (two parts of 50k
samples, 10k poses) is checked at 16 of its poses, both readouts against the
oracle's float64 energy, force and torque stored in tests/golden."""

import os

import numpy as np
import pytest
import torch

import oracle as O
import synth

pytestmark = pytest.mark.gpu

FIELD_TOL = 1e-5
FORCE_TOL = 1e-4
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


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


def _plan(G, n, batch=1):
    return G.Plan(n, max_batch=batch, flags=G.GA_PLAN_AXIS_PASSES)


@pytest.mark.parametrize("n,npts", [(32, 200), (96, 700)])
def test_axis_splat_matches_oracle(G, n, npts):
    p = _part(n, 1100 + n, npts, 0.5, 4.0)
    plan = _plan(G, n)
    R = synth.shoemake_rotations(17 + n, 1)[0]
    c = p.ref_point()
    got = G.ga_splat(plan, _dev(p.xyzr), _dev(p.w), R=R, c=c, channels=4).cpu().numpy()
    u = O.splat(O.place(p.xyzr[:, :3], R, c), p.xyzr[:, 3], p.w, n)
    ref = np.concatenate([u[None], O.moment_channels(u)])
    for ch in range(4):
        assert O.rel_l2(got[ch], ref[ch]) < FIELD_TOL, ch
    # empty input: zeros; a radius reaching n/2 contributes nothing
    z = G.ga_splat(plan, torch.zeros((0, 4), device="cuda"), torch.zeros(0, device="cuda"))
    assert float(z.abs().max()) == 0.0
    big = np.array([[4.0, 5.0, 6.0, n / 2.0]], np.float32)
    assert float(G.ga_splat(plan, _dev(big), _dev(np.ones(1, np.float32))).abs().max()) == 0.0


@pytest.mark.parametrize("n", [16, 24, 48, 64, 128, 192])
def test_axis_fft3d_matches_oracle(G, n):
    rng = np.random.default_rng(300 + n)
    batch = 2
    x = rng.standard_normal((batch, n, n, n)).astype(np.float32)
    plan = _plan(G, n, batch)
    X = G.ga_fft3d(plan, G.GA_R2C, _dev(x)).cpu().numpy()
    for b in range(batch):
        assert O.rel_l2(X[b], O.rfft3(x[b].astype(np.float64))) < FIELD_TOL
    H = (rng.standard_normal((batch, n, n, n // 2 + 1)) + 1j * rng.standard_normal((batch, n, n, n // 2 + 1)))
    H = H.astype(np.complex64)
    y = G.ga_fft3d(plan, G.GA_C2R, _dev(H)).cpu().numpy()
    for b in range(batch):
        assert O.rel_l2(y[b], O.irfft3(H[b].astype(np.complex128))) < FIELD_TOL


@pytest.mark.parametrize("n", [256, 384, 512])
def test_large_edges_plane_wave_and_roundtrip(G, n):
    """cos(2 pi k0.p / n) has the half spectrum n^3/2 at k0 (and at its mirror
    where k0 has kz = 0), zero elsewhere; C2R(R2C(x)) = x."""
    plan = G.Plan(n)
    k0 = (3, n - 5, 7)
    g = np.arange(n, dtype=np.float64)
    ph = (k0[0] * g[:, None, None] + k0[1] * g[None, :, None] + k0[2] * g[None, None, :]) % n
    x = np.cos(2 * np.pi * ph / n).astype(np.float32)
    X = G.ga_fft3d(plan, G.GA_R2C, _dev(x))[0]
    peak = X[k0[0], k0[1], k0[2]].cpu().numpy()
    assert abs(peak - n ** 3 / 2) < 1e-4 * n ** 3
    X[k0[0], k0[1], k0[2]] = 0
    assert float(X.abs().max()) < 1e-4 * n ** 3
    rng = np.random.default_rng(n)
    y = rng.standard_normal((n, n, n)).astype(np.float32)
    back = G.ga_fft3d(plan, G.GA_C2R, G.ga_fft3d(plan, G.GA_R2C, _dev(y))).cpu().numpy()[0]
    assert O.rel_l2(back, y) < FIELD_TOL


@pytest.mark.parametrize("n", [32, 96])
def test_axis_correlate_and_energy_fields(G, n):
    A = _part(n, 1200 + n, 250, 1.0, 4.0)
    B = _part(n, 1300 + n, 250, 1.0, 4.0)
    nrot = 3
    rots = synth.shoemake_rotations(1400 + n, nrot)
    cB = B.ref_point()
    plan = _plan(G, n, nrot)
    Ahat = G.ga_fft3d(plan, G.GA_R2C, G.ga_splat(plan, _dev(A.xyzr), _dev(A.w)))[0].contiguous()
    E = G.ga_energy_fields(plan, Ahat, _dev(B.xyzr), _dev(B.w), _dev(rots.reshape(nrot, 9).astype(np.float32)),
                           cB).cpu().numpy()
    uA = O.splat(A.xyzr[:, :3].astype(np.float64), A.xyzr[:, 3], A.w, n)
    for r in range(nrot):
        uB = O.splat(O.place(B.xyzr[:, :3], rots[r], cB), B.xyzr[:, 3], B.w, n)
        assert O.rel_l2(E[r], O.energy_field(uA, uB)) < FIELD_TOL, r
    # ga_correlate from oracle spectra
    uB = O.splat(O.place(B.xyzr[:, :3], rots[0], cB), B.xyzr[:, 3], B.w, n)
    Ah, Bh = O.rfft3(uA), O.rfft3(uB)
    got = G.ga_correlate(plan, _dev(Ah.astype(np.complex64)), _dev(Bh.astype(np.complex64)[None])).cpu().numpy()[0]
    assert O.rel_l2(got, O.energy_field(uA, uB)) < FIELD_TOL


def test_axis_force_torque_field_grad_pose_local(G):
    n = 48
    A = _part(n, 1500, 300, 1.0, 4.0)
    B = _part(n, 1501, 200, 1.0, 4.0, conf=n / 6)
    R = synth.shoemake_rotations(1502, 1)[0]
    cB = B.ref_point()
    d = O.pair_fields(A.xyzr, A.w, B.xyzr, B.w, R, cB, n)
    plan = _plan(G, n, 4)
    u = G.ga_splat(plan, _dev(A.xyzr), _dev(A.w))
    Ahat = G.ga_fft3d(plan, G.GA_R2C, u)[0].contiguous()
    Bhat4 = G.ga_fft3d(plan, G.GA_R2C, G.ga_splat(plan, _dev(B.xyzr), _dev(B.w), R=R, c=cB, channels=4))
    rng = np.random.default_rng(3)
    lat = (n // 2 + rng.integers(-n // 4, n // 4, (30, 3))).astype(np.float32)
    fields = np.concatenate([d["E"][None], d["F"], d["tau"]])
    ref = O.lattice_read(fields, lat).T
    for mode in (G.GA_FIELDS, G.GA_SINGLE):
        got = G.ga_force_torque(plan, Ahat, Bhat4, _dev(lat), mode).cpu().numpy()
        assert O.rel_l2(got[:, 0], ref[:, 0]) < FIELD_TOL
        assert O.rel_l2(got[:, 1:4], ref[:, 1:4]) < FORCE_TOL
        assert O.rel_l2(got[:, 4:7], ref[:, 4:7]) < FORCE_TOL
    FA = G.ga_field_grad(plan, u[0], Ahat).cpu().numpy().astype(np.float64)
    assert O.rel_l2(FA[..., 0], d["uA"]) < FIELD_TOL
    assert O.rel_l2(np.moveaxis(FA[..., 1:], -1, 0), O.grad_spectral(d["uA"])) < FIELD_TOL
    loc = G.ga_pose_local(plan, _dev(FA.astype(np.float32)), _dev(B.xyzr), _dev(B.w),
                          _dev(np.repeat(R[None], len(lat), 0).reshape(-1, 9).astype(np.float32)), cB,
                          _dev(lat)).cpu().numpy()
    assert O.rel_l2(loc[:, 0], ref[:, 0]) < FIELD_TOL
    assert O.rel_l2(loc[:, 1:4], ref[:, 1:4]) < FORCE_TOL
    assert O.rel_l2(loc[:, 4:7], ref[:, 4:7]) < FORCE_TOL


@pytest.mark.timeout(900)
def test_c4_512_fields_and_forces_against_oracle(G):
    """512^3, two parts of 50k samples (r log-uniform in [0.5, 8]), identity
    rotation, force/torque fields read at the workload's 10k poses. At 16 of
    those poses, drawn by the workload's own generator (8 uniform, 8 near
    contact), both readouts match the oracle's float64 single-pose sums stored
    by tests/golden/make_c4_golden.py (E = sum_q u_A(q + t) u_B(q), F and tau
    from the oracle's spectral gradient of u_A)."""
    gold = np.load(os.path.join(GOLDEN, "c4_512_poses.npz"))
    a = synth.config_c4()
    n = a.n
    idx = gold["indices"]
    assert int(gold["n"]) == n and np.array_equal(gold["poses"], a.poses[idx])
    ref = gold["values"]
    assert np.abs(ref[:, 0]).max() > 0 and np.abs(ref[:, 1:]).max() > 0
    plan = G.Plan(n, max_batch=4)
    Ahat = G.ga_fft3d(plan, G.GA_R2C, G.ga_splat(plan, _dev(a.A.xyzr), _dev(a.A.w), sigma=a.sigma))[0].contiguous()
    uB4 = G.ga_splat(plan, _dev(a.B.xyzr), _dev(a.B.w), R=np.eye(3), c=a.cB, sigma=a.sigma, channels=4)
    Bhat4 = G.ga_fft3d(plan, G.GA_R2C, uB4)
    del uB4
    torch.cuda.empty_cache()
    out = G.ga_force_torque(plan, Ahat, Bhat4, _dev(a.poses), G.GA_FIELDS).cpu().numpy()
    assert out.shape == (len(a.poses), 7) and np.all(np.isfinite(out))
    single = G.ga_force_torque(plan, Ahat, Bhat4, _dev(a.poses[idx]), G.GA_SINGLE).cpu().numpy()
    for got in (out[idx], single):
        assert O.rel_l2(got[:, 0], ref[:, 0]) < FIELD_TOL
        assert O.rel_l2(got[:, 1:4], ref[:, 1:4]) < FORCE_TOL
        assert O.rel_l2(got[:, 4:7], ref[:, 4:7]) < FORCE_TOL
