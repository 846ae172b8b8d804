"""GPU parity of spectral rotation (Sec. 3.2, step 1): the interpolated
spectra against the oracle's, element by element, and the energy of a cube
rotation against the re-splat path (the two are the same function then)."""

import numpy as np
import pytest
import torch

import oracle as O
import synth

pytestmark = pytest.mark.gpu

FIELD_TOL = 1e-5


@pytest.fixture(scope="module")
def G():
    import paper_1711_05017_amd as pkg

    pkg.lib()
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    return pkg


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("n", [24, 32, 64, 96])
def test_spectral_rotation_matches_oracle(G, n):
    A = synth.random_part(3000 + n, n, 150, 1.0, 3.0, conf_radius=n / 4)
    B = synth.random_part(3100 + n, n, 80, 1.0, 2.5, conf_radius=n / 8)
    cB = B.ref_point()
    Q = np.array([[0, -1, 0], [0, 0, 1], [-1, 0, 0]], np.float32)  # a cube rotation
    rots = np.stack([np.eye(3, dtype=np.float32), Q, *synth.shoemake_rotations(3200 + n, 2)]).astype(np.float32)
    plan = G.Plan(n, max_batch=4)
    X4 = G.ga_fft3d(plan, G.GA_R2C, G.ga_splat(plan, _dev(B.xyzr), _dev(B.w), R=np.eye(3), c=cB, channels=4))
    got = G.ga_spectral_rotate(plan, X4, _dev(rots.reshape(-1, 9))).cpu().numpy()
    u = O.splat(O.place(B.xyzr[:, :3], np.eye(3), cB), B.xyzr[:, 3], B.w, n)
    F4 = np.stack([O.fft3(u)] + [O.fft3(m) for m in O.moment_channels(u)])
    for b, R in enumerate(rots):
        ref = O.spectral_rotate4(F4, R)[:, :, :, : n // 2 + 1]
        for ch in range(4):
            assert O.rel_l2(got[b, ch], ref[ch]) < FIELD_TOL, (b, ch)
    # energy: rotated spectrum vs the re-splat path; exact for the cube rotation
    Ahat = G.ga_fft3d(plan, G.GA_R2C, G.ga_splat(plan, _dev(A.xyzr), _dev(A.w)))[0].contiguous()
    Erot = G.ga_correlate(plan, Ahat, torch.from_numpy(got[:, 0]).cuda().contiguous()).cpu().numpy()
    Eres = G.ga_energy_fields(plan, Ahat, _dev(B.xyzr), _dev(B.w), _dev(rots.reshape(-1, 9)), cB).cpu().numpy()
    assert O.rel_l2(Erot[0], Eres[0]) < FIELD_TOL
    assert O.rel_l2(Erot[1], Eres[1]) < FIELD_TOL
    for b in (2, 3):
        assert O.rel_l2(Erot[b], Eres[b]) < 0.35  # interpolation of the spectrum approximates the re-splat
    with pytest.raises(G.GaError):  # two channels
        G.ga_spectral_rotate(plan, X4[:2].contiguous(), _dev(rots.reshape(-1, 9)))


def test_spectral_rotation_128_and_batch_stride(G):
    """128^3 (many LDS tiles per axis) with a batch larger than the rotations
    used by the oracle check: every member must equal its own rotation."""
    n = 128
    B = synth.random_part(3400, n, 300, 1.0, 4.0, conf_radius=n / 6)
    cB = B.ref_point()
    rots = synth.shoemake_rotations(3401, 5).astype(np.float32)
    plan = G.Plan(n, max_batch=8)
    X4 = G.ga_fft3d(plan, G.GA_R2C, G.ga_splat(plan, _dev(B.xyzr), _dev(B.w), R=np.eye(3), c=cB, channels=4))
    got = G.ga_spectral_rotate(plan, X4, _dev(rots.reshape(-1, 9))).cpu().numpy()
    one = G.ga_spectral_rotate(plan, X4, _dev(rots[3:4].reshape(-1, 9))).cpu().numpy()
    assert np.array_equal(one[0], got[3])
    u = O.splat(O.place(B.xyzr[:, :3], np.eye(3), cB), B.xyzr[:, 3], B.w, n)
    F4 = np.stack([O.fft3(u)] + [O.fft3(m) for m in O.moment_channels(u)])
    ref = O.spectral_rotate4(F4, rots[3])[:, :, :, : n // 2 + 1]
    for ch in range(4):
        assert O.rel_l2(got[3, ch], ref[ch]) < FIELD_TOL, ch


@pytest.mark.parametrize("n", [24, 64, 128])
def test_packed_rotation_matches_planar_and_oracle(G, n):
    """The packed source (one 32-byte record of the 4 channels per frequency)
    gives the planar path's outputs: the same corners, weights and summation
    order per channel, so equal values; and the oracle's rotated spectra, for
    rotations (which load only the box elements an interpolation can read)
    and for a scaled rotation (which loads every box element)."""
    B = synth.random_part(3500 + n, n, 120, 1.0, 3.0, conf_radius=n / 6)
    cB = B.ref_point()
    rots = np.concatenate([np.eye(3, dtype=np.float32)[None], synth.shoemake_rotations(3600 + n, 3)]).astype(np.float32)
    rots[3] *= 1.01  # not orthogonal: every box element is loaded
    plan = G.Plan(n, max_batch=4)
    X4 = G.ga_fft3d(plan, G.GA_R2C, G.ga_splat(plan, _dev(B.xyzr), _dev(B.w), R=np.eye(3), c=cB, channels=4))
    P = G.ga_spectral_pack4(plan, X4)
    Xh = X4.cpu().numpy()
    Ph = P.cpu().numpy()
    for ch in range(4):
        assert np.array_equal(Ph[..., ch], Xh[ch])
    Rd = _dev(rots.reshape(-1, 9))
    planar = G.ga_spectral_rotate(plan, X4, Rd).cpu().numpy()
    packed = G.ga_spectral_rotate_packed(plan, P, Rd).cpu().numpy()
    assert np.array_equal(packed, planar)
    u = O.splat(O.place(B.xyzr[:, :3], np.eye(3), cB), B.xyzr[:, 3], B.w, n)
    F4 = np.stack([O.fft3(u)] + [O.fft3(m) for m in O.moment_channels(u)])
    for b in (0, 2, 3):
        ref = O.spectral_rotate4(F4, rots[b])[:, :, :, : n // 2 + 1]
        for ch in range(4):
            assert O.rel_l2(packed[b, ch], ref[ch]) < FIELD_TOL, (b, ch)
    with pytest.raises(G.GaError):  # output overlapping the packed source
        G.ga_spectral_rotate_packed(plan, P, Rd[:1].contiguous(), out=P.view(1, 4, n, n, n // 2 + 1))
