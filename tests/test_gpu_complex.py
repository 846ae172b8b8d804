"""GPU parity of the score function of complex affinities (eq. 3 and eq. 5
with the reflection of the moving part; interior/exterior skeletons of
Sec. 2.3) against the oracle's complex transforms."""

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


def _two_channel_part(seed, n, npts, conf):
    """Interior and exterior skeleton samples: imaginary-channel weights +1 /
    -PENALTY, and an independent real channel (random weights) so that both
    halves of the complex product are exercised."""
    P = synth.random_part(seed, n, npts, 1.0, 3.0, conf_radius=conf)
    rng = np.random.default_rng(seed)
    ext = rng.random(P.n) < 0.4
    w_im = np.where(ext, -synth.PENALTY, 1.0).astype(np.float32)
    w_re = rng.uniform(-1.0, 1.0, P.n).astype(np.float32)
    return P.xyzr, w_re, w_im


def _spectra(G, plan, xyzr, w_re, w_im, R=None, c=None):
    chans = [G.ga_fft3d(plan, G.GA_R2C, G.ga_splat(plan, _dev(xyzr), _dev(w), R=R, c=c))[0] for w in (w_re, w_im)]
    return torch.stack(chans).contiguous()


def _oracle_rho(xyzr, w_re, w_im, n, R=None, c=None):
    y = xyzr[:, :3].astype(np.float64) if R is None else O.place(xyzr[:, :3], R, c)
    return O.splat(y, xyzr[:, 3], w_re, n) + 1j * O.splat(y, xyzr[:, 3], w_im, n)


@pytest.mark.parametrize("n,flags", [(32, 0), (96, 0), (128, 0), (64, 1)])
def test_score_matches_oracle(G, n, flags):
    print(f"score parity n={n} flags={flags}", flush=True)
    xa, ar, ai = _two_channel_part(3000 + n, n, 160, n / 4)
    xb, br, bi = _two_channel_part(3100 + n, n, 120, n / 6)
    cB = xb[:, :3].astype(np.float64).mean(0).astype(np.float32)
    Rs = synth.shoemake_rotations(3200 + n, 3)
    plan = G.Plan(n, max_batch=4, flags=flags)
    A2 = _spectra(G, plan, xa, ar, ai)
    B2 = torch.stack([_spectra(G, plan, xb, br, bi, R=R, c=cB) for R in Rs]).contiguous()
    out = G.ga_score(plan, A2, B2).cpu().numpy()
    assert out.shape == (3, 2, n, n, n)
    rho1 = _oracle_rho(xa, ar, ai, n)
    for b, R in enumerate(Rs):
        f = O.score_fft(rho1, _oracle_rho(xb, br, bi, n, R, cB))
        assert np.abs(f.real).max() > 0 and np.abs(f.imag).max() > 0
        assert O.rel_l2(out[b, 0], f.real) < FIELD_TOL, (n, b, "re")
        assert O.rel_l2(out[b, 1], f.imag) < FIELD_TOL, (n, b, "im")


def test_score_parts_and_per_member_stationary_spectra(G):
    n = 48
    plan = G.Plan(n, max_batch=4)
    parts = [_two_channel_part(3300 + k, n, 80, n / 5) for k in range(3)]
    S = [_spectra(G, plan, *p) for p in parts]
    B2 = torch.stack(S[1:]).contiguous()
    both = G.ga_score(plan, S[0], B2).cpu().numpy()
    re = G.ga_score(plan, S[0], B2, parts=G.GA_SCORE_RE).cpu().numpy()
    im = G.ga_score(plan, S[0], B2, parts=G.GA_SCORE_IM).cpu().numpy()
    assert re.shape == (2, 1, n, n, n) and im.shape == (2, 1, n, n, n)
    assert np.array_equal(re[:, 0], both[:, 0]) and np.array_equal(im[:, 0], both[:, 1])
    # one stationary pair per member (a_stride = 2 spectra)
    A2s = torch.stack([S[2], S[0]]).contiguous()
    per = G.ga_score(plan, A2s, B2).cpu().numpy()
    ref1 = G.ga_score(plan, S[2], B2[:1].contiguous()).cpu().numpy()
    assert np.array_equal(per[0], ref1[0]) and np.array_equal(per[1], both[1])
    # the score against itself is symmetric under t -> -t for real parts: spot
    # check against the oracle at a few translations from the samples
    rho = [_oracle_rho(*p, n) for p in parts]
    ts = np.random.default_rng(5).integers(0, n, (6, 3))
    ref = O.score_direct(rho[0], rho[1], ts)
    got = both[0, 0][ts[:, 0], ts[:, 1], ts[:, 2]] + 1j * both[0, 1][ts[:, 0], ts[:, 1], ts[:, 2]]
    assert O.rel_l2(got, ref) < FIELD_TOL


def test_score_errors(G):
    n = 32
    plan = G.Plan(n, max_batch=2)
    A2 = torch.zeros((2, n, n, n // 2 + 1), dtype=torch.complex64, device="cuda")
    B2 = torch.zeros((1, 2, n, n, n // 2 + 1), dtype=torch.complex64, device="cuda")
    for parts in (0, 4, 7):
        with pytest.raises(G.GaError):
            G.ga_score(plan, A2, B2, parts=parts)
    with pytest.raises(G.GaError):  # output overlapping the input
        G.ga_score(plan, A2, B2, out=B2.view(torch.float32).reshape(-1)[: 2 * n ** 3].view(1, 2, n, n, n))
    with pytest.raises(G.GaError):  # short workspace
        G.ga_score(plan, A2, B2, work=torch.empty(16, dtype=torch.uint8, device="cuda"))


def test_peg_in_hole_with_exterior_hole_axis_snaps_in(G):
    """C2 with the hole's axis as an exterior skeleton: the best score over all
    translations is the inserted pose, and the field agrees with the oracle."""
    a = synth.config_c2(4, exterior=True)
    n = a.n
    plan = G.Plan(n, max_batch=2)
    zA, zB = np.zeros(a.A.n, np.float32), np.zeros(a.B.n, np.float32)
    I3 = np.eye(3, dtype=np.float32)
    A2 = _spectra(G, plan, a.A.xyzr, zA, a.A.w)
    B2 = _spectra(G, plan, a.B.xyzr, zB, a.B.w, R=I3, c=a.cB)[None].contiguous()
    f = G.ga_score(plan, A2, B2, parts=G.GA_SCORE_RE).cpu().numpy()[0, 0]
    assert np.unravel_index(np.argmax(f), f.shape) == (64, 64, 64)
    ref = O.score_fft(1j * O.splat(a.A.xyzr[:, :3], a.A.xyzr[:, 3], a.A.w, n, a.sigma),
                      1j * O.splat(O.place(a.B.xyzr[:, :3], I3, a.cB), a.B.xyzr[:, 3], a.B.w, n, a.sigma)).real
    assert O.rel_l2(f, ref) < FIELD_TOL
