"""A stationary spectrum computed on the GPU, stored, and loaded back (in
place of recomputing it) gives the same bits and the same energy fields,
which still match the FP64 oracle."""

import numpy as np
import pytest
import torch

import oracle as O
import synth

pytestmark = pytest.mark.gpu

FIELD_TOL = 1e-5


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("n,npts,nrot", [(32, 200, 2), (128, 1500, 2)])
def test_stored_spectrum_replaces_the_fresh_one(tmp_path, n, npts, nrot):
    import paper_1711_05017_amd as G

    G.lib()
    torch.cuda.set_device(0)
    A = synth.random_part(8100 + n, n, npts, 1.0, 3.0)
    B = synth.random_part(8200 + n, n, npts, 1.0, 3.0)
    R = synth.shoemake_rotations(8300 + n, nrot)
    cB = B.ref_point()
    sigma = 0.5
    plan = G.Plan(n, max_batch=nrot)
    Ahat = G.ga_fft3d(plan, G.GA_R2C, G.ga_splat(plan, _dev(A.xyzr), _dev(A.w), sigma=sigma))[0].contiguous()

    key = G.skeleton_key(A.xyzr, A.w, n, sigma)
    assert G.load_spectrum(str(tmp_path), key, n, device="cuda") is None
    G.save_spectrum(str(tmp_path), key, Ahat, n, sigma)
    A2 = G.load_spectrum(str(tmp_path), key, n, sigma=sigma, device="cuda")[0].contiguous()
    assert A2.is_cuda and torch.equal(torch.view_as_real(A2), torch.view_as_real(Ahat))

    xb, wb, Rd = _dev(B.xyzr), _dev(B.w), _dev(R)
    E1 = G.ga_energy_fields(plan, Ahat, xb, wb, Rd, cB, sigma)
    E2 = G.ga_energy_fields(plan, A2, xb, wb, Rd, cB, sigma)
    torch.cuda.synchronize()
    assert torch.equal(E1, E2)

    uA = O.splat(A.xyzr[:, :3].astype(np.float64), A.xyzr[:, 3], A.w, n, sigma)
    E = E2.cpu().numpy()
    for r in range(nrot):
        uB = O.splat(O.place(B.xyzr[:, :3], R[r], cB), B.xyzr[:, 3], B.w, n, sigma)
        assert O.rel_l2(E[r], O.energy_field(uA, uB)) < FIELD_TOL, r
