"""GPU check of ga_force_torque_noalloc, the GA_SINGLE readout that allocates
nothing (its partial sums live in the library's static device array): the
same outputs as ga_force_torque(..., GA_SINGLE, ...) with a workspace, on two
calls in a row (the second with a smaller input), within the oracle's
tolerances of the lattice fields; an input beyond the array is refused before
anything is enqueued."""

import ctypes

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


def _pair(G, n, seed, npts):
    A = synth.random_part(seed, n, npts, 1.0, 3.0)
    B = synth.random_part(seed + 1, n, npts, 1.0, 3.0, conf_radius=n / 4)
    R = synth.shoemake_rotations(seed + 2, 1)[0]
    cB = B.ref_point()
    plan = G.Plan(n, max_batch=4)
    Ahat = G.ga_fft3d(plan, G.GA_R2C, G.ga_splat(plan, _dev(A.xyzr), _dev(A.w)))[0]
    Bhat4 = G.ga_fft3d(plan, G.GA_R2C, G.ga_splat(plan, _dev(B.xyzr), _dev(B.w), R=R, c=cB, channels=4))
    ref = O.pair_fields(A.xyzr, A.w, B.xyzr, B.w, R, cB, n)
    fields = np.concatenate([ref["E"][None], ref["F"], ref["tau"]])
    return plan, Ahat, Bhat4, fields


def _poses(n, count, seed):
    rng = np.random.default_rng(seed)
    lat = rng.integers(-n, 2 * n, (count, 3)).astype(np.float32)
    lat[: count // 2] = (rng.integers(-3, 4, (count // 2, 3)) + n // 2).astype(np.float32)  # near contact
    return lat


def _check_vs_oracle(got, fields, poses):
    ref = O.lattice_read(fields, poses).T
    assert O.rel_l2(got[:, 0], ref[:, 0]) < FIELD_TOL
    assert O.rel_l2(got[:, 1:4], ref[:, 1:4]) < FORCE_TOL
    assert O.rel_l2(got[:, 4:7], ref[:, 4:7]) < FORCE_TOL


def test_noalloc_matches_workspace_call_twice(G):
    """Two calls in a row on the shared array: 64^3 with 700 poses, then 32^3
    with 37 poses (smaller input, and a different partial-sum layout), each
    equal to the workspace call and within tolerance of the oracle."""
    for n, npts, count, seed in ((64, 600, 700, 11), (32, 200, 37, 12)):
        plan, Ahat, Bhat4, fields = _pair(G, n, 9000 + n, npts)
        poses = _poses(n, count, seed)
        t = _dev(poses)
        want = G.ga_force_torque(plan, Ahat, Bhat4, t, G.GA_SINGLE)
        out = torch.full((count, 7), float("nan"), dtype=torch.float32, device="cuda")
        G.ga_force_torque_noalloc(plan, Ahat, Bhat4, t, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.array_equal(got, want.cpu().numpy())  # same kernels, fixed-order float64 sums
        _check_vs_oracle(got.astype(np.float64), fields, poses)


def test_noalloc_refuses_input_beyond_scratch(G):
    n = 32
    plan = G.Plan(n)
    h = (n // 2 + 1) * n
    per_pose = -(-h // 64) * 7 * 8
    too_many = G.ga.GA_NOALLOC_SCRATCH_BYTES // per_pose + 1
    spec = torch.zeros((4, n, n, n // 2 + 1), dtype=torch.complex64, device="cuda")
    t = torch.zeros((too_many, 3), dtype=torch.float32, device="cuda")
    out = torch.zeros((too_many, 7), dtype=torch.float32, device="cuda")
    lib = G.lib()
    st = lib.ga_force_torque_noalloc(plan.handle, ctypes.c_void_p(spec.data_ptr()), ctypes.c_void_p(spec.data_ptr()),
                                     ctypes.c_void_p(t.data_ptr()), too_many, ctypes.c_void_p(out.data_ptr()), None)
    assert st == -2  # GA_ENOMEM, nothing enqueued
    assert lib.ga_force_torque_noalloc(None, None, None, None, 1, None, None) == -1
