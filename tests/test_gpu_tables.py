"""GPU parity of field tables for restricted orientations (Sec. 4.2): the 7
fields per orientation against the oracle's, read at lattice and fractional
translations by queries that mix orientations."""

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


def test_field_tables_match_oracle(G):
    n = 32
    A = synth.random_part(4000, n, 200, 1.0, 3.0, conf_radius=n / 4)
    B = synth.random_part(4001, n, 120, 1.0, 3.0, conf_radius=n / 6)
    cB = B.ref_point()
    rots = np.stack([np.eye(3, dtype=np.float32), *synth.shoemake_rotations(4002, 2)]).astype(np.float32)
    plan = G.Plan(n, max_batch=4)
    Ahat = G.ga_fft3d(plan, G.GA_R2C, G.ga_splat(plan, _dev(A.xyzr), _dev(A.w)))[0].contiguous()
    B4 = torch.stack([G.ga_fft3d(plan, G.GA_R2C, G.ga_splat(plan, _dev(B.xyzr), _dev(B.w), R=R, c=cB, channels=4))
                      for R in rots]).contiguous()
    tables = G.ga_field_table(plan, Ahat, B4)
    assert tables.shape == (3, n, n, n, 8)
    assert float(tables[..., 7].abs().max()) == 0.0
    fields = []
    for R in rots:
        d = O.pair_fields(A.xyzr, A.w, B.xyzr, B.w, R, cB, n)
        fields.append(np.concatenate([d["E"][None], d["F"], d["tau"]]))
    for o in range(3):
        t7 = np.moveaxis(tables[o, ..., :7].cpu().numpy(), -1, 0)
        assert O.rel_l2(t7[0], fields[o][0]) < FIELD_TOL
        assert O.rel_l2(t7[1:4], fields[o][1:4]) < FORCE_TOL
        assert O.rel_l2(t7[4:7], fields[o][4:7]) < FORCE_TOL
    rng = np.random.default_rng(5)
    nq = 60
    orient = rng.integers(0, 3, nq).astype(np.int32)
    t = (n / 2 + rng.uniform(-6, 6, (nq, 3))).astype(np.float32)
    t[:20] = np.round(t[:20])
    got = G.ga_field_table_query(plan, tables, _dev(orient), _dev(t)).cpu().numpy()
    ref = np.stack([O.trilinear_read(fields[o], t[q:q + 1])[:, 0] for q, o in enumerate(orient)])
    assert O.rel_l2(got[:, 0], ref[:, 0]) < FIELD_TOL
    assert O.rel_l2(got[:, 1:4], ref[:, 1:4]) < FORCE_TOL
    assert O.rel_l2(got[:, 4:7], ref[:, 4:7]) < FORCE_TOL
    bad = G.ga_field_table_query(plan, tables, _dev(np.array([-1, 3, 1], np.int32)), _dev(t[:3])).cpu().numpy()
    assert np.all(np.isnan(bad[:2])) and np.all(np.isfinite(bad[2]))


def test_field_tables_128_sampled(G):
    """128^3 tables (the benchmark grid) for two orientations, read at lattice
    translations and compared with the oracle's single-translation sums of
    eq. 7b from its own spectra."""
    n = 128
    A = synth.random_part(4100, n, 1500, 1.0, 4.0, conf_radius=n / 4)
    B = synth.random_part(4101, n, 1000, 1.0, 4.0, conf_radius=n / 6)
    cB = B.ref_point()
    rots = np.stack([np.eye(3, dtype=np.float32), synth.shoemake_rotations(4102, 1)[0]]).astype(np.float32)
    plan = G.Plan(n, max_batch=4)  # the 4-channel transforms
    Ahat = G.ga_fft3d(plan, G.GA_R2C, G.ga_splat(plan, _dev(A.xyzr), _dev(A.w)))[0].contiguous()
    B4 = torch.stack([G.ga_fft3d(plan, G.GA_R2C, G.ga_splat(plan, _dev(B.xyzr), _dev(B.w), R=R, c=cB, channels=4))
                      for R in rots]).contiguous()
    tables = G.ga_field_table(plan, Ahat, B4)
    rng = np.random.default_rng(41)
    t = (n // 2 + rng.integers(-12, 13, (10, 3))).astype(np.float32)
    orient = np.array([0, 1] * 5, np.int32)
    got = G.ga_field_table_query(plan, tables, _dev(orient), _dev(t)).cpu().numpy()
    Ah = O.fft3(O.splat(A.xyzr[:, :3].astype(np.float64), A.xyzr[:, 3], A.w, n))
    ref = np.zeros((len(t), 7))
    for o, R in enumerate(rots):
        uB = O.splat(O.place(B.xyzr[:, :3], R, cB), B.xyzr[:, 3], B.w, n)
        Bh = O.fft3(uB)
        Mh = np.stack([O.fft3(m) for m in O.moment_channels(uB)])
        for q in np.nonzero(orient == o)[0]:
            ref[q] = O.single_pose_sum(Ah, Bh, Mh, t[q])
    assert np.abs(ref[:, 0]).max() > 0
    assert O.rel_l2(got[:, 0], ref[:, 0]) < FIELD_TOL
    assert O.rel_l2(got[:, 1:4], ref[:, 1:4]) < FORCE_TOL
    assert O.rel_l2(got[:, 4:7], ref[:, 4:7]) < FORCE_TOL
