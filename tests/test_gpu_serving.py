"""GPU tests of the serving loop (ga_server_* / ga_submit / ga_poll):
results against the FP64 oracle, the same query alone and in a mix of many
concurrent queries of other pairs and grid sizes, admission and error paths.
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


def _pair(n, seed, npts):
    A = synth.random_part(seed, n, npts, 1.0, 3.0, conf_radius=n / 4)
    B = synth.random_part(seed + 1, n, npts, 1.0, 3.0, conf_radius=n / 6)
    return A, B


def _oracle_single(A, B, n, R, t, sigma=0.5):
    d = O.pair_fields(A.xyzr, A.w, B.xyzr, B.w, R, B.ref_point(), n, sigma)
    t_lat = np.array([[np.floor(abs(v) + 0.5) * np.sign(v) for v in t]])  # round half away from zero
    return np.concatenate([O.lattice_read(d["E"], t_lat), O.lattice_read(d["F"], t_lat)[:, 0],
                           O.lattice_read(d["tau"], t_lat)[:, 0]])


def _close(got, ref):
    got = np.asarray(got, np.float64)
    scale_f = max(np.linalg.norm(ref[1:4]), 1e-30)
    scale_t = max(np.linalg.norm(ref[4:7]), 1e-30)
    return (abs(got[0] - ref[0]) <= FIELD_TOL * max(abs(ref[0]), 1e-30)
            and np.linalg.norm(got[1:4] - ref[1:4]) <= FORCE_TOL * scale_f
            and np.linalg.norm(got[4:7] - ref[4:7]) <= FORCE_TOL * scale_t)


MODES = pytest.mark.parametrize("mode", ["local", "spectral"])


def _mode(G, mode):
    return G.GA_SERVE_LOCAL if mode == "local" else G.GA_SERVE_SPECTRAL


@MODES
def test_single_queries_match_oracle(G, mode):
    srv = G.Server(max_slots=4, queue_depth=64, mode=_mode(G, mode))
    try:
        for n, seed in ((32, 11), (48, 13)):
            A, B = _pair(n, seed, 150)
            pid = srv.register_pair(A.xyzr, A.w, B.xyzr, B.w, B.ref_point(), n)
            R = synth.shoemake_rotations(seed, 1)[0]
            t = [n / 2 + 1.4, n / 2 - 2.0, n / 2 + 0.6]
            res = srv.wait(srv.submit(pid, R, t))
            ref = _oracle_single(A, B, n, R, t)
            assert np.abs(ref[0]) > 0
            assert _close(res.values(), ref), (n, res.values(), ref)
            assert res.t_submit_ns <= res.t_start_ns <= res.t_done_ns
    finally:
        srv.close()


@MODES
def test_alone_and_in_the_mix_agree(G, mode):
    """A query's result does not depend on what else is in flight: the same
    query alone, then among 200 queries of 6 pairs on 3 grid sizes."""
    srv = G.Server(max_slots=8, queue_depth=1024, mode=_mode(G, mode))
    try:
        pairs = []
        for i, n in enumerate((32, 48, 64, 32, 48, 64)):
            A, B = _pair(n, 100 + 7 * i, 120 + 40 * i)
            pairs.append((srv.register_pair(A.xyzr, A.w, B.xyzr, B.w, B.ref_point(), n), n, A, B))
        probe_pid, probe_n, pA, pB = pairs[2]
        R = synth.shoemake_rotations(5, 1)[0]
        t = [probe_n / 2 + 1, probe_n / 2, probe_n / 2 - 1]
        alone = np.array(srv.wait(srv.submit(probe_pid, R, t)).values(), np.float64)
        rng = np.random.default_rng(0)
        rots = synth.shoemake_rotations(77, 256)
        tickets, probe = [], None
        for q in range(200):
            if q == 97:
                probe = srv.submit(probe_pid, R, t)
                continue
            pid, n, _, _ = pairs[rng.integers(len(pairs))]
            tickets.append(srv.submit(pid, rots[q], n / 2 + rng.integers(-3, 4, 3)))
        assert probe is not None and all(tk is not None for tk in tickets)
        mixed = np.array(srv.wait(probe).values(), np.float64)
        for tk in tickets:
            srv.wait(tk)
        ref = _oracle_single(pA, pB, probe_n, R, t)
        assert _close(alone, ref)
        assert _close(mixed, ref)
        assert _close(mixed, alone)
        st = srv.stats()
        assert st.completed == st.submitted == 201  # the lone probe and 200 in the mix
        assert st.launches < 201  # queries were batched
    finally:
        srv.close()


@MODES
def test_errors_and_admission(G, mode):
    srv = G.Server(max_slots=2, queue_depth=16, hbm_budget_bytes=8 << 20, mode=_mode(G, mode))
    try:
        A, B = _pair(32, 5, 60)
        pid = srv.register_pair(A.xyzr, A.w, B.xyzr, B.w, B.ref_point(), 32)
        I = np.eye(3)
        with pytest.raises(G.GaError):  # improper rotation
            srv.submit(pid, np.diag([1.0, 1.0, -1.0]), [0, 0, 0])
        with pytest.raises(G.GaError):  # unknown pair
            srv.submit(pid + 99, I, [0, 0, 0])
        with pytest.raises(G.GaError):  # unknown ticket
            srv.poll(123456789)
        tk = srv.submit(pid, I, [16, 16, 16])
        srv.wait(tk)
        with pytest.raises(G.GaError):  # a ticket completes once
            srv.poll(tk)
        with pytest.raises(G.GaError):  # a radius reaching n/2 is refused at registration
            bad = B.xyzr.copy()
            bad[0, 3] = 16.0
            srv.register_pair(A.xyzr, A.w, bad, B.w, B.ref_point(), 32)
        with pytest.raises(G.GaError):  # over the device-memory budget
            A2, B2 = _pair(128, 9, 100)
            srv.register_pair(A2.xyzr, A2.w, B2.xyzr, B2.w, B2.ref_point(), 128)
        srv.release_pair(pid)
        with pytest.raises(G.GaError):
            srv.submit(pid, I, [0, 0, 0])
        assert srv.stats().pairs == 0
    finally:
        srv.close()
    with pytest.raises(G.GaError):  # unknown mode
        G.Server(mode=7)


def test_local_and_spectral_modes_agree(G):
    """The two evaluation modes of the server give the same values for the
    same queries (rotations and translations drawn at random, 64^3)."""
    n = 64
    A, B = _pair(n, 21, 300)
    rots = synth.shoemake_rotations(22, 24)
    rng = np.random.default_rng(23)
    ts = n / 2 + rng.uniform(-4, 4, (24, 3))
    out = {}
    for mode in ("local", "spectral"):
        srv = G.Server(max_slots=8, queue_depth=64, mode=_mode(G, mode))
        try:
            pid = srv.register_pair(A.xyzr, A.w, B.xyzr, B.w, B.ref_point(), n)
            tks = [srv.submit(pid, rots[i], ts[i]) for i in range(24)]
            out[mode] = np.array([srv.wait(tk).values() for tk in tks], np.float64)
        finally:
            srv.close()
    ref = np.stack([_oracle_single(A, B, n, rots[i], ts[i]) for i in range(3)])
    for mode in out:
        assert O.rel_l2(out[mode][:3, 0], ref[:, 0]) < FIELD_TOL
        assert O.rel_l2(out[mode][:3, 1:], ref[:, 1:]) < FORCE_TOL
    assert O.rel_l2(out["local"][:, 0], out["spectral"][:, 0]) < FIELD_TOL
    assert O.rel_l2(out["local"][:, 1:4], out["spectral"][:, 1:4]) < FORCE_TOL
    assert O.rel_l2(out["local"][:, 4:7], out["spectral"][:, 4:7]) < FORCE_TOL


def _oracle_queries(A, B, n, rots, ts, sigma=0.5):
    """(E, F, tau) of each query (rotation of B about its reference point,
    translation rounded half away from zero) by the oracle's single-pose sums
    with the spectral gradient of u_A computed once."""
    uA = O.splat(A.xyzr[:, :3].astype(np.float64), A.xyzr[:, 3], A.w, n, sigma)
    g = O.grad_spectral(uA)
    out = []
    for R, t in zip(rots, ts):
        uB = O.splat(O.place(B.xyzr[:, :3], R, B.ref_point()), B.xyzr[:, 3], B.w, n, sigma)
        t_lat = [np.floor(abs(v) + 0.5) * np.sign(v) for v in t]
        out.append(O.local_pose_sum(uA, uB, t_lat, grad=g))
    return np.array(out)


@pytest.mark.timeout(900)
@MODES
def test_served_grid_sizes_match_oracle_alone_and_in_the_mix(G, mode):
    """The serving workload's grid sizes 96, 128 and 192 (64 is covered
    above), parts of 500-5000 samples with radii U[1,4]: two queries per size
    alone against the oracle, then the same queries again among 150 queries
    of the three sizes in flight together."""
    srv = G.Server(max_slots=8, queue_depth=1024, mode=_mode(G, mode))
    try:
        pairs = {}
        for i, (n, npts) in enumerate(((96, 600), (128, 2500), (192, 5000))):
            A = synth.random_part(300 + i, n, npts, 1.0, 4.0, conf_radius=n / 4)
            B = synth.random_part(350 + i, n, max(500, npts // 2), 1.0, 4.0, conf_radius=n / 6)
            rots = synth.shoemake_rotations(400 + i, 2)
            ts = [[n / 2 + 1.4, n / 2 - 2.0, n / 2 + 0.6], [n / 2 - 3.0, n / 2 + 2.5, n / 2]]
            pid = srv.register_pair(A.xyzr, A.w, B.xyzr, B.w, B.ref_point(), n)
            pairs[n] = (pid, rots, ts, _oracle_queries(A, B, n, rots, ts))
        alone = {}
        for n, (pid, rots, ts, ref) in pairs.items():
            got = np.array([srv.wait(srv.submit(pid, rots[q], ts[q])).values() for q in range(2)], np.float64)
            assert np.abs(ref[:, 0]).max() > 0 and np.abs(ref[:, 1:]).max() > 0
            assert O.rel_l2(got[:, 0], ref[:, 0]) < FIELD_TOL, n
            assert O.rel_l2(got[:, 1:4], ref[:, 1:4]) < FORCE_TOL, n
            assert O.rel_l2(got[:, 4:7], ref[:, 4:7]) < FORCE_TOL, n
            alone[n] = got
        rng = np.random.default_rng(9)
        others = synth.shoemake_rotations(450, 150)
        sizes = list(pairs)
        probes, tickets = {}, []
        for q in range(150):
            if q in (40, 41, 80, 81, 120, 121):
                n = sizes[(q - 40) // 40]
                pid, rots, ts, _ = pairs[n]
                probes[(n, q % 2)] = srv.submit(pid, rots[q % 2], ts[q % 2])
            n = sizes[rng.integers(3)]
            tickets.append(srv.submit(pairs[n][0], others[q], n / 2 + rng.integers(-3, 4, 3)))
        for (n, q), tk in probes.items():
            mixed = np.array(srv.wait(tk).values(), np.float64)
            assert O.rel_l2(mixed[0:1], alone[n][q, 0:1]) < FIELD_TOL, (n, q)
            assert O.rel_l2(mixed[1:4], alone[n][q, 1:4]) < FORCE_TOL, (n, q)
            assert O.rel_l2(mixed[4:7], alone[n][q, 4:7]) < FORCE_TOL, (n, q)
        for tk in tickets:
            srv.wait(tk)
    finally:
        srv.close()


def test_sticky_error_drops_queued_queries_and_close_returns(G):
    """A failed scratch reallocation (forced from the host with
    GA_TEST_FAIL_REGROW=1, nothing is launched) makes the server's error
    sticky: queries still queued are dropped and poll with that error, later
    calls return it, and close() returns."""
    import os
    import time

    srv = G.Server(max_slots=4, queue_depth=8192, mode=G.GA_SERVE_LOCAL)
    closed = False
    try:
        A, B = _pair(32, 61, 50)
        pid = srv.register_pair(A.xyzr, A.w, B.xyzr, B.w, B.ref_point(), 32)
        I = np.eye(3)
        tks = [srv.submit(pid, I, [16, 16, 16]) for _ in range(3000)]
        A2, B2 = _pair(32, 63, 120)  # more samples than the size class holds: regrow
        os.environ["GA_TEST_FAIL_REGROW"] = "1"
        try:
            with pytest.raises(G.GaError):
                srv.register_pair(A2.xyzr, A2.w, B2.xyzr, B2.w, B2.ref_point(), 32)
        finally:
            del os.environ["GA_TEST_FAIL_REGROW"]
        with pytest.raises(G.GaError):
            srv.submit(pid, I, [16, 16, 16])
        done = failed = 0
        for tk in tks:
            try:
                res = srv.poll(tk)
                done += res is not None
            except G.GaError:
                failed += 1
        assert done + failed > 0
        t0 = time.time()
        srv.close()
        closed = True
        assert time.time() - t0 < 30
    finally:
        if not closed:
            srv.close()
