"""Host-side tests of the serving scheduler with its test executor (no GPU):
the server schedules exactly as on the device (size-class queues, two launch
groups per size, continuous batching, admission by budget and queue depth,
sticky errors) while each launched query is answered by a callback. The
callback here is the FP64 oracle's single-pose sums (Sec. 3.3; the local
sums of S20), so the routing of pair, rotation and lattice translation
through the queues is checked against the oracle, alone and in a mix."""

import threading
import time

import numpy as np
import pytest

import oracle as O
import synth

GA_EDEVICE, GA_ENOMEM, GA_ENOTFOUND = -4, -2, -5


@pytest.fixture(scope="module")
def G():
    import paper_1711_05017_amd as pkg

    pkg.lib()
    return pkg


class OracleExecutor:
    """mock(pair_id, n, R, t) -> the oracle's (E, F, tau) of that pair at
    rotation R and lattice translation t (float32, as the device returns)."""

    def __init__(self):
        self.pairs = {}
        self.calls = []
        self.fail_pairs = set()
        self.lock = threading.Lock()

    def add(self, pid, A, B, cB, n):
        uA = O.splat(A.xyzr[:, :3].astype(np.float64), A.xyzr[:, 3], A.w, n)
        self.pairs[pid] = (uA, O.grad_spectral(uA), B, cB, n)

    def expected(self, pid, R, t_lat):
        uA, g, B, cB, n = self.pairs[pid]
        uB = O.splat(O.place(B.xyzr[:, :3], np.asarray(R, np.float64).reshape(3, 3), cB), B.xyzr[:, 3], B.w, n)
        return np.asarray(O.local_pose_sum(uA, uB, list(t_lat), grad=g), np.float64).astype(np.float32)

    def __call__(self, pid, n, R, t):
        with self.lock:
            self.calls.append((pid, n, tuple(t)))
        if pid in self.fail_pairs:
            raise RuntimeError("injected executor error")
        assert self.pairs[pid][4] == n
        return self.expected(pid, R, t)


def _lattice(t, n):
    """The server's lattice point: nearest, ties away from zero, modulo n."""
    return [int(np.floor(abs(v) + 0.5) * np.sign(v)) % n for v in t]


def _pairs(G, ex, server, sizes, seed):
    out = []
    for i, n in enumerate(sizes):
        A = synth.random_part(seed + 10 * i, n, 60, 1.0, 2.5)
        B = synth.random_part(seed + 10 * i + 1, n, 30, 1.0, 2.0, conf_radius=n / 6)
        cB = B.ref_point()
        pid = server.register_pair(A.xyzr, A.w, B.xyzr, B.w, cB, n)
        ex.add(pid, A, B, cB, n)
        out.append((pid, n))
    return out


def test_results_route_through_the_queues_alone_and_in_the_mix(G):
    ex = OracleExecutor()
    srv = G.Server(max_slots=3, mock=ex, mock_launch_us=300)
    try:
        pairs = _pairs(G, ex, srv, (16, 24, 32, 16), 700)
        rng = np.random.default_rng(5)
        queries = []
        for q in range(24):
            pid, n = pairs[q % len(pairs)]
            R = synth.shoemake_rotations(800 + q, 1)[0].astype(np.float32)
            t = rng.uniform(-n, 2 * n, 3).astype(np.float32)
            queries.append((pid, n, R, t))
        # alone: one query at a time
        alone = []
        for pid, n, R, t in queries:
            alone.append(srv.wait(srv.submit(pid, R, t)).values())
        # in the mix: all at once
        tickets = [srv.submit(pid, R, t) for pid, n, R, t in queries]
        mixed = [srv.wait(tk).values() for tk in tickets]
        for (pid, n, R, t), a, m in zip(queries, alone, mixed):
            ref = ex.expected(pid, R, _lattice(t, n))
            assert np.array_equal(np.asarray(a, np.float32), ref)
            assert np.array_equal(np.asarray(m, np.float32), ref)
        assert np.abs([r[0] for r in mixed]).max() > 0
        st = srv.stats()
        assert st.completed == st.submitted == 48 and st.rejected_full == 0
        assert st.launches < 48  # the burst was batched
    finally:
        srv.close()


def test_continuous_batching_admits_arrivals_as_groups_free(G):
    """Two groups of 2 slots per size: 4 queries start at once, the fifth and
    later start when a group completes; every ticket completes once."""
    ex = OracleExecutor()
    srv = G.Server(max_slots=2, mock=ex, mock_launch_us=30000)
    try:
        (pid, n), = _pairs(G, ex, srv, (16,), 900)
        tks = [srv.submit(pid, np.eye(3), [i, 0, 0]) for i in range(7)]
        res = [srv.wait(tk) for tk in tks]
        starts = sorted({r.t_start_ns for r in res})
        assert len(starts) == 4  # groups of 2, 2, 2, 1
        first_done = min(r.t_done_ns for r in res)
        late = [r for r in res if r.t_start_ns > starts[1]]
        assert late and all(r.t_start_ns >= first_done for r in late)
        for r in res:
            assert r.t_submit_ns <= r.t_start_ns and r.t_done_ns - r.t_start_ns >= 30e6
        assert srv.stats().launches == 4
        with pytest.raises(G.GaError) as e:  # a ticket completes exactly once
            srv.poll(tks[0])
        assert e.value.status == GA_ENOTFOUND
    finally:
        srv.close()


def test_admission_by_budget_and_queue_depth(G):
    ex = OracleExecutor()
    n = 32
    A = synth.random_part(1000, n, 40, 1.0, 2.0)
    # local mode holds 16 n^3 B per pair plus the launch groups' scratch
    budget = 16 * n ** 3 * 3 // 2  # room for one pair's field and the groups' scratch, not two fields
    srv = G.Server(hbm_budget_bytes=budget, max_slots=2, queue_depth=3, mock=ex, mock_launch_us=200000)
    try:
        pid = srv.register_pair(A.xyzr, A.w, A.xyzr, A.w, A.ref_point(), n)
        ex.add(pid, A, A, A.ref_point(), n)
        with pytest.raises(G.GaError) as e:
            srv.register_pair(A.xyzr, A.w, A.xyzr, A.w, A.ref_point(), n)
        assert e.value.status == GA_ENOMEM
        used = srv.stats().bytes_in_use
        assert 16 * n ** 3 <= used <= budget
        # one query into each of the two groups (each runs 200 ms), then 3
        # queued, then the queue is full
        tks = []
        for i in range(2):
            tks.append(srv.submit(pid, np.eye(3), [i, 0, 0]))
            time.sleep(0.02)  # the scheduler moves it into a free group
        tks += [srv.submit(pid, np.eye(3), [i, 0, 0]) for i in range(2, 5)]
        assert all(tk is not None for tk in tks)
        assert srv.submit(pid, np.eye(3), [0, 0, 0]) is None
        assert srv.stats().rejected_full == 1
        for tk in tks:
            srv.wait(tk)
        srv.release_pair(pid)
        assert srv.stats().pairs == 0 and srv.stats().bytes_in_use < used
        with pytest.raises(G.GaError):
            srv.submit(pid, np.eye(3), [0, 0, 0])
    finally:
        srv.close()


def test_executor_error_is_sticky_drains_queues_and_close_returns(G):
    ex = OracleExecutor()
    srv = G.Server(max_slots=1, mock=ex, mock_launch_us=20000)
    try:
        (p_ok, n1), (p_bad, n2) = _pairs(G, ex, srv, (16, 24), 1100)
        ok = srv.wait(srv.submit(p_ok, np.eye(3), [1, 2, 3]))
        assert np.array_equal(np.asarray(ok.values(), np.float32), ex.expected(p_ok, np.eye(3), [1, 2, 3]))
        ex.fail_pairs.add(p_bad)
        tks = [srv.submit(p_bad, np.eye(3), [i, 0, 0]) for i in range(5)]
        tks += [srv.submit(p_ok, np.eye(3), [i, 0, 0]) for i in range(3)]
        deadline = time.time() + 10
        failed = 0
        for tk in tks:
            while True:
                try:
                    if srv.poll(tk) is not None:
                        break
                except G.GaError as e:
                    assert e.status == GA_EDEVICE
                    failed += 1
                    break
                assert time.time() < deadline
                time.sleep(0.001)
        assert failed >= 5
        with pytest.raises(G.GaError) as e:
            srv.submit(p_ok, np.eye(3), [0, 0, 0])
        assert e.value.status == GA_EDEVICE
    finally:
        t0 = time.time()
        srv.close()
        assert time.time() - t0 < 5
