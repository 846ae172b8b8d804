"""CPU checks of the LDS index arithmetic of the 128^3 pass-1 kernel
(k_plane_splat_fwd): the slot layout al(t) + be(k) restated from the kernel,
every address each lane forms in each barrier-free phase, and the premise
that makes those phases safe without workgroup barriers: a transform's lanes
lie in one wavefront, and no two transforms (hence no two wavefronts) touch
the same slot within a phase. No GPU needed."""

import numpy as np

N, T, L, S, SIZE, WAVES = 128, 64, 8, 136, 8778, 8


def al(t):
    return t * S + (t >> 2) * 4 + (t >> 3) * 2


def be(k):
    return k + (k >> 4)


def lanes():
    for wave in range(WAVES):
        for lane in range(64):
            yield wave, lane, lane // L, lane % L


def test_layout_is_a_bijection_into_the_lds_plane():
    slots = np.array([al(t) + be(k) for t in range(T) for k in range(N)])
    assert len(np.unique(slots)) == T * N and slots.min() == 0 and slots.max() < SIZE
    assert SIZE % 2 == 0 and SIZE * 8 <= 160 * 1024 // 2  # two workgroups per CU
    # the splat's float index of voxel (y, z): real part row y < N/2, imaginary part row y - N/2
    fl = {2 * (al(y & (T - 1)) + be(z)) + (1 if y >= T else 0) for y in range(N) for z in range(N)}
    assert len(fl) == N * N and max(fl) < 2 * SIZE


def test_lane_base_plus_immediate_decomposition():
    for l in range(L):
        for r in range(16):
            assert be(l + 8 * r) == l + be(8 * r)
            assert be(16 * l + r) == 17 * l + r
        for bb in range(2):
            for r in range(8):
                assert be(l + 8 * bb + 16 * r) == l + be(8 * bb + 16 * r)
        for r in range(8):
            assert al(l + 8 * r) == al(l) + al(8 * r)
            assert al(8 * l + r) == al(8 * l) + al(r)


def _z_slots(t, l):
    """Slots lane l of z transform t reads or writes (stage 0 in, stage 0
    out, stage 1 in/out)."""
    s = {al(t) + l + be(8 * r) for r in range(16)}
    s |= {al(t) + 17 * l + r for r in range(16)}
    s |= {al(t) + l + be(8 * bb + 16 * r) for bb in range(2) for r in range(8)}
    return s


def _y_slots(c, l):
    b1, b2 = be(c), be(T if c == 0 else N - c)
    s = {al(l) + al(8 * r) + b for r in range(8) for b in (b1, b2)}  # stage 0 in, stage 1 in/out
    s |= {al(8 * l) + al(r) + b for r in range(8) for b in (b1, b2)}  # stage 0 out
    if c == 0:  # the packed column's split reads its mirror positions
        for bb in range(2):
            for r in range(8):
                m = (N - (l + 8 * bb + 16 * r)) & (N - 1)
                s.add(al((m & 7) | ((m >> 4) << 3)) + (b2 if (m >> 3) & 1 else b1))
    return s


def test_barrier_free_phases_touch_disjoint_slots_per_transform():
    for phase, slots_of in (("z", _z_slots), ("y", _y_slots)):
        owner = {}
        for wave, lane, tau, l in lanes():
            tr = 8 * wave + tau  # z: row pair, y: column transform
            for sl in slots_of(tr, l):
                assert 0 <= sl < SIZE, (phase, tr, l, sl)
                prev = owner.setdefault(sl, (tr, wave))
                assert prev == (tr, wave), (phase, sl, prev, tr)  # one transform, one wavefront per slot
        assert len(owner) == T * N, phase  # and together they cover the plane


def test_y_transforms_read_exactly_the_z_outputs_they_own():
    z_out = {}
    for t in range(T):
        for l in range(L):
            for bb in range(2):
                for r in range(8):
                    z_out[al(t) + l + be(8 * bb + 16 * r)] = (t, l + 8 * bb + 16 * r)
    assert len(z_out) == T * N
    for c in range(T):
        k1, k2 = c, (T if c == 0 else N - c)
        got = {z_out[al(l) + al(8 * r) + be(k)] for l in range(L) for r in range(8) for k in (k1, k2)}
        assert got == {(t, k) for t in range(T) for k in (k1, k2)}


def test_column_zero_split_after_the_barrier_reads_what_the_transform_stored():
    """Spectra path: the column-0 transform stores C(q), q = l + 8 bb + 16 r,
    back in its slots; after the workgroup barrier thread k < N splits the
    packed column from C(k) and C(N - k), read at slot(q). Every such read is
    in bounds and finds the C(q) it wants, and each q has a slot of its own."""
    stored = {}
    for l in range(L):
        for bb in range(2):
            for r in range(8):
                q = l + 8 * bb + 16 * r
                stored[al(l) + al(8 * r) + (be(T) if bb else be(0))] = q
    assert len(stored) == N

    def slot(q):
        return al((q & 7) | ((q >> 4) << 3)) + (be(T) if (q >> 3) & 1 else be(0))

    for k in range(N):
        for q in (k, (N - k) & (N - 1)):
            assert 0 <= slot(q) < SIZE and stored[slot(q)] == q
