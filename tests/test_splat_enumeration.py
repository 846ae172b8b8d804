"""Host emulation of the per-wavefront splat's row enumeration (wave_splat in
csrc/ga_kernels.hpp), lane by lane: the DPP prefix sum, the compaction of a
batch of hits into the wave's slots, the per-step start flags, ballot and
masked bit count that give each lane its hit. Checks that every (hit, row) of
the bounding squares is visited exactly once, and that every slot, flag and
hit index stays inside its array, for random hit sets including empty waves,
full waves and batches beyond the slot capacity.
"""

import numpy as np
import pytest


def dpp_incl_scan(v):
    """Inclusive prefix sum over 64 lanes as the kernel forms it: row shifts by
    1, 2, 4, 8 within rows of 16 lanes (lanes shifted in from outside the row
    read 0), then the totals of lanes 15, 31, 47 added to the rows above."""
    v = list(v)
    for d in (1, 2, 4, 8):
        v = [v[i] + (v[i - d] if i % 16 >= d else 0) for i in range(64)]
    t0, t1, t2 = v[15], v[31], v[47]
    return [v[i] + (t0 if i >= 16 else 0) + (t1 if i >= 32 else 0) + (t2 if i >= 48 else 0) for i in range(64)]


def lanes_below(mask, lane):
    return bin(mask & ((1 << lane) - 1)).count("1")


def enumerate_rows(sy, cap):
    """sy[lane] > 0 for a lane holding a hit (its square's row count), else 0.
    Returns the visited (lane, row) pairs in order."""
    hit = [s > 0 for s in sy]
    hm = sum(1 << i for i in range(64) if hit[i])
    nh = bin(hm).count("1")
    rank = [lanes_below(hm, i) for i in range(64)]
    seen = []
    for r0 in range(0, nh, cap):
        mine = [hit[i] and r0 <= rank[i] < r0 + cap for i in range(64)]
        cnt = [sy[i] if mine[i] else 0 for i in range(64)]
        incl = dpp_incl_scan(cnt)
        assert incl == list(np.cumsum(cnt))
        total = incl[63]
        start = [incl[i] - cnt[i] for i in range(64)]
        slots = [None] * cap
        for i in range(64):
            if mine[i]:
                s = rank[i] - r0
                assert 0 <= s < cap and slots[s] is None
                slots[s] = (i, start[i])
        before = 0
        for base in range(0, total, 64):
            flag = [0] * 64
            for i in range(64):
                if mine[i] and base <= start[i] < base + 64:
                    assert flag[start[i] - base] == 0
                    flag[start[i] - base] = 1
            fm = sum(1 << i for i in range(64) if flag[i])
            for lane in range(64):
                j = before + lanes_below(fm, lane) + flag[lane] - 1
                if base + lane < total:
                    assert 0 <= j < cap and slots[j] is not None
                    owner, st = slots[j]
                    row = base + lane - st
                    assert 0 <= row < sy[owner]
                    seen.append((owner, row))
            before += bin(fm).count("1")
    return seen


@pytest.mark.parametrize("cap", [16, 32])
def test_every_row_once_and_indices_in_bounds(cap):
    rng = np.random.default_rng(20261203 + cap)
    cases = [[0] * 64, [1] * 64, [9] * 64]
    for _ in range(300):
        k = int(rng.choice([0, 1, 2, 5, 10, 31, 32, 33, 40, 64]))
        sy = [0] * 64
        for lane in rng.choice(64, size=k, replace=False):
            sy[int(lane)] = int(rng.integers(1, 9 if rng.random() < 0.9 else 129))
        cases.append(sy)
    for sy in cases:
        seen = enumerate_rows(sy, cap)
        want = sorted((i, r) for i in range(64) for r in range(sy[i]))
        assert sorted(seen) == want
        assert len(set(seen)) == len(seen)

