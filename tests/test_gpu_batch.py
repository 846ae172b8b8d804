"""GPU tests of ga_batch_*: items of different grid edges recorded into one
HIP graph and replayed. Every replay is compared with eager ga_energy_fields
calls on the same inputs, with eager work and synchronisation between the
replays; an in-place update of the rotations is picked up by the next replay;
every field of every item is checked against the FP64 oracle."""

import ctypes

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


def _item(G, n, seed, npts, nrot):
    A = synth.random_part(seed, n, npts, 1.0, 3.0, conf_radius=n / 4)
    B = synth.random_part(seed + 1, n, npts, 1.0, 3.0, conf_radius=n / 6)
    plan = G.Plan(n, max_batch=8)
    Ahat = G.ga_fft3d(plan, G.GA_R2C, G.ga_splat(plan, _dev(A.xyzr), _dev(A.w)))[0].contiguous()
    R = _dev(synth.shoemake_rotations(seed + 2, nrot).reshape(nrot, 9).astype(np.float32))
    return {"plan": plan, "Ahat": Ahat, "xyzr": _dev(B.xyzr), "w": _dev(B.w), "R": R, "c": B.ref_point(),
            "sigma": 0.5, "_A": A, "_B": B}


def _eager(G, it):
    return G.ga_energy_fields(it["plan"], it["Ahat"], it["xyzr"], it["w"], it["R"], it["c"], it["sigma"])


def test_graph_batch_of_mixed_grid_sizes(G):
    items = [_item(G, 32, 11, 120, 3), _item(G, 48, 21, 200, 2), _item(G, 64, 31, 300, 4), _item(G, 32, 41, 90, 1)]
    refs = [_eager(G, it) for it in items]
    b = G.Batch(items)
    try:
        side = _item(G, 48, 51, 100, 2)
        for rep in range(3):
            outs = b.launch()
            torch.cuda.synchronize()
            for E, ref in zip(outs, refs):
                assert O.rel_l2(E.double().cpu().numpy(), ref.double().cpu().numpy()) < 1e-6, rep
            # eager work of the program between replays
            _ = _eager(G, side)
            _ = (side["xyzr"] * 2).sum()
            torch.cuda.synchronize()
        # new rotations written in place are read by the next replay
        it = items[2]
        it["R"].copy_(_dev(synth.shoemake_rotations(99, 4).reshape(4, 9).astype(np.float32)))
        torch.cuda.synchronize()
        ref2 = _eager(G, it)
        outs = b.launch()
        torch.cuda.synchronize()
        assert O.rel_l2(outs[2].double().cpu().numpy(), ref2.double().cpu().numpy()) < 1e-6
        # every member of every item against the oracle
        for i, it in enumerate(items):
            Rh = it["R"].cpu().numpy().reshape(-1, 3, 3)
            for r in range(Rh.shape[0]):
                d = O.pair_fields(it["_A"].xyzr, it["_A"].w, it["_B"].xyzr, it["_B"].w, Rh[r], it["c"],
                                  it["plan"].n, want_torque=False)
                assert O.rel_l2(outs[i][r].double().cpu().numpy(), d["E"]) < FIELD_TOL, (i, r)
    finally:
        b.close()


def test_graph_batch_errors(G):
    it = _item(G, 32, 61, 60, 2)
    lib = G.lib()
    h = ctypes.c_void_p()
    arr = (G.ga.BatchItem * 1)()
    assert lib.ga_batch_create(ctypes.byref(h), arr, 0) != 0  # no items
    E = torch.empty((2, 32, 32, 32), dtype=torch.float32, device="cuda")
    work = it["plan"].workspace(G.ga.GA_OP_ENERGY, 2, it["xyzr"].shape[0])

    def item(E_ptr, work_ptr, work_bytes):
        return G.ga.BatchItem(it["plan"].handle.value, it["Ahat"].data_ptr(), it["xyzr"].data_ptr(),
                              it["w"].data_ptr(), it["xyzr"].shape[0], it["R"].data_ptr(),
                              (ctypes.c_float * 3)(*[float(v) for v in it["c"]]), 0.5, 2, E_ptr, work_ptr,
                              work_bytes)

    arr[0] = item(E.data_ptr(), work.data_ptr(), 16)  # workspace too small
    assert lib.ga_batch_create(ctypes.byref(h), arr, 1) != 0
    two = (G.ga.BatchItem * 2)()
    two[0] = item(E.data_ptr(), work.data_ptr(), work.numel())
    two[1] = item(E.data_ptr(), work.data_ptr(), work.numel())  # same output and workspace
    assert lib.ga_batch_create(ctypes.byref(h), two, 2) != 0
    assert lib.ga_batch_launch(None, None) != 0


def test_graph_batch_records_overlapped_items_as_parts(G):
    """Items whose plan asks for 2 or 4 parts are recorded as parallel branches
    of their batch slices: every replay equals the eager one-stream call."""
    items = [_item(G, 32, 71, 150, 7), _item(G, 64, 81, 300, 8)]
    items[0]["plan"].set_overlap(4)
    items[1]["plan"].set_overlap(2)
    refs = []
    for it in items:
        it["plan"].set_overlap(1)
        refs.append(_eager(G, it))
    items[0]["plan"].set_overlap(4)
    items[1]["plan"].set_overlap(2)
    b = G.Batch(items)
    try:
        for rep in range(3):
            outs = b.launch()
            torch.cuda.synchronize()
            for E, ref in zip(outs, refs):
                assert O.rel_l2(E.double().cpu().numpy(), ref.double().cpu().numpy()) < 1e-6, rep
            _ = _eager(G, items[1])  # overlapped eager call between replays
            torch.cuda.synchronize()
    finally:
        b.close()
