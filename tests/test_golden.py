"""The stored oracle values (written by tests/golden/make_golden.py, which
calls only the oracle) still match the oracle: guards the oracle's arithmetic
against unreviewed change."""

import json
import os

import numpy as np

import oracle as O
import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def test_c1_golden_values_reproduce():
    rec = json.load(open(os.path.join(HERE, "golden", "c1_oracle.json")))
    a = synth.config_c1()
    d = O.pair_fields(a.A.xyzr, a.A.w, a.B.xyzr, a.B.w, a.rotations[0], a.cB, a.n, a.sigma)
    poses = np.array(rec["poses"], np.float32)
    assert np.allclose(O.lattice_read(d["E"], poses), rec["E"], rtol=1e-12, atol=1e-9)
    assert np.allclose(O.lattice_read(d["F"], poses).T, rec["F"], rtol=1e-12, atol=1e-9)
    assert np.allclose(O.lattice_read(d["tau"], poses).T, rec["tau"], rtol=1e-12, atol=1e-9)
    assert abs(d["E"].sum() - rec["E_sum"]) < 1e-9 * abs(rec["E_sum"])
    assert abs(d["uA"].sum() - rec["uA_sum"]) < 1e-12 * rec["uA_sum"]


def test_c4_golden_file_describes_the_workload():
    """The 512^3 reference values (tests/golden/make_c4_golden.py, oracle
    only; 20 minutes to recompute, so checked here for consistency only):
    poses drawn by the workload's generator, contact poses with energy,
    uniform ones mostly without, all values finite."""
    import importlib.util

    spec = importlib.util.spec_from_file_location("make_c4", os.path.join(HERE, "golden", "make_c4_golden.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    g = np.load(os.path.join(HERE, "golden", "c4_512_poses.npz"))
    a = synth.config_c4(n_poses=10000)
    idx = mk.pose_indices(len(a.poses))
    assert np.array_equal(g["indices"], idx) and np.array_equal(g["poses"], a.poses[idx])
    v = g["values"]
    assert v.shape == (16, 7) and np.all(np.isfinite(v))
    assert np.all(v[8:, 0] > 0)  # contact poses overlap
    assert int(g["n"]) == 512 and float(g["sigma"]) == a.sigma
