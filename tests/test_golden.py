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
