"""Writes tests/golden/c1_oracle.json from the FP64 oracle only.

Workload: the 32^3 two-part case (three polylines per part, identity
rotation). Stored: E, F, tau at the workload's pose and at four more lattice
translations, plus summary statistics of the E field. Run from the
repository root: python tests/golden/make_golden.py
"""

import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import synth  # noqa: E402


def main():
    a = synth.config_c1()
    d = O.pair_fields(a.A.xyzr, a.A.w, a.B.xyzr, a.B.w, a.rotations[0], a.cB, a.n, a.sigma)
    poses = np.concatenate([a.poses, np.array([[16, 16, 16], [15, 17, 16], [18, 14, 13], [0, 0, 0]], np.float32)])
    rec = {
        "workload": "32^3, 3 polylines per part, identity rotation (seeds 101/102/103)",
        "source": "oracle.pair_fields (float64)",
        "poses": poses.tolist(),
        "E": O.lattice_read(d["E"], poses).tolist(),
        "F": O.lattice_read(d["F"], poses).T.tolist(),
        "tau": O.lattice_read(d["tau"], poses).T.tolist(),
        "E_sum": float(d["E"].sum()),
        "E_max": float(d["E"].max()),
        "uA_sum": float(d["uA"].sum()),
        "uB_sum": float(d["uB"].sum()),
    }
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c1_oracle.json")
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    print("wrote", out)


if __name__ == "__main__":
    main()
