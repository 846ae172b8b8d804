"""Writes tests/golden/c4_512_poses.npz: energy, force and torque of the 512^3
workload (two parts of 50,000 samples on 40 polylines, radii log-uniform in
[0.5, 8], identity rotation) at 16 lattice poses drawn by the workload's own
seeded generator (the first 8 uniform and the first 8 contact poses), by the
oracle's physical-space single-pose sums: E = sum_q u_A(q + t) u_B(q),
F = -sum_q grad u_A(q + t) u_B(q), tau = sum_q (grad u_A(q + t) x yhat(q)) u_B(q),
with grad the spectral gradient of eq. 6a computed by the oracle's own FFT
in float64. Calls only the oracle and the input generator; about 10 minutes
and 16 GB of host memory.

    python tests/golden/make_c4_golden.py
"""

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c4_512_poses.npz")


def pose_indices(n_poses):
    half = n_poses // 2
    return np.concatenate([np.arange(8), half + np.arange(8)])


def main():
    a = synth.config_c4()
    n = a.n
    idx = pose_indices(len(a.poses))
    poses = a.poses[idx].astype(np.float64)
    t0 = time.time()
    uA = O.splat(a.A.xyzr[:, :3].astype(np.float64), a.A.xyzr[:, 3], a.A.w, n, a.sigma)
    uB = O.splat(O.place(a.B.xyzr[:, :3], np.eye(3), a.cB), a.B.xyzr[:, 3], a.B.w, n, a.sigma)
    print(f"splats {time.time() - t0:.0f} s", flush=True)
    g = O.grad_spectral(uA)
    print(f"gradient {time.time() - t0:.0f} s", flush=True)
    vals = np.array([O.local_pose_sum(uA, uB, t, grad=g) for t in poses])
    print(f"sums {time.time() - t0:.0f} s", flush=True)
    np.savez(OUT, poses=poses.astype(np.float32), indices=idx, values=vals, n=n, sigma=a.sigma)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
