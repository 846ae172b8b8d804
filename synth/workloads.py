"""Seeded generators for the synthetic parts, rotations and poses.

The paper's own part pair (a CAD model with three zero-clearance peg/hole
pairs, Fig. 4) is not available, so every workload here is synthetic: a part
is a set of medial-axis (skeleton) samples, each a ball centre, a ball radius
in voxels and a signed weight. The shapes and sizes follow the five benchmark
workloads:

* C1 -- 32^3 grid, two parts of three random polylines (~200 points, spacing
  0.5 voxel, one radius ~U[1,3] per polyline), identity rotation, one pose.
* C2 -- 128^3 grid, a hole (8 rods of radius 2 on a ring, clearance 0.5) and a
  peg (one axis polyline of 400 points, radius 4), 1000 poses.
* C3 -- 128^3 grid, two parts of ~2k points (radii ~U[1,4]) and 64 rotations
  drawn uniformly on SO(3).
* C4 -- 512^3 grid, two parts of 40 polylines x 1250 points, radii
  log-uniform in [0.5, 8], 10k poses.
* C5 -- 16 assemblies with grids from {64, 96, 128, 192}, 500-5k points each,
  Poisson pose queries at an aggregate 16 kHz.

All arrays handed to either implementation are float32; the oracle promotes
those exact values to float64. Nothing in this module evaluates a density, a
transform or a correlation.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np

# Thickness factor used by the paper for its experiments (Sec. 4, sigma = 0.5).
SIGMA = 0.5
# Penalty factor lambda2/lambda1 used by the paper (Sec. 4.1): an interior
# skeleton sample carries +1, an exterior one -PENALTY (complex affinities).
PENALTY = 3.0


@dataclass
class Part:
    """Skeleton samples of one part, in voxel units of its own grid frame."""

    xyzr: np.ndarray  # float32 [n, 4]: ball centre (x, y, z) and ball radius r
    w: np.ndarray  # float32 [n]: signed weight (+1 interior skeleton, -PENALTY exterior)
    exterior: np.ndarray = None  # bool [n]: sample lies on the exterior skeleton (None: all interior)

    @property
    def n(self) -> int:
        return int(self.xyzr.shape[0])

    def ref_point(self) -> np.ndarray:
        """Unweighted mean of the sample centres, rounded to float32.

        Used as the moving part's reference point c_B (rotation centre)."""
        return self.xyzr[:, :3].astype(np.float64).mean(axis=0).astype(np.float32)


@dataclass
class Assembly:
    """A stationary part A, a moving part B and the queries on the pair."""

    name: str
    n: int  # grid edge
    A: Part
    B: Part
    cB: np.ndarray  # float32 [3], reference point of B
    rotations: np.ndarray  # float32 [n_rot, 3, 3], row-major, proper orthogonal
    poses: np.ndarray  # float32 [n_poses, 3], translation of c_B in A's grid frame
    sigma: float = SIGMA
    extra: dict = field(default_factory=dict)


def _unit_vectors(rng: np.random.Generator, k: int) -> np.ndarray:
    v = rng.normal(size=(k, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _reflect_into_ball(v: np.ndarray, centre: np.ndarray, radius: float) -> np.ndarray:
    d = v - centre
    r = float(np.linalg.norm(d))
    if r <= radius:
        return v
    r2 = max(2.0 * radius - r, 0.0)
    return centre + d * (r2 / r)


def _polyline_points(rng, n_points, spacing, centre, conf_radius, n_seg=4):
    """Random walk of n_seg straight segments, vertices reflected into a ball,
    resampled at uniform arc length (nominal spacing `spacing`)."""
    centre = np.asarray(centre, dtype=np.float64)
    seg_len = (n_points - 1) * spacing / n_seg
    start = centre + _unit_vectors(rng, 1)[0] * conf_radius * 0.5 * rng.random()
    verts = [start]
    dirs = _unit_vectors(rng, n_seg)
    for s in range(n_seg):
        nxt = _reflect_into_ball(verts[-1] + seg_len * dirs[s], centre, conf_radius)
        verts.append(nxt)
    verts = np.asarray(verts)
    seg = np.linalg.norm(np.diff(verts, axis=0), axis=1)
    cum = np.concatenate([[0.0], np.cumsum(seg)])
    total = cum[-1]
    if total <= 0.0:
        return np.repeat(verts[:1], n_points, axis=0)
    s = np.linspace(0.0, total, n_points)
    out = np.empty((n_points, 3))
    for a in range(3):
        out[:, a] = np.interp(s, cum, verts[:, a])
    return out


def polyline_part(rng, n_poly, pts_per_poly, spacing, centre, conf_radius, radius_sampler,
                  weight=1.0) -> Part:
    """A part made of `n_poly` random polylines, one ball radius per polyline."""
    xyz, rad = [], []
    counts = pts_per_poly if isinstance(pts_per_poly, (list, tuple)) else [pts_per_poly] * n_poly
    for c in counts:
        pts = _polyline_points(rng, c, spacing, centre, conf_radius)
        r = float(radius_sampler(rng))
        xyz.append(pts)
        rad.append(np.full(c, r))
    xyz = np.concatenate(xyz)
    rad = np.concatenate(rad)
    xyzr = np.concatenate([xyz, rad[:, None]], axis=1).astype(np.float32)
    w = np.full(xyzr.shape[0], weight, dtype=np.float32)
    return Part(xyzr, w)


def random_part(seed: int, n: int, n_points: int, r_lo=1.0, r_hi=3.0, conf_radius=None,
                n_poly=None, spacing=0.5) -> Part:
    """Generic polyline part centred in an n^3 grid (used for small test cases)."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    if conf_radius is None:
        conf_radius = n / 4.0
    if n_poly is None:
        n_poly = max(1, int(np.ceil(n_points / 250)))
    base = n_points // n_poly
    counts = [base + (1 if i < n_points - base * n_poly else 0) for i in range(n_poly)]
    return polyline_part(rng, n_poly, counts, spacing, np.full(3, n / 2.0), conf_radius,
                         lambda g: g.uniform(r_lo, r_hi))


def shoemake_rotations(seed: int, k: int) -> np.ndarray:
    """k rotations uniform on SO(3) (Shoemake, Graphics Gems III, 1992)."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    u = rng.random((k, 3))
    a = np.sqrt(1.0 - u[:, 0])
    b = np.sqrt(u[:, 0])
    x = a * np.sin(2 * np.pi * u[:, 1])
    y = a * np.cos(2 * np.pi * u[:, 1])
    z = b * np.sin(2 * np.pi * u[:, 2])
    w = b * np.cos(2 * np.pi * u[:, 2])
    R = np.empty((k, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R.astype(np.float32)


def lattice_poses(rng, n, k_uniform, k_contact, centre, half_extent) -> np.ndarray:
    """Integer translations: k_uniform anywhere on the n^3 torus, k_contact in
    the box centre +- half_extent where the supports overlap."""
    uni = rng.integers(0, n, size=(k_uniform, 3))
    he = np.asarray(half_extent, dtype=np.int64)
    con = np.asarray(centre, dtype=np.int64) + rng.integers(-he, he + 1, size=(k_contact, 3))
    return np.concatenate([uni, con]).astype(np.float32)


def _identity(k=1):
    return np.repeat(np.eye(3, dtype=np.float32)[None], k, axis=0)


def config_c1() -> Assembly:
    """32^3, 3 polylines per part (~200 points), r ~ U[1,3], one lattice pose
    drawn where the supports overlap."""
    n = 32
    centre = np.full(3, n / 2.0)
    A = polyline_part(np.random.default_rng(np.random.PCG64(101)), 3, [67, 67, 66], 0.5, centre,
                      n / 2.0 - 4.0, lambda g: g.uniform(1.0, 3.0))
    B = polyline_part(np.random.default_rng(np.random.PCG64(102)), 3, [67, 67, 66], 0.5, centre,
                      n / 2.0 - 4.0, lambda g: g.uniform(1.0, 3.0))
    rng = np.random.default_rng(np.random.PCG64(103))
    poses = (n // 2 + rng.integers(-4, 5, size=(1, 3))).astype(np.float32)  # near contact
    return Assembly("C1", n, A, B, B.ref_point(), _identity(), poses)


def config_c2(n_poses: int = 1000, exterior: bool = False) -> Assembly:
    """128^3 peg-in-hole: hole = 8 rods (r = 2) on a ring of radius 6.5 around
    the z axis (clearance 0.5 to the peg), peg = one axis polyline of 400
    points (r = 4). The hole is stationary, the peg moves. With exterior=True
    the hole's axis is added to A as an exterior skeleton polyline (400
    points, r = 4.5, the free radius inside the ring of rods) with weight
    -PENALTY: the guidance "valley" that the inserted peg fills."""
    n = 128
    c = n / 2.0
    length = 48.0
    z = np.linspace(c - length / 2, c + length / 2, 400)
    rods = []
    for k in range(8):
        ang = 2 * np.pi * k / 8
        xyz = np.stack([np.full(400, c + 6.5 * np.cos(ang)), np.full(400, c + 6.5 * np.sin(ang)), z], 1)
        rods.append(np.concatenate([xyz, np.full((400, 1), 2.0)], 1))
    A = Part(np.concatenate(rods).astype(np.float32), np.ones(3200, np.float32))
    if exterior:
        axis = np.stack([np.full(400, c), np.full(400, c), z, np.full(400, 6.5 - 2.0)], 1)
        A = Part(np.concatenate([A.xyzr, axis]).astype(np.float32),
                 np.concatenate([A.w, np.full(400, -PENALTY)]).astype(np.float32),
                 np.concatenate([np.zeros(3200, bool), np.ones(400, bool)]))
    peg = np.stack([np.full(400, c), np.full(400, c), z, np.full(400, 4.0)], 1)
    B = Part(peg.astype(np.float32), np.ones(400, np.float32))
    rng = np.random.default_rng(np.random.PCG64(203))
    half = n_poses // 2
    poses = lattice_poses(rng, n, half, n_poses - half, (int(c),) * 3, (10, 10, 40))
    return Assembly("C2", n, A, B, B.ref_point(), _identity(), poses)


def config_c3(n_rot: int = 64) -> Assembly:
    """128^3, ~2k points per part (8 polylines x 250, r ~ U[1,4]), 64 rotations."""
    n = 128
    centre = np.full(3, n / 2.0)
    A = polyline_part(np.random.default_rng(np.random.PCG64(301)), 8, 250, 0.5, centre, n / 4.0,
                      lambda g: g.uniform(1.0, 4.0))
    B = polyline_part(np.random.default_rng(np.random.PCG64(302)), 8, 250, 0.5, centre, n / 4.0,
                      lambda g: g.uniform(1.0, 4.0))
    R = shoemake_rotations(303, n_rot)
    rng = np.random.default_rng(np.random.PCG64(304))
    poses = lattice_poses(rng, n, 8, 8, (n // 2,) * 3, (12, 12, 12))
    return Assembly("C3", n, A, B, B.ref_point(), R, poses)


def config_c4(n_poses: int = 10000) -> Assembly:
    """512^3, 40 polylines x 1250 points per part, r log-uniform in [0.5, 8]."""
    n = 512
    centre = np.full(3, n / 2.0)
    logu = lambda g: float(np.exp(g.uniform(np.log(0.5), np.log(8.0))))  # noqa: E731
    A = polyline_part(np.random.default_rng(np.random.PCG64(401)), 40, 1250, 0.5, centre, n / 4.0, logu)
    B = polyline_part(np.random.default_rng(np.random.PCG64(402)), 40, 1250, 0.5, centre, n / 4.0, logu)
    rng = np.random.default_rng(np.random.PCG64(403))
    half = n_poses // 2
    poses = lattice_poses(rng, n, half, n_poses - half, (n // 2,) * 3, (48, 48, 48))
    return Assembly("C4", n, A, B, B.ref_point(), _identity(), poses)


@dataclass
class ServingWorkload:
    assemblies: List[Assembly]
    arrival_s: np.ndarray  # float64 [q], arrival times in seconds
    pair: np.ndarray  # int32 [q], assembly index per query
    rotations: np.ndarray  # float32 [q, 3, 3]
    poses: np.ndarray  # float32 [q, 3], integer-valued translations


def config_c5(n_queries: int = 100000, rate_hz: float = 16000.0, sizes=(64, 96, 128, 192),
              n_assemblies: int = 16) -> ServingWorkload:
    """16 assemblies, grid edges uniform in `sizes`, 500-5k points per part,
    r ~ U[1,4]; Poisson queries at `rate_hz`, each a new rotation and a
    lattice translation near contact."""
    asm = []
    for i in range(n_assemblies):
        rng = np.random.default_rng(np.random.PCG64(500 + i))
        n = int(rng.choice(sizes))
        npts = int(rng.integers(500, 5001))
        n_poly = max(1, int(np.ceil(npts / 250)))
        base = npts // n_poly
        counts = [base + (1 if k < npts - base * n_poly else 0) for k in range(n_poly)]
        centre = np.full(3, n / 2.0)
        A = polyline_part(rng, n_poly, counts, 0.5, centre, n / 4.0, lambda g: g.uniform(1.0, 4.0))
        B = polyline_part(rng, n_poly, counts, 0.5, centre, n / 4.0, lambda g: g.uniform(1.0, 4.0))
        asm.append(Assembly(f"C5-{i}", n, A, B, B.ref_point(), _identity(), np.zeros((0, 3), np.float32)))
    rng = np.random.default_rng(np.random.PCG64(599))
    gaps = rng.exponential(1.0 / rate_hz, size=n_queries)
    arrival = np.cumsum(gaps)
    pair = rng.integers(0, n_assemblies, size=n_queries).astype(np.int32)
    R = shoemake_rotations(int(rng.integers(0, 2**31)), n_queries)
    ns = np.array([asm[p].n for p in pair])
    off = rng.integers(-8, 9, size=(n_queries, 3))
    poses = (ns[:, None] // 2 + off).astype(np.float32)
    return ServingWorkload(asm, arrival, pair, R, poses)
