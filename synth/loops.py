"""Closed hexagonal glide loops in a BCC-like crystal, drawn from a seed.

The paper's own loop ensembles (a 210-loop set in a (4000 b)^3 cube, Sec. 5.2,
and the 460k/160k-segment networks of Sec. 5.5) are not available, so these
seeded loop ensembles stand in for them: each loop is a planar hexagon on a
{110} plane with a unit 1/2<111>-type Burgers vector lying in that plane,
discretised into 40 straight segments (the paper discretises loops into
polygons of straight segments, Sec. 2).

Draw order per loop (numpy ``default_rng(seed)``), fixed so that every
consumer sees the same segments:
  1. centre ~ U[0,1]^3
  2. radius ~ U[r_min, r_max]
  3. plane index ~ integers(6) over (110),(1-10),(101),(10-1),(011),(01-1)
  4. Burgers direction: integers(2) over the two <111> directions normal to
     the plane normal, then the sign via integers(2)
  5. theta0 ~ U[0, 2 pi)
Hexagon vertices are c + r (cos(theta0 + k pi/3) e1 + sin(...) e2) with
e1 = b_hat and e2 = n x e1 (counter-clockwise about n); the six edges are split
into 7,7,7,7,6,6 equal sub-segments.
"""
from __future__ import annotations

import numpy as np

_PLANES = np.array(
    [[1, 1, 0], [1, -1, 0], [1, 0, 1], [1, 0, -1], [0, 1, 1], [0, 1, -1]],
    dtype=np.float64,
)
_DIRS111 = np.array(
    [[1, 1, 1], [1, 1, -1], [1, -1, 1], [-1, 1, 1]], dtype=np.float64
)
_SPLIT = (7, 7, 7, 7, 6, 6)
SEGS_PER_LOOP = sum(_SPLIT)

# Root cube shared by every generated ensemble: it holds every loop whose
# centre lies in the unit cube and whose radius is at most 0.05.
BOX_LO = (-0.05, -0.05, -0.05)
BOX_SIZE = 1.1


def make_loops(n_loops: int, r_min: float, r_max: float, seed: int):
    """Return (seg [N_s,2,3] f64, burgers [N_s,3] f64) for n_loops loops."""
    rng = np.random.default_rng(seed)
    segs = np.empty((n_loops * SEGS_PER_LOOP, 2, 3), dtype=np.float64)
    burg = np.empty((n_loops * SEGS_PER_LOOP, 3), dtype=np.float64)
    for il in range(n_loops):
        c = rng.uniform(0.0, 1.0, size=3)
        r = rng.uniform(r_min, r_max)
        ip = int(rng.integers(6))
        n = _PLANES[ip] / np.linalg.norm(_PLANES[ip])
        cands = [d for d in _DIRS111 if abs(np.dot(d, _PLANES[ip])) < 0.5]
        ib = int(rng.integers(2))
        sg = 1.0 if int(rng.integers(2)) == 0 else -1.0
        b = sg * cands[ib] / np.linalg.norm(cands[ib])
        th0 = rng.uniform(0.0, 2.0 * np.pi)
        e1 = b
        e2 = np.cross(n, e1)
        ang = th0 + np.arange(7) * (np.pi / 3.0)
        verts = c + r * (np.cos(ang)[:, None] * e1 + np.sin(ang)[:, None] * e2)
        k = il * SEGS_PER_LOOP
        for ie, ns in enumerate(_SPLIT):
            a0, a1 = verts[ie], verts[ie + 1]
            t = np.arange(ns + 1) / ns
            pts = a0 + t[:, None] * (a1 - a0)
            segs[k:k + ns, 0] = pts[:-1]
            segs[k:k + ns, 1] = pts[1:]
            burg[k:k + ns] = b
            k += ns
    return segs, burg


def make_clustered(n_clusters: int, per_cluster: int, cluster_r: float, r_small: tuple, n_spread: int,
                   r_spread: tuple, seed: int):
    """Loops of very uneven density: n_clusters tight clusters, each of
    per_cluster small loops (radii r_small) whose centres are moved to
    uniform points of a ball of radius cluster_r around the cluster centre
    (cluster centres uniform in [0.1, 0.9]^3), plus n_spread loops spread over
    the unit cube (radii r_spread).  Drawn from make_loops' streams (seed, and
    seed + 1 for the spread loops) and default_rng(seed + 2) for the moves."""
    segs, burg = make_loops(n_clusters * per_cluster, r_small[0], r_small[1], seed)
    rng = np.random.default_rng(seed + 2)
    centres = rng.uniform(0.1, 0.9, size=(n_clusters, 3))
    for il in range(n_clusters * per_cluster):
        s = segs[il * SEGS_PER_LOOP:(il + 1) * SEGS_PER_LOOP]
        d = rng.normal(size=3)
        d *= cluster_r * rng.uniform() ** (1.0 / 3.0) / np.linalg.norm(d)
        s += centres[il // per_cluster] + d - s.reshape(-1, 3).mean(axis=0)
    seg2, b2 = make_loops(n_spread, r_spread[0], r_spread[1], seed + 1)
    return np.concatenate([segs, seg2]), np.concatenate([burg, b2])


# Isotropic medium: shear modulus 1, Poisson ratio 0.3 -> cubic constants
# C11 = lambda + 2 mu, C12 = lambda, C44 = mu.
_MU, _NU = 1.0, 0.3
_LAM = 2.0 * _MU * _NU / (1.0 - 2.0 * _NU)
ISO = (_LAM + 2.0 * _MU, _LAM, _MU)
CUBIC_A25 = (1.0, 0.6, 0.5)

# Named workloads: loop ensemble, medium, FMM order p (nodes per dimension)
# and leaf depth D.  Sizes follow the configurations the method is exercised
# on: a small isotropic case the oracle finishes in seconds, a 200k-segment
# isotropic case, a 100k-segment cubic case (Zener ratio 2.5) and a
# 1M-segment cubic case, and a 10M-segment cubic case for one GPU's capacity.
WORKLOADS = {
    "iso2k": dict(n_loops=50, r=(0.01, 0.05), seed=1, C=ISO, order=4, depth=3),
    "iso200k": dict(n_loops=5000, r=(0.002, 0.02), seed=2, C=ISO, order=5, depth=6),
    "cubic100k": dict(n_loops=2500, r=(0.002, 0.02), seed=3, C=CUBIC_A25, order=5, depth=5),
    "cubic1m": dict(n_loops=25000, r=(0.002, 0.02), seed=5, C=CUBIC_A25, order=6, depth=7),
    # ten times the 1M case in the same cube
    "cubic10m": dict(n_loops=250000, r=(0.002, 0.02), seed=6, C=CUBIC_A25, order=6, depth=8),
    # 1M segments of very uneven density: 40 clusters of 500 small loops in
    # balls of radius 0.01, and 5,000 loops spread over the cube
    "cluster1m": dict(clusters=(40, 500, 0.01, (0.001, 0.003)), n_loops=5000, r=(0.002, 0.02), seed=7,
                      C=CUBIC_A25, order=6, depth=7),
}
CORE_A = 1e-3


def make_workload(name: str):
    """Return (seg, burgers, params dict) for a named workload."""
    w = WORKLOADS[name]
    if "clusters" in w:
        nc, per, cr, rs = w["clusters"]
        seg, b = make_clustered(nc, per, cr, rs, w["n_loops"], w["r"], w["seed"])
    else:
        seg, b = make_loops(w["n_loops"], w["r"][0], w["r"][1], w["seed"])
    prm = dict(
        c11=w["C"][0], c12=w["C"][1], c44=w["C"][2], core_a=CORE_A,
        order=w["order"], depth=w["depth"], box_lo=BOX_LO, box_size=BOX_SIZE,
    )
    return seg, b, prm


def segment_subset(n_seg: int, k: int, seed: int) -> np.ndarray:
    """Sorted seeded random subset of k distinct segment indices."""
    rng = np.random.default_rng(seed)
    k = min(k, n_seg)
    return np.sort(rng.choice(n_seg, size=k, replace=False)).astype(np.int64)


def batch_sizes(n_cfg: int = 64, seed: int = 4, lo: int = 5000, hi: int = 150000):
    """Segment counts of the batched ensemble: 40 * round(exp(U[ln lo, ln hi]) / 40)."""
    rng = np.random.default_rng(seed)
    return [int(40 * round(float(np.exp(rng.uniform(np.log(lo), np.log(hi)))) / 40)) for _ in range(n_cfg)]


def make_batch(n_cfg: int = 64, seed: int = 4):
    """n_cfg independent isotropic loop ensembles of log-uniform size in
    [5000, 150000] segments, radii [0.01, 0.05], ensemble i seeded 4000 + i."""
    return [make_loops(n // SEGS_PER_LOOP, 0.01, 0.05, 4000 + i) for i, n in enumerate(batch_sizes(n_cfg, seed))]
