"""Seeded synthetic point clouds shaped like the paper's workloads.

The paper evaluates on ModelNet objects (about 10k points), the Stanford Bunny
(about 40k) and TUM RGB-D scenes (over 200k), all scaled into a unit sphere and
then perturbed (Sec. IV.A, "Dataset").  None of those datasets is available
here, so these generators produce stand-ins of the same scale and structure:

* ``sphere``   -- 2,048 points on the unit sphere, isotropic noise.
* ``bumpy``    -- the closed surface r(theta, phi) = 1 + 0.1 sin(5 theta) sin(4 phi),
                  area-uniform, 40k / 35k points (object scale).
* ``room``     -- a 4 x 3 x 2.5 m box room with 20 boxes on the floor, sampled
                  with density falling as 1/d^2 from a sensor at the centre,
                  226k / 200k points (scene scale, very uneven voxel occupancy).
* ``batched``  -- 64 pairs of log-uniform size in [5k, 120k], alternating the
                  bumpy and room generators.
* ``diff``     -- 16 bumpy pairs of 40k / 40k points plus small se(3) poses.

This module is input generation only: it draws random numbers and applies the
known rigid perturbation that makes a source cloud.  It contains none of the
registration method's arithmetic and is shared, unchanged, by the CPU oracle
tests and the GPU path.  Every array is float32 in structure-of-arrays layout,
shape (3, n), C-contiguous.  The order of random draws is part of each
generator's contract: the same seed gives the same bytes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from functools import lru_cache

import numpy as np

__all__ = [
    "Pair", "sphere_pair", "bumpy_pair", "room_pair", "batched_pairs",
    "diff_pairs", "config", "CONFIGS", "random_rotation", "tiny_cloud",
]


@dataclass
class Pair:
    """One registration problem: align ``p`` (source) to ``q`` (target)."""
    name: str
    q: np.ndarray              # (3, n) float32 target, SoA
    p: np.ndarray              # (3, m) float32 source, SoA
    voxel: float               # voxel edge length
    rings: int                 # dilation rings L
    iters: int                 # ICP iterations K
    R_true: np.ndarray         # (3, 3) float64: p was made as R_true @ x + t_true
    t_true: np.ndarray         # (3,) float64
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.q.shape[1])

    @property
    def m(self) -> int:
        return int(self.p.shape[1])

    @property
    def extent(self) -> float:
        """Largest side of the target's axis-aligned bounding box."""
        return float((self.q.max(axis=1) - self.q.min(axis=1)).max())


# ----------------------------------------------------------------------------
# small helpers (random draws only)
# ----------------------------------------------------------------------------

def _unit_vectors(rng: np.random.Generator, k: int) -> np.ndarray:
    u = rng.standard_normal((k, 3))
    return u / np.linalg.norm(u, axis=1, keepdims=True)


def random_rotation(axis: np.ndarray, angle: float) -> np.ndarray:
    """Rotation matrix about a unit ``axis`` by ``angle`` radians (Rodrigues)."""
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0.0, -a[2], a[1]], [a[2], 0.0, -a[0]], [-a[1], a[0], 0.0]])
    return np.eye(3) + math.sin(angle) * K + (1.0 - math.cos(angle)) * (K @ K)


def _perturb(rng, pts: np.ndarray, max_deg: float, t_norm_max: float,
             fixed_angle: bool = False, fixed_t: bool = False):
    """Apply a random rigid motion to (k, 3) float64 points.

    Rotation axis uniform on S^2; angle ``max_deg`` (fixed_angle) or
    U(0, max_deg) degrees; translation direction uniform on S^2 with norm
    ``t_norm_max`` (fixed_t) or U(0, t_norm_max).
    """
    axis = _unit_vectors(rng, 1)[0]
    ang = math.radians(max_deg if fixed_angle else rng.uniform(0.0, max_deg))
    tdir = _unit_vectors(rng, 1)[0]
    tn = t_norm_max if fixed_t else rng.uniform(0.0, t_norm_max)
    R = random_rotation(axis, ang)
    t = tdir * tn
    return pts @ R.T + t, R, t


def _soa(pts: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(pts.T.astype(np.float32))


# ----------------------------------------------------------------------------
# surfaces
# ----------------------------------------------------------------------------

def _sphere_points(rng, k: int, noise: float) -> np.ndarray:
    u = _unit_vectors(rng, k)
    return u + rng.normal(0.0, noise, size=(k, 3))


def _bumpy_xyz(th, ph):
    r = 1.0 + 0.1 * np.sin(5.0 * th) * np.sin(4.0 * ph)
    st = np.sin(th)
    return np.stack([r * st * np.cos(ph), r * st * np.sin(ph), r * np.cos(th)], axis=1)


def _bumpy_area_density(th, ph):
    """|dx/dtheta x dx/dphi| for the bumpy surface (analytic partials)."""
    s5, c5 = np.sin(5 * th), np.cos(5 * th)
    s4, c4 = np.sin(4 * ph), np.cos(4 * ph)
    r = 1.0 + 0.1 * s5 * s4
    r_t = 0.5 * c5 * s4
    r_p = 0.4 * s5 * c4
    st, ct = np.sin(th), np.cos(th)
    sp, cp = np.sin(ph), np.cos(ph)
    # x = r * (st cp, st sp, ct)
    xt = np.stack([r_t * st * cp + r * ct * cp, r_t * st * sp + r * ct * sp, r_t * ct - r * st], 1)
    xp = np.stack([r_p * st * cp - r * st * sp, r_p * st * sp + r * st * cp, r_p * ct], 1)
    return np.linalg.norm(np.cross(xt, xp), axis=1)


# Upper bound of the area density: |x_t||x_p| <= sqrt(1.1^2+0.5^2) sqrt(1.1^2+0.4^2).
_BUMPY_BOUND = math.sqrt(1.1 ** 2 + 0.5 ** 2) * math.sqrt(1.1 ** 2 + 0.4 ** 2)


def _bumpy_points(rng, k: int, noise: float) -> np.ndarray:
    if k == 0:
        return np.zeros((0, 3))
    out = []
    have = 0
    while have < k:
        b = max(4096, int(1.6 * (k - have)) + 64)
        th = rng.uniform(0.0, math.pi, b)
        ph = rng.uniform(0.0, 2.0 * math.pi, b)
        acc = rng.uniform(0.0, 1.0, b) * _BUMPY_BOUND < _bumpy_area_density(th, ph)
        x = _bumpy_xyz(th[acc], ph[acc])
        out.append(x)
        have += x.shape[0]
    pts = np.concatenate(out, 0)[:k]
    return pts + rng.normal(0.0, noise, size=(k, 3))


ROOM_LO = np.array([-2.0, -1.5, -1.25])
ROOM_HI = np.array([2.0, 1.5, 1.25])


def _room_faces(rng, nboxes: int = 20):
    """Axis-aligned rectangles as (axis, coord, lo2, hi2) over the other two axes."""
    faces = []

    def box_faces(lo, hi, bottom: bool):
        for ax in range(3):
            o = [a for a in range(3) if a != ax]
            for side, c in ((0, lo[ax]), (1, hi[ax])):
                if ax == 2 and side == 0 and not bottom:
                    continue
                faces.append((ax, c, np.array([lo[o[0]], lo[o[1]]]), np.array([hi[o[0]], hi[o[1]]])))

    box_faces(ROOM_LO, ROOM_HI, bottom=True)
    for _ in range(nboxes):
        side = rng.uniform(0.2, 1.0, 3)
        cx = rng.uniform(ROOM_LO[0] + side[0] / 2, ROOM_HI[0] - side[0] / 2)
        cy = rng.uniform(ROOM_LO[1] + side[1] / 2, ROOM_HI[1] - side[1] / 2)
        lo = np.array([cx - side[0] / 2, cy - side[1] / 2, ROOM_LO[2]])
        hi = np.array([cx + side[0] / 2, cy + side[1] / 2, ROOM_LO[2] + side[2]])
        box_faces(lo, hi, bottom=False)
    return faces


def _face_min_dist(face) -> float:
    ax, c, lo2, hi2 = face
    clamp = np.clip(np.zeros(2), lo2, hi2)
    return math.sqrt(c * c + float(clamp @ clamp))


def _room_points(rng, faces, k: int, noise: float) -> np.ndarray:
    areas = np.array([float(np.prod(f[3] - f[2])) for f in faces])
    cum = np.cumsum(areas) / areas.sum()
    d0 = min(_face_min_dist(f) for f in faces)
    ax = np.array([f[0] for f in faces])
    c = np.array([f[1] for f in faces])
    lo2 = np.stack([f[2] for f in faces])
    hi2 = np.stack([f[3] for f in faces])
    o0 = np.where(ax == 0, 1, 0)
    o1 = np.where(ax == 2, 1, 2)
    if k == 0:
        return np.zeros((0, 3))
    out = []
    have = 0
    while have < k:
        b = 1 << 20
        fi = np.minimum(np.searchsorted(cum, rng.uniform(0.0, 1.0, b), side="right"), len(faces) - 1)
        uv = rng.uniform(0.0, 1.0, (b, 2))
        pts = np.empty((b, 3))
        rows = np.arange(b)
        pts[rows, ax[fi]] = c[fi]
        pts[rows, o0[fi]] = lo2[fi, 0] + uv[:, 0] * (hi2[fi, 0] - lo2[fi, 0])
        pts[rows, o1[fi]] = lo2[fi, 1] + uv[:, 1] * (hi2[fi, 1] - lo2[fi, 1])
        d2 = np.einsum("ij,ij->i", pts, pts)
        acc = rng.uniform(0.0, 1.0, b) * d2 < d0 * d0
        x = pts[acc]
        out.append(x)
        have += x.shape[0]
    pts = np.concatenate(out, 0)[:k]
    if noise > 0:
        pts = pts + rng.normal(0.0, noise, size=(k, 3))
    return pts


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------

def sphere_pair(seed: int = 0, n: int = 2048, m: int = 2048) -> Pair:
    """Unit-sphere pair: 5 deg about a random axis, translation of norm 0.02."""
    rng = np.random.default_rng(seed)
    q = _sphere_points(rng, n, 0.002)
    x = _sphere_points(rng, m, 0.002)
    p, R, t = _perturb(rng, x, 5.0, 0.02, fixed_angle=True, fixed_t=True)
    return Pair("sphere_2k", _soa(q), _soa(p), 0.05, 2, 20, R, t)


def bumpy_pair(seed: int = 1, n: int = 40000, m: int = 35000, voxel: float = 0.03,
               rings: int = 2, iters: int = 50, max_deg: float = 10.0, name: str = "bumpy_40k") -> Pair:
    """Bumpy closed surface; rotation <= max_deg, translation <= 2% of extent."""
    rng = np.random.default_rng(seed)
    q = _bumpy_points(rng, n, 0.003)
    x = _bumpy_points(rng, m, 0.003)
    ext = float((q.max(0) - q.min(0)).max())
    p, R, t = _perturb(rng, x, max_deg, 0.02 * ext)
    return Pair(name, _soa(q), _soa(p), voxel, rings, iters, R, t, {"extent": ext})


def room_pair(seed: int = 2, n: int = 226000, m: int = 200000, voxel: float = 0.05,
              rings: int = 3, iters: int = 30, max_deg: float = 5.0, t_max: float = 0.1,
              name: str = "room_226k") -> Pair:
    """Indoor scene with 1/d^2 density; rotation <= 5 deg, translation <= 0.1 m."""
    rng = np.random.default_rng(seed)
    faces = _room_faces(rng)
    q = _room_points(rng, faces, n, 0.0)
    x = _room_points(rng, faces, m, 0.005)
    p, R, t = _perturb(rng, x, max_deg, t_max)
    return Pair(name, _soa(q), _soa(p), voxel, rings, iters, R, t)


def batched_pairs(seed: int = 3, npairs: int = 64, lo: float = 5e3, hi: float = 1.2e5,
                  rings: int = 3, iters: int = 30) -> list:
    """Pairs of log-uniform size; even index bumpy, odd index room."""
    rng = np.random.default_rng(seed)
    sizes = [int(round(math.exp(rng.uniform(math.log(lo), math.log(hi))))) for _ in range(npairs)]
    seeds = rng.integers(0, 2 ** 31 - 1, size=npairs)
    pairs = []
    for k, (n, s) in enumerate(zip(sizes, seeds)):
        r2 = np.random.default_rng(int(s))
        if k % 2 == 0:
            q = _bumpy_points(r2, n, 0.003)
            x = _bumpy_points(r2, n, 0.003)
        else:
            faces = _room_faces(r2)
            q = _room_points(r2, faces, n, 0.0)
            x = _room_points(r2, faces, n, 0.005)
        ext = float((q.max(0) - q.min(0)).max())
        p, R, t = _perturb(r2, x, 10.0, 0.02 * ext)
        pairs.append(Pair(f"batch{k}", _soa(q), _soa(p), ext / 60.0, rings, iters, R, t,
                          {"extent": ext, "surface": "bumpy" if k % 2 == 0 else "room"}))
    return pairs


def diff_pairs(seed: int = 4, npairs: int = 16, n: int = 40000):
    """Bumpy pairs for the differentiable loss, plus a small random pose per pair.

    Returns (pairs, xi) where xi is (npairs, 6) float64 = (rho, phi) with
    |phi| <= 0.1 rad and |rho| <= 0.02.
    """
    rng = np.random.default_rng(seed)
    seeds = rng.integers(0, 2 ** 31 - 1, size=npairs)
    pairs = [bumpy_pair(int(s), n, n, 0.03, 2, 1, name=f"diff{k}") for k, s in enumerate(seeds)]
    phi = _unit_vectors(rng, npairs) * rng.uniform(0.0, 0.1, (npairs, 1))
    rho = _unit_vectors(rng, npairs) * rng.uniform(0.0, 0.02, (npairs, 1))
    xi = np.concatenate([rho, phi], axis=1)
    return pairs, xi


def tiny_cloud(seed: int, n: int, scale: float = 1.0, dup: int = 0) -> np.ndarray:
    """(3, n) float32 uniform cloud in [-scale, scale]^3 with ``dup`` duplicated points."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(-scale, scale, (n, 3))
    if dup:
        idx = rng.integers(0, n, dup)
        x[rng.integers(0, n, dup)] = x[idx]
    return _soa(x)


CONFIGS = ("sphere_2k", "bumpy_40k", "room_226k", "batched_64", "diff_16x40k")


def normalize_unit_sphere(P: Pair, name: str, N: int = 4, rings: int = 10, iters: int = 50) -> Pair:
    """The paper's setting (Sec. IV.A): both clouds moved and scaled by the
    same map so that the target fits inside the unit sphere (centre of the
    target's bounding box, radius its farthest point, enlarged by 1e-6 so
    that no target lands on the sphere itself), and a fixed grid of 2^N
    voxels per axis over [-1, 1)^3 with L dilation rings.  The source keeps
    its misalignment (the map is applied to both)."""
    q64 = P.q.astype(np.float64)
    c = 0.5 * (q64.min(1) + q64.max(1))
    r = float(np.sqrt(((q64 - c[:, None]) ** 2).sum(0)).max()) * (1.0 + 1e-6)
    q = ((q64 - c[:, None]) / r).astype(np.float32)
    p = ((P.p.astype(np.float64) - c[:, None]) / r).astype(np.float32)
    side = 1 << N
    meta = dict(P.meta)
    meta.update({"grid_origin": (-1.0, -1.0, -1.0), "grid_dims": (side, side, side), "N": N,
                 "rmse_eps": 1e-5, "early_stop": True, "scale": r, "centre": c.tolist()})
    return Pair(name, q, p, 2.0 / side, rings, iters, P.R_true, (P.t_true - c + P.R_true @ c) / r, meta)


@lru_cache(maxsize=8)
def config(name: str):
    """The named workload (cached per process)."""
    if name == "paper_bunny_40k":
        return normalize_unit_sphere(bumpy_pair(), name)
    if name == "paper_room_226k":
        return normalize_unit_sphere(room_pair(), name)
    if name == "sphere_2k":
        return sphere_pair()
    if name == "bumpy_40k":
        return bumpy_pair()
    if name == "room_226k":
        return room_pair()
    if name == "batched_64":
        return batched_pairs()
    if name == "diff_16x40k":
        return diff_pairs()
    raise KeyError(name)
