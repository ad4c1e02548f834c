"""GPU parity of the global search (Alg. 4's search over all n targets when a
query's voxel is empty and undilated, or the query is outside the grid).  The
search kernel resolves such queries itself by visiting voxel cubes around
them until a bound rules out every target outside the visited cube, and
lists the rest for the exhaustive search; either way the result must be the
exact lexicographic minimum of (d, j) over all n targets, which the oracle
computes by brute force.  Queries at every distance from the cloud (inside
the grid and far outside it, some beyond the largest cube), on voxel faces,
and equidistant from duplicated targets (ties broken by the lower index)."""
import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2512_04996_amd.api import build_grid  # noqa: E402

IDENT = np.array([1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0], np.float32)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def sphere(rng, n, noise):
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    return (u + noise * rng.normal(size=(n, 3))).astype(np.float32)


def check(q, p, voxel, rings, Rt=IDENT):
    g = build_grid(dev(q), voxel, rings).dilate(rings)
    og = oracle.dilate(oracle.build_grid(q, voxel, rings), rings)
    idx, d2, fb = g.nns(dev(p), Rt)
    ridx, rd2, rF, _ = oracle.nns(og, q, p, Rt)
    idx, d2 = idx.cpu().numpy(), d2.cpu().numpy()
    bad = np.nonzero((idx != ridx) | (d2.view(np.uint32) != rd2.view(np.uint32)))[0]
    assert bad.size == 0, (bad[:10], idx[bad[:10]], ridx[bad[:10]], d2[bad[:10]], rd2[bad[:10]])
    assert int(fb.cpu().numpy()[0]) == int(rF)
    return int(rF)


@pytest.mark.parametrize("rings", [0, 1, 3])
def test_queries_at_every_distance(rings):
    # a unit sphere of 20k points, voxel 0.05; queries displaced from target
    # points by up to 12 voxels (inside the padded grid and beyond it)
    rng = np.random.default_rng(11 + rings)
    q = sphere(rng, 20000, 0.002).T.copy()
    base = q[:, rng.integers(0, q.shape[1], 30000)]
    step = rng.normal(size=(3, 30000))
    step /= np.linalg.norm(step, axis=0)
    p = (base + step * rng.uniform(0.0, 0.6, 30000)).astype(np.float32)
    F = check(q, p, 0.05, rings)
    assert F > 3000   # most of these take the global search


def test_far_outside_and_beyond_the_largest_cube():
    # queries 1 to 50 units from a room-sized box of points: outside the grid,
    # many beyond the largest cube the shells visit (exhaustive search)
    rng = np.random.default_rng(5)
    q = rng.uniform(-2.0, 2.0, (3, 30000)).astype(np.float32)
    d = rng.normal(size=(3, 4000))
    d /= np.linalg.norm(d, axis=0)
    p = (d * rng.uniform(3.0, 50.0, 4000)).astype(np.float32)
    assert check(q, p, 0.1, 1) == 4000


def test_ties_between_duplicated_targets():
    # every target point appears twice (two indices, same coordinates), and
    # queries sit exactly between pairs of targets on a lattice, in empty
    # voxels: equal distances, the lower index must win
    rng = np.random.default_rng(7)
    lat = (np.stack(np.meshgrid(np.arange(12), np.arange(12), np.arange(12), indexing="ij"), 0).reshape(3, -1)
           * 0.5).astype(np.float32)
    q = np.concatenate([lat, lat[:, ::-1]], 1)
    q = q[:, rng.permutation(q.shape[1])].copy()
    # midpoints between lattice neighbours along x, and cell centres (8
    # equidistant targets, 16 with the duplicates)
    mid = (lat + np.array([[0.25], [0.0], [0.0]], np.float32)).astype(np.float32)
    ctr = (lat + np.float32(0.25)).astype(np.float32)
    p = np.concatenate([mid, ctr], 1)
    assert check(q, p, 0.1, 0) > 0


def test_queries_on_voxel_faces():
    rng = np.random.default_rng(3)
    q = sphere(rng, 8000, 0.0).T.copy()
    g = build_grid(dev(q), 0.04, 1)
    o = g.describe()["origin"]
    # queries whose coordinates are whole numbers of voxels from the origin
    k = rng.integers(0, 40, (3, 3000)).astype(np.float32)
    p = (o[:, None] + k * np.float32(0.04)).astype(np.float32)
    g.free()
    check(q, p, 0.04, 1)


def test_global_searches_under_a_pose():
    # a rotated and shifted source: the misses come from the pose
    rng = np.random.default_rng(9)
    q = sphere(rng, 30000, 0.003).T.copy()
    p = sphere(rng, 20000, 0.003).T.copy()
    a = 0.2
    Rt = np.array([np.cos(a), -np.sin(a), 0, np.sin(a), np.cos(a), 0, 0, 0, 1, 0.05, -0.03, 0.02], np.float32)
    assert check(q, p, 0.03, 2, Rt) > 500


def test_coarse_grid_with_crowded_voxels():
    # two dense clusters in a coarse grid (thousands of points per voxel):
    # a query in an empty voxel has too many points around it for the shells,
    # so the exhaustive search resolves it, with the same result
    rng = np.random.default_rng(13)
    a = rng.normal(size=(3, 20000)) * 0.05 + np.array([[0.0], [0.0], [0.0]])
    b = rng.normal(size=(3, 20000)) * 0.05 + np.array([[1.5], [1.5], [1.5]])
    q = np.concatenate([a, b], 1).astype(np.float32)
    p = rng.uniform(-0.2, 1.7, (3, 3000)).astype(np.float32)
    assert check(q, p, 0.3, 0) > 500
