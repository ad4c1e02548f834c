"""GPU properties of a grid at the size limits of the offset-addressed layout
(Alg. 1-4): V just under 2^31 voxels and n + 2V just under 2^32 segment
words, the largest grid whose offsets fit 32 bits.

No V-sized array leaves the device (each is several GB).  The checks use
sparse closed forms built from the occupied voxels alone: the occupied and
dilated voxel counts (dilation reaches exactly the empty voxels within L1
distance L of an occupied one), the largest count, and searches whose
expected correspondences follow from Alg. 4 with the dilation's closed form
(root = nearest occupied voxel in L1 distance, lowest id on ties), with
distances in exact float32 rounding.
"""
import numpy as np
import pytest

from bruteforce import voxel_ids_np
from exact_f32 import dist2_f32

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():   # collected on CPU machines, skipped there
    pytest.skip("no GPU", allow_module_level=True)

from paper_2512_04996_amd.api import build_grid_fixed  # noqa: E402

DIMS = (1290, 1290, 1290)   # V = 2,146,689,000 = 2^31 - 794,648
L = 2
IDENT = np.array([1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0], np.float32)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def l1_offsets(r):
    return [(dx, dy, dz) for dx in range(-r, r + 1) for dy in range(-r, r + 1) for dz in range(-r, r + 1)
            if abs(dx) + abs(dy) + abs(dz) <= r]


def clustered_cloud(rng, voxel):
    # 2,000 clusters of 25 points within about a voxel of their centres
    # (segments of several points), eight of them at the corners and a few
    # at the faces; then ten exact duplicates (the lowest index wins a tie)
    c = rng.uniform(-0.99, 0.99, (3, 2000))
    c[:, :8] = np.array([[sx, sy, sz] for sx in (-0.999, 0.999) for sy in (-0.999, 0.999)
                         for sz in (-0.999, 0.999)]).T
    c[0, 8:20] = 0.9995
    q = np.repeat(c, 25, axis=1) + rng.normal(0.0, 0.8 * float(voxel), (3, 2000 * 25))
    q = np.clip(q, -0.9995, 0.9995).astype(np.float32)
    q = np.concatenate([q, q[:, 100:110]], axis=1)
    return q


def test_grid_at_the_offset_limits():
    if torch.cuda.get_device_properties(0).total_memory < (160 << 30):
        pytest.skip("needs about 90 GB of device memory")
    Dx, Dy, Dz = DIMS
    V = Dx * Dy * Dz
    voxel = np.float32(2.0 / Dx)
    origin = np.array([-1.0, -1.0, -1.0], np.float32)
    inv = np.float32(1.0) / voxel
    rng = np.random.default_rng(2024)
    q = clustered_cloud(rng, voxel)
    n = q.shape[1]
    assert V < 2 ** 31 and n + 2 * V < 2 ** 32 and n + 2 * V > 2 ** 32 - 2 * 10 ** 6

    vid = voxel_ids_np(q, origin, inv, DIMS)
    assert (vid >= 0).all()
    members = {}
    for j, v in enumerate(vid.tolist()):
        members.setdefault(v, []).append(j)
    occ = np.array(sorted(members), np.int64)
    occ_set = set(occ.tolist())

    def coords(v):
        return v % Dx, (v // Dx) % Dy, v // (Dx * Dy)

    def vid_of(x, y, z):
        return x + Dx * (y + Dy * z)

    # dilated voxels: empty voxels within L1 distance L of an occupied one
    reach = set()
    for v in occ.tolist():
        x, y, z = coords(v)
        for dx, dy, dz in l1_offsets(L):
            a, b, c = x + dx, y + dy, z + dz
            if 0 <= a < Dx and 0 <= b < Dy and 0 <= c < Dz:
                reach.add(vid_of(a, b, c))
    dilated = len(reach - occ_set)

    g = build_grid_fixed(dev(q), origin, float(voxel), DIMS, L)
    try:
        g.dilate(L)
        d = g.describe()
        assert d["V"] == V and d["n"] == n
        assert d["occupied"] == len(occ) and d["dilated"] == dilated
        assert d["max_count"] == max(len(m) for m in members.values())
        assert d["static_bytes"] == 8 * V and d["dynamic_bytes"] == 4 * (n + 2 * V)

        # every target point finds itself (or its lowest-indexed exact twin)
        # in its own segment
        idx, d2, fb = g.nns(dev(q), IDENT)
        idx = idx.cpu().numpy()
        first = {}
        expect = np.array([first.setdefault(q[:, j].tobytes(), j) for j in range(n)])
        assert (expect[n - 10:] == np.arange(100, 110)).all()
        assert int(fb.cpu()[0]) == 0
        assert np.array_equal(idx, expect) and (d2.cpu().numpy() == 0).all()

        # queries one voxel over and a voxel and a half over: own segment
        # when occupied, else the root's segment (closed form), else none
        # of these (the global search, left out here: it is size-free)
        sel = rng.choice(n, 1500, replace=False)
        shifts = [np.array([voxel, 0, 0], np.float32), np.array([0, -voxel, 1.5 * voxel], np.float32)]
        p = np.concatenate([q[:, sel] + s[:, None] for s in shifts], axis=1).astype(np.float32)
        pv = voxel_ids_np(p, origin, inv, DIMS)
        keep, cand_lists = [], []
        for i, u in enumerate(pv.tolist()):
            if u < 0:
                continue
            seg = u if u in occ_set else None
            if seg is None:
                x, y, z = coords(u)
                best = None
                for dx, dy, dz in l1_offsets(L):
                    a, b, c = x + dx, y + dy, z + dz
                    if 0 <= a < Dx and 0 <= b < Dy and 0 <= c < Dz:
                        o = vid_of(a, b, c)
                        if o in occ_set and (best is None or (abs(dx) + abs(dy) + abs(dz), o) < best):
                            best = (abs(dx) + abs(dy) + abs(dz), o)
                seg = None if best is None else best[1]
            if seg is not None:
                keep.append(i)
                cand_lists.append(members[seg])
        assert len(keep) > 2500
        p = np.ascontiguousarray(p[:, keep])
        idx, d2, fb = g.nns(dev(p), IDENT)
        idx = idx.cpu().numpy()
        d2 = d2.cpu().numpy()
        assert int(fb.cpu()[0]) == 0
        for i, cand in enumerate(cand_lists):
            best = min((dist2_f32(p[:, i], q[:, j]), j) for j in cand)
            assert (idx[i], d2[i]) == (best[1], best[0]), i
    finally:
        g.free()
