"""Independent numpy/pure-Python checker used to pin the oracle.

It follows different routes from the oracle on purpose: counts by
``np.bincount``, segments by a stable ``argsort``, dilation by its closed form
(nearest occupied voxel in L1 distance, lowest id on ties) instead of the ring
recursion, and distances with exact rational rounding.  Only for tiny inputs.
"""
import numpy as np

from exact_f32 import dist2_f32, transform_f32

MASK = np.uint32(0x80000000)


def voxel_ids_np(x, origin, inv, dims):
    """float32 (x - o) * inv per axis, floor, x fastest; -1 outside."""
    x = np.asarray(x, np.float32)
    f = (x - np.asarray(origin, np.float32)[:, None]) * np.float32(inv)
    inside = np.all((f >= 0) & (f < np.asarray(dims, np.float32)[:, None]), axis=0)
    i = np.floor(np.where(inside, f, 0)).astype(np.int64)
    v = i[0] + int(dims[0]) * (i[1] + int(dims[1]) * i[2])
    return np.where(inside, v, -1)


def segments_np(q, origin, inv, dims, V):
    vid = voxel_ids_np(q, origin, inv, dims)
    assert (vid >= 0).all()
    n = q.shape[1]
    hist = np.bincount(vid, minlength=V).astype(np.uint32)
    off = np.zeros(V + 1, np.int64)
    off[1:] = np.cumsum(hist.astype(np.int64) + 2)
    vm = np.zeros(n + 2 * V, np.uint32)
    order = np.argsort(vid, kind="stable")
    vm[off[:-1] + 1] = hist
    pos = np.zeros(V, np.int64)
    for i in order:
        v = vid[i]
        vm[off[v] + 2 + pos[v]] = i
        pos[v] += 1
    return hist, off.astype(np.uint32), vm


def closed_form_roots(hist, dims, L):
    """root[v] = lexicographic min of (|v - o|_1, o) over occupied o with |v - o|_1 <= L."""
    Dx, Dy, Dz = (int(d) for d in dims)
    V = Dx * Dy * Dz
    occ = np.nonzero(hist)[0]
    ox, oy, oz = occ % Dx, (occ // Dx) % Dy, occ // (Dx * Dy)
    roots = np.full(V, 0xFFFFFFFF, np.uint32)
    for v in range(V):
        x, y, z = v % Dx, (v // Dx) % Dy, v // (Dx * Dy)
        d = np.abs(ox - x) + np.abs(oy - y) + np.abs(oz - z)
        ok = d <= L
        if ok.any():
            dm = d[ok].min()
            roots[v] = occ[ok][d[ok] == dm].min()
    return roots


def nns_rule(q, p, Rt, origin, inv, dims, hist, off, vm, counts=False):
    """Alg. 4 with exact float32 rounding, pure Python.  With counts, also
    returns the candidates scanned by local searches and the number of
    queries whose voxel holds Mask(root)."""
    q = np.asarray(q, np.float32)
    n = q.shape[1]
    idx, d2, fb, nloc, ndil = [], [], 0, 0, 0
    for i in range(p.shape[1]):
        s = transform_f32(Rt, p[:, i])
        v = voxel_ids_np(np.array(s, np.float32).reshape(3, 1), origin, inv, dims)[0]
        cand = None
        if v >= 0:
            h = int(vm[off[v] + 1])
            ndil += 1 if (h & 0x80000000) else 0
            seg = (h & 0x7FFFFFFF) if (h & 0x80000000) else v
            c = int(hist[seg])
            if c > 0:
                cand = [int(j) for j in vm[off[seg] + 2: off[seg] + 2 + c]]
                nloc += c
        if cand is None:
            cand = range(n)
            fb += 1
        best = None
        for j in cand:
            d = dist2_f32(s, q[:, j])
            if best is None or (d, j) < best:
                best = (d, j)
        idx.append(best[1])
        d2.append(best[0])
    if counts:
        return np.array(idx, np.int32), np.array(d2, np.float32), fb, nloc, ndil
    return np.array(idx, np.int32), np.array(d2, np.float32), fb


def direct_layout_nns(q, p, Rt, origin, inv, dims, roots, capacity):
    """VANICP's layout written out literally: every voxel owns a block of
    ``capacity`` point records, filled in point order; a block that would
    take more points is marked overflowed; a dilated voxel's block is a copy
    of its root's (overflow included).  A query searches its voxel's block,
    or the whole target when the block is empty, overflowed or the point is
    outside the grid.  Returns (idx, d2, number of global searches)."""
    q = np.asarray(q, np.float32)
    n = q.shape[1]
    vid = voxel_ids_np(q, origin, inv, dims)
    blocks, over = {}, set()
    for i in range(n):
        v = int(vid[i])
        b = blocks.setdefault(v, [])
        if len(b) < capacity:
            b.append(i)
        else:
            over.add(v)
    for v in range(len(roots)):
        r = int(roots[v])
        if r != 0xFFFFFFFF and v not in blocks and r in blocks:
            blocks[v] = list(blocks[r])
            if r in over:
                over.add(v)
    idx, d2, fb = [], [], 0
    for i in range(p.shape[1]):
        s = transform_f32(Rt, p[:, i])
        v = int(voxel_ids_np(np.array(s, np.float32).reshape(3, 1), origin, inv, dims)[0])
        cand = blocks.get(v) if (v >= 0 and v not in over) else None
        if not cand:
            cand = range(n)
            fb += 1
        best = min((dist2_f32(s, q[:, j]), j) for j in cand)
        idx.append(best[1])
        d2.append(best[0])
    return np.array(idx, np.int32), np.array(d2, np.float32), fb


def kabsch_svd(p, q):
    """Textbook SVD solution of Eq. 1 (numpy), float64."""
    p = np.asarray(p, np.float64)
    q = np.asarray(q, np.float64)
    pb, qb = p.mean(1, keepdims=True), q.mean(1, keepdims=True)
    H = (p - pb) @ (q - qb).T
    U, S, Vt = np.linalg.svd(H)
    d = np.sign(np.linalg.det(Vt.T @ U.T))
    R = Vt.T @ np.diag([1.0, 1.0, d]) @ U.T
    t = qb[:, 0] - R @ pb[:, 0]
    return R, t, S
