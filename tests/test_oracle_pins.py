"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Nothing here uses the GPU.  Each test checks the oracle against something
other than itself: hand-derived values, the independent numpy checker
(``bruteforce.py``: bincount, stable argsort, the closed form of dilation,
exact rational rounding), textbook library routines (numpy SVD, scipy expm),
closed-form recovery of a known rigid motion, finite differences, and the
numbers printed in Table 1.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from bruteforce import closed_form_roots, direct_layout_nns, kabsch_svd, nns_rule, segments_np, voxel_ids_np
from exact_f32 import dist2_f32, transform_f32
from paper_2512_04996_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
IDENT = np.array([1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0], np.float32)


def soa(pts):
    return np.ascontiguousarray(np.asarray(pts, np.float32).T)


# ---------------------------------------------------------------- grid spec

def test_grid_spec_hand_example():
    # two points, voxel 0.5 (exact in binary), one ring of padding:
    # origin = 0 - 1*0.5 = -0.5; f(hi) = (1 - (-0.5)) * 2 = 3 -> D = 3 + 1 + 1 = 5
    q = soa([[0, 0, 0], [1, 1, 1]])
    origin, inv, dims, V = oracle.grid_spec(q, 0.5, 1)
    assert origin.tolist() == [-0.5, -0.5, -0.5]
    assert inv == 2.0
    assert dims.tolist() == [5, 5, 5] and V == 125
    # point (0,0,0) -> f = 1 -> voxel (1,1,1) = 1 + 5*(1 + 5*1) = 31; (1,1,1) -> (3,3,3) = 93
    assert oracle.voxel_ids(q, origin, inv, dims).tolist() == [31, 93]


def test_grid_spec_anisotropic_and_no_padding():
    q = soa([[0, 0, 0], [2.0, 0.25, 0.75]])
    origin, inv, dims, V = oracle.grid_spec(q, 0.25, 0)
    # f = (hi - lo) * 4 = 8, 1, 3 -> D = 9, 2, 4
    assert dims.tolist() == [9, 2, 4] and V == 72
    assert origin.tolist() == [0, 0, 0]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_every_target_inside_its_box(seed):
    q = synth.tiny_cloud(seed, 500, scale=1.7)
    for voxel, L in ((0.1, 2), (0.37, 0), (0.05, 3)):
        origin, inv, dims, V = oracle.grid_spec(q, voxel, L)
        vid = oracle.voxel_ids(q, origin, inv, dims)
        assert (vid >= 0).all() and (vid < V).all()
        # geometric check: each point lies in its voxel's box (to float rounding)
        i = np.stack([vid % dims[0], (vid // dims[0]) % dims[1], vid // (dims[0] * dims[1])])
        lo = origin.astype(np.float64)[:, None] + i * float(voxel)
        assert (q >= lo - 1e-5).all() and (q <= lo + float(voxel) + 1e-5).all()
        # at least L-1 empty layers beyond the occupied range on every side, L on the high side
        assert (i.max(1) + L + 1 == dims).all()
        assert (i.min(1) >= max(L - 1, 0)).all()


def test_grid_spec_errors():
    q = soa([[0, 0, 0], [1, 1, 1]])
    with pytest.raises(oracle.OracleError) as e:
        oracle.grid_spec(q, 0.0, 1)
    assert e.value.code == oracle.ERR_ARG
    with pytest.raises(oracle.OracleError) as e:
        oracle.grid_spec(q, 1e-6, 1)       # 1e6 voxels per axis -> V >= 2^31
    assert e.value.code == oracle.ERR_TOO_LARGE
    bad = q.copy()
    bad[1, 0] = np.nan
    with pytest.raises(oracle.OracleError) as e:
        oracle.grid_spec(bad, 0.5, 1)
    assert e.value.code == oracle.ERR_NONFINITE


# ------------------------------------------------ counts, offsets, segments

@pytest.mark.parametrize("seed,n,voxel,L", [(0, 300, 0.3, 1), (1, 1000, 0.2, 2), (2, 50, 2.5, 0), (3, 700, 0.11, 3)])
def test_build_matches_counting_sort(seed, n, voxel, L):
    q = synth.tiny_cloud(seed, n, dup=n // 10)
    g = oracle.build_grid(q, voxel, L)
    hist, off, vm = segments_np(q, g.origin, g.inv, g.dims, g.V)
    assert np.array_equal(g.hist, hist)
    assert np.array_equal(g.off, off)
    assert np.array_equal(g.vm, vm)
    # invariants
    assert int(g.hist.sum()) == n
    assert np.array_equal(np.diff(g.off.astype(np.int64)), g.hist.astype(np.int64) + 2)
    assert int(g.off[-1]) == n + 2 * g.V
    assert (g.vm[g.off[:-1]] == 0).all()
    pts = np.concatenate([g.vm[g.off[v] + 2: g.off[v] + 2 + g.hist[v]] for v in range(g.V)])
    assert np.array_equal(np.sort(pts), np.arange(n))


def test_voxel_ids_match_numpy_and_out_of_grid():
    q = synth.tiny_cloud(5, 400)
    origin, inv, dims, V = oracle.grid_spec(q, 0.13, 2)
    p = synth.tiny_cloud(6, 400, scale=1.6)     # some outside the grid
    a = oracle.voxel_ids(p, origin, inv, dims)
    b = voxel_ids_np(p, origin, inv, dims)
    assert np.array_equal(a, b)
    assert (a < 0).any() and (a >= 0).any()


# --------------------------------------------------------------- dilation

@pytest.mark.parametrize("seed,n,voxel,L", [(0, 40, 0.25, 1), (1, 25, 0.2, 2), (2, 60, 0.3, 3), (3, 8, 0.15, 4)])
def test_dilation_matches_closed_form(seed, n, voxel, L):
    q = synth.tiny_cloud(seed, n)
    g = oracle.dilate(oracle.build_grid(q, voxel, L), L)
    want = closed_form_roots(g.hist, g.dims, L)
    assert np.array_equal(g.roots, want)
    hdr = g.vm[g.off[:-1] + 1]
    occ = g.hist > 0
    assert np.array_equal(hdr[occ], g.hist[occ])                 # occupied headers unchanged
    dil = (~occ) & (want != 0xFFFFFFFF)
    assert np.array_equal(hdr[dil], want[dil] | np.uint32(0x80000000))
    assert (hdr[(~occ) & (want == 0xFFFFFFFF)] == 0).all()       # out of reach stays empty


def test_dilation_zero_rings_is_identity():
    q = synth.tiny_cloud(7, 100)
    g = oracle.build_grid(q, 0.2, 2)
    before = g.vm.copy()
    oracle.dilate(g, 0)
    assert np.array_equal(before, g.vm)


def test_dilation_saturates_and_tie_break():
    # one voxel per axis-aligned location; a single point fills the whole grid
    q = soa([[0.05, 0.05, 0.05]])
    g = oracle.dilate(oracle.build_grid(q, 0.1, 3), 9)           # diameter of a 7^3 grid is 18; 9 rings from the centre
    assert (g.roots == g.roots[0]).all() and g.hist[g.roots[0]] == 1
    # two occupied voxels equidistant from an empty one: lower id wins
    q = soa([[0.05, 0.05, 0.05], [0.25, 0.05, 0.05]])             # voxels x=0 and x=2 (plus padding)
    g = oracle.dilate(oracle.build_grid(q, 0.1, 1), 1)
    occ = np.nonzero(g.hist)[0]
    mid = (occ[0] + occ[1]) // 2
    assert g.hist[mid] == 0 and g.roots[mid] == occ[0]


def test_dilation_ring_semantics_are_synchronous():
    # voxel 0.125 (exact); two points on one row, 3 rings of padding:
    # origin = 0.1875 - 0.375 = -0.1875, so the points sit in x = 3 and x = 9
    q = soa([[0.1875, 0.0625, 0.0625], [0.9375, 0.0625, 0.0625]])
    g = oracle.build_grid(q, 0.125, 3)
    row = lambda v: v % g.dims[0]
    occ = np.nonzero(g.hist)[0]
    assert [row(v) for v in occ] == [3, 9]
    oracle.dilate(g, 2)
    base = occ[0] - 3
    got = [g.roots[base + x] for x in range(13)]
    N = 0xFFFFFFFF
    a, b = occ
    # ring r reaches exactly distance r: x = 6 is 3 away from both and stays empty
    assert got == [N, a, a, a, a, a, N, b, b, b, b, b, N]


# ---------------------------------------------------------------------- NNS

def _exact_nn(q, s):
    best = None
    for j in range(q.shape[1]):
        d = dist2_f32(s, q[:, j])
        if best is None or (d, j) < best:
            best = (d, j)
    return best


def test_nns_single_voxel_grid_is_exact_nn():
    q = synth.tiny_cloud(11, 120, dup=10)
    p = synth.tiny_cloud(12, 60, scale=0.5)                     # stays inside the one voxel
    g = oracle.build_grid(q, 10.0, 0)                            # one voxel holds everything
    assert g.V == 1
    Rt = np.array([0.99, -0.05, 0.1, 0.05, 0.99, 0.0, -0.1, 0.0, 0.99, 0.01, -0.02, 0.03], np.float32)
    idx, d2, F, _ = oracle.nns(g, q, p, Rt)
    assert F == 0
    for i in range(p.shape[1]):
        s = transform_f32(Rt, p[:, i])
        d, j = _exact_nn(q, s)
        assert idx[i] == j and d2[i] == d


def test_nns_all_outside_falls_back_to_exact_nn():
    q = synth.tiny_cloud(13, 150)
    p = synth.tiny_cloud(14, 40) + np.float32(5.0)              # far outside the grid
    g = oracle.dilate(oracle.build_grid(q, 0.2, 2), 2)
    idx, d2, F, C = oracle.nns(g, q, p, IDENT)
    assert F == p.shape[1] and C == F * q.shape[1]
    for i in range(p.shape[1]):
        d, j = _exact_nn(q, p[:, i])
        assert idx[i] == j and d2[i] == d


@pytest.mark.parametrize("seed,L", [(20, 0), (21, 1), (22, 2)])
def test_nns_matches_independent_rule(seed, L):
    q = synth.tiny_cloud(seed, 200, dup=20)
    p = synth.tiny_cloud(seed + 100, 80, scale=1.15)
    g = oracle.dilate(oracle.build_grid(q, 0.3, L), L)
    Rt = np.array([0.98, -0.17, 0.0, 0.17, 0.98, 0.0, 0.0, 0.0, 1.0, 0.02, 0.0, -0.01], np.float32)
    idx, d2, F, _ = oracle.nns(g, q, p, Rt)
    ridx, rd2, rF, rC, rD = nns_rule(q, p, Rt, g.origin, g.inv, g.dims, g.hist, g.off, g.vm, counts=True)
    assert np.array_equal(idx, ridx) and np.array_equal(d2, rd2) and F == rF
    # the counts the GPU path reports per iteration
    assert oracle.nns_counts(g, q, p, Rt) == (rF, rC, rD)
    if L > 0:
        assert rD > 0


@pytest.mark.parametrize("seed,L,cap", [(23, 0, 1), (24, 1, 2), (25, 2, 3), (26, 2, 5), (27, 1, 10 ** 6)])
def test_capacity_nns_matches_literal_direct_layout(seed, L, cap):
    """VANICP's fixed blocks (Sec. II.B) with the global search for points
    beyond a block (Sec. IV.B): the oracle's capacity rule on the segmented
    grid against the block layout built literally, with roots from the
    closed form of the dilation."""
    q = synth.tiny_cloud(seed, 220, dup=25)
    p = synth.tiny_cloud(seed + 100, 90, scale=1.15)
    g = oracle.dilate(oracle.build_grid(q, 0.3, L), L)
    Rt = np.array([0.98, -0.17, 0.0, 0.17, 0.98, 0.0, 0.0, 0.0, 1.0, 0.02, 0.0, -0.01], np.float32)
    roots = closed_form_roots(g.hist, g.dims, L)
    idx, d2, F, _ = oracle.nns(g, q, p, Rt, capacity=cap)
    ridx, rd2, rF = direct_layout_nns(q, p, Rt, g.origin, g.inv, g.dims, roots, cap)
    assert np.array_equal(idx, ridx) and np.array_equal(d2, rd2) and F == rF
    base = oracle.nns(g, q, p, Rt)
    if cap >= int(g.hist.max()):
        assert np.array_equal(idx, base[0]) and F == base[2]
    else:
        assert F > base[2]          # some block overflowed and sent its queries to the global search


def test_register_direct_capacity():
    q = synth.tiny_cloud(28, 300, dup=40)
    p = synth.tiny_cloud(29, 120, scale=1.1)
    a = oracle.register(q, p, 0.3, 2, 6)
    b = oracle.register_direct(q, p, 0.3, 2, 6)                 # 64 KiB blocks: nothing overflows
    assert np.array_equal(a.Rt, b.Rt) and np.array_equal(a.fallbacks, b.fallbacks)
    c = oracle.register_direct(q, p, 0.3, 2, 6, block_bytes=2 * oracle.RECORD_BYTES)
    g = oracle.dilate(oracle.build_grid(q, 0.3, 2), 2)
    roots = closed_form_roots(g.hist, g.dims, 2)
    _, _, rF = direct_layout_nns(q, p, oracle.identity_rt().astype(np.float32), g.origin, g.inv, g.dims, roots, 2)
    assert c.fallbacks[0] == rF and rF > a.fallbacks[0]


def test_nns_never_beats_exact_and_ties_go_low():
    q = synth.tiny_cloud(30, 300)
    q = np.concatenate([q, q[:, :50]], axis=1)                  # exact duplicates at j + 300
    p = synth.tiny_cloud(31, 100)
    g = oracle.dilate(oracle.build_grid(q, 0.25, 1), 1)
    idx, d2, F, _ = oracle.nns(g, q, p, IDENT)
    for i in range(p.shape[1]):
        d, j = _exact_nn(q, p[:, i])
        assert d2[i] >= d
        if d2[i] == d:
            assert idx[i] <= j or dist2_f32(p[:, i], q[:, idx[i]]) == d
    assert (idx < 300).all()                                     # a duplicate never beats its original


def test_nns_midpoint_tie():
    q = soa([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
    p = soa([[0.5, 0.0, 0.0]])
    g = oracle.build_grid(q, 4.0, 0)
    idx, d2, _, _ = oracle.nns(g, q, p, IDENT)
    assert idx[0] == 0 and d2[0] == 0.25


def test_transform_op_order():
    p = synth.tiny_cloud(40, 30)
    q = synth.tiny_cloud(41, 30)
    g = oracle.build_grid(q, 10.0, 0)
    Rt = np.array([0.3, -0.9, 0.31, 0.95, 0.29, -0.1, 0.07, 0.33, 0.94, 0.123, -0.456, 0.789], np.float32)
    idx, d2, _, _ = oracle.nns(g, q, p, Rt)
    for i in range(30):
        s = transform_f32(Rt, p[:, i])
        assert d2[i] == dist2_f32(s, q[:, idx[i]])


# ---------------------------------------------------------------- solve

def _rot(axis, ang):
    return synth.random_rotation(np.asarray(axis, float), ang)


@pytest.mark.parametrize("axis,ang", [([1, 2, 3], 0.3), ([0, 0, 1], math.pi), ([1, -1, 0.5], 2.9), ([0.2, 0.1, -1], 1e-4)])
def test_solve_recovers_known_motion(axis, ang):
    rng = np.random.default_rng(5)
    p64 = rng.uniform(-1, 1, (3, 500))
    p = p64.astype(np.float32)
    R = _rot(axis, ang)
    t = np.array([0.3, -0.2, 0.7])
    q = (R @ p.astype(np.float64) + t[:, None]).astype(np.float32)
    # float32 targets: the exact solve of the rounded data is within ~1e-7 of (R, t)
    Rt, sv, deg = oracle.solve(p, q, np.arange(500, dtype=np.int32))
    assert not deg
    assert np.abs(Rt[:9].reshape(3, 3) - R).max() < 1e-6
    assert np.abs(Rt[9:] - t).max() < 1e-6
    # and agrees with the textbook SVD solution on the same float32 data
    Rk, tk, S = kabsch_svd(p, q)
    assert np.abs(Rt[:9].reshape(3, 3) - Rk).max() < 1e-10
    assert np.abs(Rt[9:] - tk).max() < 1e-10
    assert np.allclose(np.sort(sv)[::-1], S, rtol=1e-9)


def test_solve_exact_data_to_1e12():
    # coordinates and motion exactly representable: a 90 degree turn about z
    p = soa([[0, 0, 0], [1, 0, 0], [0, 2, 0], [0, 0, 3], [1, 1, 1]])
    q = soa([[1, 2, 3], [1, 3, 3], [-1, 2, 3], [1, 2, 6], [0, 3, 4]])   # (x,y,z) -> (-y, x, z) + (1,2,3)
    Rt, _, deg = oracle.solve(p, q, np.arange(5, dtype=np.int32))
    R = np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1]], float)
    assert not deg
    assert np.abs(Rt[:9].reshape(3, 3) - R).max() < 1e-12
    assert np.abs(Rt[9:] - [1, 2, 3]).max() < 1e-12


def test_solve_reflection_case_gives_rotation():
    # targets are a mirror image: the best proper rotation must have det +1
    rng = np.random.default_rng(8)
    p = rng.uniform(-1, 1, (3, 200)).astype(np.float32)
    q = p.copy()
    q[0] *= -1
    Rt, _, deg = oracle.solve(p, q, np.arange(200, dtype=np.int32))
    R = Rt[:9].reshape(3, 3)
    assert abs(np.linalg.det(R) - 1) < 1e-12 and np.abs(R @ R.T - np.eye(3)).max() < 1e-12
    Rk, tk, _ = kabsch_svd(p, q)
    assert np.abs(R - Rk).max() < 1e-9


def test_solve_planar_and_degenerate():
    rng = np.random.default_rng(9)
    p = rng.uniform(-1, 1, (3, 100)).astype(np.float32)
    p[2] = 0                                                     # planar: rank 2, still unique
    R = _rot([0.3, 0.2, 1], 0.4)
    q = (R @ p.astype(np.float64)).astype(np.float32)
    Rt, sv, deg = oracle.solve(p, q, np.arange(100, dtype=np.int32))
    assert not deg and np.abs(Rt[:9].reshape(3, 3) - R).max() < 1e-6
    line = np.zeros((3, 50), np.float32)
    line[0] = np.linspace(-1, 1, 50)                             # collinear: rank 1
    prev = np.arange(12, dtype=np.float64)
    Rt, sv, deg = oracle.solve(line, line, np.arange(50, dtype=np.int32), prev)
    assert deg and np.array_equal(Rt, prev)


def test_solve_identity_at_alignment():
    q = synth.tiny_cloud(50, 300)
    Rt, _, deg = oracle.solve(q, q, np.arange(300, dtype=np.int32))
    assert np.abs(Rt - oracle.identity_rt()).max() < 1e-12


# ------------------------------------------------------------------ ICP

def test_icp_fixed_point_at_alignment():
    q = synth.tiny_cloud(60, 400)
    r = oracle.register(q, q, 0.2, 2, 3)
    assert (r.nn_idx == np.arange(400)).all() and (r.nn_d2 == 0).all()
    assert np.abs(r.Rt - oracle.identity_rt()).max() < 1e-12
    assert (r.rmse == 0).all() and (r.fallbacks == 0).all()


def test_icp_recovers_rigid_copy():
    # the source is the target itself under a small known motion.  With one
    # voxel holding every target point the local search is the exact nearest
    # neighbour, so ICP must return the exact inverse (to the float32
    # rounding of the source) and the identity correspondence.
    P = synth.bumpy_pair(seed=70, n=3000, m=3000, voxel=0.08, rings=2)
    q = P.q
    R = _rot([1, 2, 2], math.radians(3))
    t = np.array([0.01, -0.015, 0.02])
    p = (R @ q.astype(np.float64) + t[:, None]).astype(np.float32)
    r = oracle.register(q, p, 10.0, 0, 15)
    assert np.abs(r.Rt[:9].reshape(3, 3) - R.T).max() < 1e-8
    assert np.abs(r.Rt[9:] + R.T @ t).max() < 1e-8
    assert (r.nn_idx == np.arange(3000)).all()
    assert r.rmse[-1] < 1e-6 and r.rmse[0] > 1e-2


def test_icp_stop_rule():
    P = synth.sphere_pair()
    full = oracle.register(P.q, P.p, P.voxel, P.rings, 20)
    assert full.iters == 20
    early = oracle.register(P.q, P.p, P.voxel, P.rings, 20, rmse_eps=1e-3, early_stop=True)
    k = early.iters
    d = np.abs(np.diff(full.rmse))
    first = int(np.argmax(d < 1e-3)) + 1 if (d < 1e-3).any() else 20
    assert k == min(first + 1, 20)
    assert np.array_equal(early.rmse, full.rmse[:k])


def _dilated_vm_np(hist, off, vm, roots):
    """vm with Mask(root) written into the count word of every empty voxel
    that has a root (Alg. 3), from the closed-form roots."""
    vm = vm.copy()
    for v in np.nonzero((hist == 0) & (roots != np.uint32(0xFFFFFFFF)))[0]:
        vm[int(off[v]) + 1] = roots[v] | np.uint32(0x80000000)
    return vm


@pytest.mark.parametrize("seed,n,m,voxel,L", [(90, 300, 200, 0.25, 2), (91, 250, 180, 0.4, 1)])
def test_icp_rmse_is_root_mean_of_the_iterations_squared_distances(seed, n, m, voxel, L):
    # Sec. IV.A's stop rule compares RMSE values: RMSE_k = sqrt((1/m) sum_i d_i),
    # d_i the squared distance of query i to its Alg. 4 correspondence at
    # iteration k's float32 pose.  The d_i come from the independent rule
    # (exact rational float32 rounding), the grid from bincount/argsort and
    # the closed form of dilation, the sum is exact (fsum); iteration k's pose
    # is the pose after k iterations.  The last iteration's correspondences,
    # which a registration reports, are pinned the same way.
    q = synth.tiny_cloud(seed, n, dup=n // 10)
    p = synth.tiny_cloud(seed + 1, m, scale=1.2)
    K = 4
    ref = oracle.register(q, p, voxel, L, K)
    origin, inv, dims, V = oracle.grid_spec(q, voxel, L)
    hist, off, vm = segments_np(q, origin, inv, dims, V)
    vm = _dilated_vm_np(hist, off, vm, closed_form_roots(hist, dims, L))
    fallbacks = 0
    for k in range(K):
        pose = oracle.register(q, p, voxel, L, k).Rt if k else oracle.identity_rt()
        idx, d2, fb = nns_rule(q, p, pose.astype(np.float32), origin, inv, dims, hist, off, vm)
        want = math.sqrt(math.fsum(float(d) for d in d2.astype(np.float64)) / m)
        assert ref.rmse[k] == pytest.approx(want, rel=1e-12, abs=0), k
        assert ref.fallbacks[k] == fb, k
        fallbacks += fb
    assert fallbacks > 0                      # the source reaches outside the grid
    assert np.array_equal(ref.nn_idx, idx) and np.array_equal(ref.nn_d2.view(np.uint32), d2.view(np.uint32))


@pytest.mark.parametrize("name", ["sphere_2k", "bumpy_40k"])
def test_threaded_search_gives_identical_results(name):
    # Alg. 4's per-query loop on several threads (the oracle's one parallel
    # loop) returns the same registration, bit for bit, as one thread
    P = synth.config(name)
    K = 6
    try:
        assert oracle.set_threads(1) == 1
        a = oracle.register(P.q, P.p, P.voxel, P.rings, K)
        assert oracle.set_threads(8) in (1, 8)
        b = oracle.register(P.q, P.p, P.voxel, P.rings, K)
        og = oracle.dilate(oracle.build_grid(P.q, P.voxel, P.rings), P.rings)
        Rt = np.asarray(a.Rt, np.float32)
        n8 = oracle.nns_counts(og, P.q, P.p, Rt)
        oracle.set_threads(1)
        n1 = oracle.nns_counts(og, P.q, P.p, Rt)
    finally:
        oracle.set_threads(1)
    assert np.array_equal(a.Rt, b.Rt) and np.array_equal(a.rmse, b.rmse)
    assert np.array_equal(a.fallbacks, b.fallbacks)
    assert np.array_equal(a.nn_idx, b.nn_idx) and np.array_equal(a.nn_d2, b.nn_d2)
    assert n1 == n8


def test_icp_empty_source_is_noop():
    q = synth.tiny_cloud(80, 10)
    r = oracle.register(q, np.zeros((3, 0), np.float32), 0.2, 1, 5)
    assert r.iters == 0 and np.array_equal(r.Rt, oracle.identity_rt())


# ------------------------------------------------------ differentiable loss

def test_se3_exp_matches_matrix_exponential():
    from scipy.linalg import expm
    rng = np.random.default_rng(90)
    for scale in (1e-7, 1e-3, 0.04, 0.3, 2.0):
        xi = rng.standard_normal(6) * scale
        R, t, J = oracle.se3_exp(xi)
        X = np.zeros((4, 4))
        X[:3, :3] = [[0, -xi[5], xi[4]], [xi[5], 0, -xi[3]], [-xi[4], xi[3], 0]]
        X[:3, 3] = xi[:3]
        T = expm(X)
        assert np.abs(T[:3, :3] - R).max() < 1e-13 and np.abs(T[:3, 3] - t).max() < 1e-13


@pytest.mark.parametrize("scale", [1e-5, 0.03, 0.5, 1.5])
def test_se3_left_jacobian_by_differences(scale):
    # Exp(xi + e) ~= Exp(J e) Exp(xi): columns of J from central differences of log
    from scipy.linalg import expm, logm
    rng = np.random.default_rng(91)
    xi = rng.standard_normal(6) * scale
    _, _, J = oracle.se3_exp(xi)

    def T(x):
        R, t, _ = oracle.se3_exp(x)
        M = np.eye(4)
        M[:3, :3] = R
        M[:3, 3] = t
        return M

    Ti = np.linalg.inv(T(xi))
    h = 1e-6
    for k in range(6):
        e = np.zeros(6)
        e[k] = h
        Lp = logm(T(xi + e) @ Ti).real
        Lm = logm(T(xi - e) @ Ti).real
        D = (Lp - Lm) / (2 * h)
        col = np.array([D[0, 3], D[1, 3], D[2, 3], D[2, 1], D[0, 2], D[1, 0]])
        assert np.abs(col - J[:, k]).max() < 1e-7


def _p2p_setup(seed=100, n=800, m=600):
    P = synth.bumpy_pair(seed=seed, n=n, m=m, voxel=0.1, rings=2)
    g = oracle.dilate(oracle.build_grid(P.q, 0.1, 2), 2)
    return P, g


@pytest.mark.parametrize("xi_scale", [0.0, 0.05])
def test_p2p_gradient_by_finite_differences(xi_scale):
    P, g = _p2p_setup()
    rng = np.random.default_rng(101)
    xi = rng.standard_normal(6) * xi_scale
    loss, dP, dxi, idx = oracle.p2p(g, P.q, P.p, xi)
    p64 = P.p.astype(np.float64)
    assert abs(loss - oracle.p2p_loss_fixed(P.q, p64, idx, xi)) < 1e-15 * max(1, loss)
    h = 1e-6
    for _ in range(8):
        dp = rng.standard_normal(p64.shape)
        dx = rng.standard_normal(6)
        nrm = math.sqrt((dp * dp).sum() + (dx * dx).sum())
        dp, dx = dp / nrm, dx / nrm
        fp = oracle.p2p_loss_fixed(P.q, p64 + h * dp, idx, xi + h * dx)
        fm = oracle.p2p_loss_fixed(P.q, p64 - h * dp, idx, xi - h * dx)
        fd = (fp - fm) / (2 * h)
        an = float((dP * dp).sum() + (dxi * dx).sum())
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * np.abs(dxi).max())


def test_p2p_gradient_zero_at_alignment():
    q = synth.tiny_cloud(110, 300)
    g = oracle.dilate(oracle.build_grid(q, 0.2, 1), 1)
    loss, dP, dxi, idx = oracle.p2p(g, q, q, np.zeros(6))
    assert loss == 0 and (dP == 0).all() and (dxi == 0).all()


def test_p2p_translation_gradient_closed_form():
    # with R = I the rho-gradient is (2/m) sum r_i and dL/dp_i = (2/m) r_i
    P, g = _p2p_setup(seed=102)
    xi = np.array([0.01, -0.02, 0.005, 0, 0, 0])
    loss, dP, dxi, idx = oracle.p2p(g, P.q, P.p, xi)
    r = P.p.astype(np.float64) + xi[:3, None] - P.q[:, idx].astype(np.float64)
    m = P.m
    assert np.allclose(dxi[:3], 2.0 / m * r.sum(1), rtol=1e-12, atol=1e-15)
    assert np.allclose(dP, 2.0 / m * r, rtol=1e-12, atol=1e-18)
    assert abs(loss - (r * r).sum() / m) < 1e-14


# ------------------------------------------------- Table 1 memory accounting

def test_table1_static_footprint_and_units():
    t = json.load(open(os.path.join(GOLDEN, "table1_memory.json")))
    V = (2 ** t["grid_N"]) ** 3
    assert oracle.paper_static_bytes(V) / 2 ** 20 == t["static_mb"]


def test_table1_vanicp_is_64k_per_voxel_and_saving_formula():
    t = json.load(open(os.path.join(GOLDEN, "table1_memory.json")))
    for row in t["rows"]:
        voxels = row["vanicp_mb"] * 2 ** 20 / oracle.VANICP_BYTES_PER_VOXEL
        assert voxels == int(voxels)                               # whole 64 KB blocks
        assert oracle.vanicp_bytes(int(voxels)) == row["vanicp_mb"] * 2 ** 20
        s = 100.0 * oracle.saving(row["ours_mb"], row["vanicp_mb"])
        # Table 1 prints one decimal, apparently truncated in one row (TUM: 99.908 -> 99.9)
        assert abs(s - row["saving_pct"]) < 0.1, row


def test_dynamic_bytes_counts_two_header_words_per_voxel():
    q = synth.tiny_cloud(120, 500)
    g = oracle.build_grid(q, 0.2, 1)
    assert oracle.dynamic_bytes(g.n, g.V) == 4 * len(g.vm) == 4 * int(g.off[-1])


# ---- the paper's own setting (Sec. IV.A): unit sphere, 2^N grid, L = 10 ----

def test_fixed_grid_matches_independent_voxelisation_and_table1_static():
    P = synth.config("paper_bunny_40k")
    origin, dims = P.meta["grid_origin"], P.meta["grid_dims"]
    g = oracle.build_grid_fixed(P.q, origin, P.voxel, dims)
    assert g.V == 16 ** 3 and float(g.inv) == 8.0
    vid = voxel_ids_np(P.q, g.origin, g.inv, g.dims)
    assert (vid >= 0).all()
    assert np.array_equal(g.hist, np.bincount(vid, minlength=g.V).astype(np.uint32))
    _, off, vm = segments_np(P.q, g.origin, g.inv, g.dims, g.V)
    assert np.array_equal(g.off, off) and np.array_equal(g.vm, vm)
    # Table 1 note 1: the static footprint of the N = 4 grid
    t = json.load(open(os.path.join(GOLDEN, "table1_memory.json")))
    assert oracle.paper_static_bytes(g.V) / 2 ** 20 == t["static_mb"]


def test_fixed_grid_rejects_a_target_outside():
    q = synth.tiny_cloud(40, 100) * np.float32(0.5)
    q[0, 7] = np.float32(1.0)                     # on the far face: floor((1 + 1) * 8) = 16 is outside
    with pytest.raises(ValueError):
        oracle.build_grid_fixed(q, (-1.0, -1.0, -1.0), 0.125, (16, 16, 16))


def test_paper_setting_registration_converges_and_stops_early():
    P = synth.config("paper_bunny_40k")
    r = oracle.register_fixed(P.q, P.p, P.meta["grid_origin"], P.voxel, P.meta["grid_dims"], P.rings, P.iters,
                              P.meta["rmse_eps"], True)
    assert 2 <= r.iters < P.iters                   # the RMSE-difference rule ends it
    assert abs(r.rmse[-1] - r.rmse[-2]) < P.meta["rmse_eps"]
    assert r.rmse[-1] < r.rmse[0]
    # the same grid taken through the generic entry (explicit spec) gives the same registration
    g = oracle.dilate(oracle.build_grid_fixed(P.q, P.meta["grid_origin"], P.voxel, P.meta["grid_dims"]), P.rings)
    idx, d2, F, _ = oracle.nns(g, P.q, P.p, np.asarray(r.Rt, np.float32))
    assert F == 0


def test_exhaustive_comparator_is_exact_nn_and_svd():
    # Table 2's "Brute": every correspondence is the exact nearest target and
    # the pose is the textbook SVD solution on them
    q = synth.tiny_cloud(50, 400)
    p = synth.tiny_cloud(51, 150) * np.float32(0.9)
    r = oracle.register_global(q, p, 1)
    assert r.iters == 1 and r.fallbacks[0] == p.shape[1]
    for i in range(p.shape[1]):
        d, j = _exact_nn(q, p[:, i])
        assert r.nn_idx[i] == j and r.nn_d2[i] == d
    R, t, _ = kabsch_svd(p.astype(np.float64), q[:, r.nn_idx].astype(np.float64))
    assert np.abs(r.Rt[:9].reshape(3, 3) - R).max() < 1e-11 and np.abs(r.Rt[9:] - t).max() < 1e-11
