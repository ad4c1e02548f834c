"""Element-wise parity of the registration itself: the correspondences that
the registration's own search (Alg. 4 in its moment-summing form) and solve
kernels find in the last iteration, against the oracle's, index for index
and float32 distance bit for bit.

Each case runs the full loop of Sec. II.A on the GPU and in the oracle, then
compares the last iteration's nearest-neighbour index and squared distance of
every source point, the per-iteration global-search counts, the RMSE history
(1e-9 relative) and the final pose (1e-5 rad, 1e-6 x extent).  Schedules:
the autotuned one and both candidate loops (search_mode 0 and 1, 1 to 8
lanes per query, bucketed and not), eager and graph-replayed; on sources
shorter than one wave's queries and with ragged tails; with global
searches in the compared iteration (listed queries resolved by the exact
search and added by the solve), the exhaustive comparator, VANICP's layout
and the early stop.
"""
import math
import os

import numpy as np
import pytest

import oracle
from paper_2512_04996_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2512_04996_amd._lib import ERR_INVALID_ARG, VicpError  # noqa: E402
from paper_2512_04996_amd.api import autotune_cache_clear, build_grid  # noqa: E402

ROT_TOL = 1e-5
T_TOL = 1e-6
oracle.set_threads(min(16, len(os.sched_getaffinity(0))))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def rot_angle(R1, R2):
    return float(np.arccos(np.clip((np.trace(np.asarray(R1).reshape(3, 3).T @ np.asarray(R2).reshape(3, 3)) - 1) / 2,
                                   -1.0, 1.0)))


def assert_registration_equal(res, ref, extent, pair=0):
    assert int(res.iters[pair]) == ref.iters
    assert list(res.fallbacks[pair]) == list(ref.fallbacks)
    np.testing.assert_allclose(res.rmse[pair], ref.rmse, rtol=1e-9, atol=0)
    Rt = res.Rt if res.Rt.ndim == 1 else res.Rt[pair]
    assert rot_angle(Rt[:9], ref.Rt[:9]) <= ROT_TOL
    assert np.linalg.norm(Rt[9:] - ref.Rt[9:]) <= T_TOL * extent


def assert_correspondences_equal(idx, d2, ref):
    idx = idx.cpu().numpy() if hasattr(idx, "cpu") else idx
    d2 = d2.cpu().numpy() if hasattr(d2, "cpu") else d2
    assert idx.shape == ref.nn_idx.shape
    bad = np.nonzero(idx != ref.nn_idx)[0]
    assert bad.size == 0, f"{bad.size} indices differ, first at {bad[:5]}"
    assert np.array_equal(d2.view(np.uint32), ref.nn_d2.view(np.uint32))


_REF = {}


def reference(name):
    if name not in _REF:
        P = synth.config(name)
        _REF[name] = (P, oracle.register(P.q, P.p, P.voxel, P.rings, P.iters))
    return _REF[name]


SCHEDULES = [
    "auto",
    (256, 4, True, 64, 0),
    (256, 4, True, 64, 1),
    (128, 8, False, 128, 1),
    (512, 8, True, 256, 0),
    (128, 2, True, 64, 0),
    (256, 1, False, 64, 0),
    (128, 2, True, 1024, 1),
    (256, 1, False, 64, 1),
]


@pytest.mark.parametrize("name", ["bumpy_40k", "room_226k"])
@pytest.mark.parametrize("sched", SCHEDULES, ids=lambda s: s if isinstance(s, str) else "-".join(map(str, s)))
def test_registration_correspondences_match_oracle(name, sched):
    P, ref = reference(name)
    g = build_grid(dev(P.q), P.voxel, P.rings).dilate(P.rings)
    p = dev(P.p)
    if sched == "auto":
        autotune_cache_clear()
        g.autotune(p, searches_per_plan=P.iters)
    else:
        bs, lpq, srt, fg, mode = sched
        g.set_schedule(bs, lpq, srt, fg, mode)
    for use_graph in (True, False):
        res = g.register(p, P.iters, use_graph=use_graph, correspondences=True)
        assert_registration_equal(res, ref, P.extent)
        assert_correspondences_equal(res.nn_idx, res.nn_d2, ref)


def test_correspondences_of_globally_searched_queries():
    # the source starts several voxels off the target: in iteration 0 most
    # queries (over 8192) take the global search, resolved by the search's
    # voxel shells or, the farthest, by the exhaustive search and the solve
    P = synth.bumpy_pair(seed=21, n=6000, m=20000, voxel=0.05, rings=2, iters=8)
    Rt0 = np.array([1, 0, 0, 0, 1, 0, 0, 0, 1, 0.4, -0.1, 0.05], np.float64)
    g = build_grid(dev(P.q), P.voxel, 2).dilate(2)
    p = dev(P.p)
    for K in (1, 2, 8):
        ref = oracle.register(P.q, P.p, P.voxel, 2, K, Rt0=Rt0)
        if K == 1:
            assert ref.fallbacks[0] > 8192
        for use_graph in (False, True):
            res = g.register(p, K, Rt0=Rt0, use_graph=use_graph, correspondences=True)
            assert_registration_equal(res, ref, P.extent)
            assert_correspondences_equal(res.nn_idx, res.nn_d2, ref)


def test_correspondences_exhaustive_comparator():
    P = synth.room_pair(seed=32, n=8000, m=6000, voxel=0.1, rings=2, iters=4)
    g = build_grid(dev(P.q), P.voxel, P.rings).dilate(P.rings)
    res = g.register(dev(P.p), 4, global_only=True, correspondences=True)
    ref = oracle.register_global(P.q, P.p, 4)
    assert_registration_equal(res, ref, P.extent)
    assert_correspondences_equal(res.nn_idx, res.nn_d2, ref)


def test_correspondences_direct_layout_with_overflow():
    P = synth.room_pair(seed=43, n=9000, m=7000, voxel=0.1, rings=2, iters=5)
    g = build_grid(dev(P.q), P.voxel, P.rings).dilate(P.rings)
    g.build_direct(16 * 3)                              # 3 points per block: dense voxels overflow
    res = g.register(dev(P.p), 5, layout="direct", correspondences=True)
    ref = oracle.register_direct(P.q, P.p, P.voxel, P.rings, 5, block_bytes=16 * 3)
    assert ref.fallbacks[-1] > 0
    assert_registration_equal(res, ref, P.extent)
    assert_correspondences_equal(res.nn_idx, res.nn_d2, ref)


def test_correspondences_after_early_stop():
    # the stopped pair keeps the correspondences of the last iteration it ran
    P, _ = reference("bumpy_40k")
    ref = oracle.register(P.q, P.p, P.voxel, P.rings, P.iters, rmse_eps=1e-4, early_stop=True)
    g = build_grid(dev(P.q), P.voxel, P.rings).dilate(P.rings)
    res = g.register(dev(P.p), P.iters, rmse_eps=1e-4, early_stop=True, correspondences=True)
    assert ref.iters < P.iters
    assert_registration_equal(res, ref, P.extent)
    assert_correspondences_equal(res.nn_idx, res.nn_d2, ref)


def test_grid_beyond_the_coordinate_limit_is_refused():
    q = synth.tiny_cloud(7, 100)
    q[0, 3] = np.float32(2e18)
    with pytest.raises(VicpError) as e:
        build_grid(dev(q), 1e16, 1)
    assert e.value.code == ERR_INVALID_ARG
    q[0, 3] = np.float32(9e17)                          # inside the limit, padding included
    g = build_grid(dev(q), 1e16, 1).dilate(1)
    idx, d2, _ = g.nns(dev(q), np.array([1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0], np.float32))
    assert np.isfinite(d2.cpu().numpy()).all()
    assert math.isfinite(float(d2.max()))


@pytest.mark.parametrize("m", [31, 1000, 70001])
def test_registration_on_ragged_sources(m):
    # sources shorter than one wave's queries, a few blocks, and a ragged tail
    P = synth.bumpy_pair(seed=61, n=20000, m=m, voxel=0.05, rings=2, iters=4)
    ref = oracle.register(P.q, P.p, P.voxel, 2, 4)
    g = build_grid(dev(P.q), P.voxel, 2).dilate(2)
    p = dev(P.p)
    for sched in ((128, 2, True, 64, 0), (256, 4, True, 64, 1), (512, 8, False, 64, 0), (256, 1, True, 64, 0)):
        g.set_schedule(*sched)
        for use_graph in (False, True):
            res = g.register(p, 4, use_graph=use_graph, correspondences=True)
            assert_registration_equal(res, ref, P.extent)
            assert_correspondences_equal(res.nn_idx, res.nn_d2, ref)
