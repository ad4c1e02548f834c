"""GPU parity of VANICP's monolithic layout (the comparator of Sec. II.B and
Sec. IV.B): fixed per-voxel blocks holding copies of the points, dilated
voxels holding copies of their roots' points, and the global search for a
voxel whose points exceed a block.

Without overflow the registration equals the segmented layout's bit for bit
under the same schedule (the same candidates per query, the same lowest-index
rule on ties, the same per-block moment sums).  With overflow it follows the
oracle's capacity rule: fallback counts and counters exact, the pose within
1e-5 rad and 1e-6 x extent.
"""
import numpy as np
import pytest

import oracle
from paper_2512_04996_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():   # collected on CPU machines, skipped there
    pytest.skip("no GPU", allow_module_level=True)

from paper_2512_04996_amd._lib import ERR_INVALID_ARG, ERR_STATE, VicpError  # noqa: E402
from paper_2512_04996_amd.api import build_grid, build_grid_batched, build_grid_fixed  # noqa: E402

ROT_TOL = 1e-5
T_TOL = 1e-6
IDENT = np.array([1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0], np.float32)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def rot_angle(R1, R2):
    return float(np.arccos(np.clip((np.trace(np.asarray(R1).reshape(3, 3).T @ np.asarray(R2).reshape(3, 3)) - 1) / 2,
                                   -1.0, 1.0)))


def assert_matches_oracle(res, ref, extent):
    assert res.iters[0] == ref.iters
    assert list(res.fallbacks[0]) == list(ref.fallbacks)
    np.testing.assert_allclose(res.rmse[0], ref.rmse, rtol=1e-9, atol=0)
    assert rot_angle(res.Rt[:9], ref.Rt[:9]) <= ROT_TOL
    assert np.linalg.norm(res.Rt[9:] - ref.Rt[9:]) <= T_TOL * extent


@pytest.mark.parametrize("case", ["bumpy", "room"])
def test_direct_layout_equals_segmented_without_overflow(case):
    if case == "bumpy":
        P = synth.bumpy_pair(seed=41, n=6000, m=5000, voxel=0.05, rings=2, iters=6)
    else:
        P = synth.room_pair(seed=42, n=9000, m=7000, voxel=0.1, rings=3, iters=6)
    g = build_grid(dev(P.q), P.voxel, P.rings).dilate(P.rings)
    g.set_schedule(256, 2, True, 256)
    og = oracle.build_grid(P.q, P.voxel, P.rings)
    block = 16 * (int(og.hist.max()) + 3)   # every voxel fits its block
    g.build_direct(block)
    p = dev(P.p)
    for use_graph in (False, True):
        a = g.register(p, P.iters, use_graph=use_graph)
        b = g.register(p, P.iters, use_graph=use_graph, layout="direct")
        assert np.array_equal(a.Rt, b.Rt) and np.array_equal(a.rmse[0], b.rmse[0])
        assert np.array_equal(a.fallbacks[0], b.fallbacks[0])
        assert np.array_equal(a.candidates[0], b.candidates[0])
        assert np.array_equal(a.dilated_lookups[0], b.dilated_lookups[0])
        ref = oracle.register_direct(P.q, P.p, P.voxel, P.rings, P.iters, block_bytes=block)
        assert_matches_oracle(b, ref, P.extent)


@pytest.mark.parametrize("cap", [1, 3, 8])
def test_direct_layout_overflow_matches_oracle(cap):
    P = synth.room_pair(seed=43, n=9000, m=7000, voxel=0.1, rings=2, iters=6)
    block = 16 * cap
    g = build_grid(dev(P.q), P.voxel, P.rings).dilate(P.rings)
    g.build_direct(block)
    p = dev(P.p)
    base = g.register(p, P.iters)
    for sched in ((256, 2, True, 256), (128, 4, False, 64)):
        g.set_schedule(*sched)
        res = g.register(p, P.iters, layout="direct")
        ref = oracle.register_direct(P.q, P.p, P.voxel, P.rings, P.iters, block_bytes=block)
        assert ref.fallbacks[0] > base.fallbacks[0][0]     # overflowed blocks send queries to the global search
        assert_matches_oracle(res, ref, P.extent)
    # first-iteration counters against the oracle's capacity rule
    og = oracle.dilate(oracle.build_grid(P.q, P.voxel, P.rings), P.rings)
    F, cand, dil = oracle.nns_counts(og, P.q, P.p, IDENT, capacity=cap)
    assert (int(res.fallbacks[0][0]), int(res.candidates[0][0]), int(res.dilated_lookups[0][0])) == (F, cand, dil)


def test_direct_layout_at_full_size_with_64k_blocks():
    # the room workload at 64 KiB per voxel: about 21.8 GB of blocks
    P = synth.config("room_226k")
    g = build_grid(dev(P.q), P.voxel, P.rings).dilate(P.rings)
    g.set_schedule(128, 2, True, 64)
    g.build_direct(65536)
    p = dev(P.p)
    a = g.register(p, P.iters)
    b = g.register(p, P.iters, layout="direct")
    assert np.array_equal(a.Rt, b.Rt) and np.array_equal(a.fallbacks[0], b.fallbacks[0])
    assert np.array_equal(a.candidates[0], b.candidates[0])
    ref = oracle.register_direct(P.q, P.p, P.voxel, P.rings, P.iters)
    assert_matches_oracle(b, ref, P.extent)
    g.free_direct()


def test_direct_layout_paper_setting_overflows_like_the_paper():
    # Sec. IV.A's fixed 16^3 grid: the room's densest voxels hold more than
    # 4096 points, so their queries take the global search (Sec. IV.B)
    P = synth.config("paper_room_226k")
    o, d = P.meta["grid_origin"], P.meta["grid_dims"]
    g = build_grid_fixed(dev(P.q), o, P.voxel, d, P.rings).dilate(P.rings)
    g.build_direct(65536)
    K = 5
    res = g.register(dev(P.p), K, layout="direct")
    seg = g.register(dev(P.p), K)
    ref = oracle.register_fixed(P.q, P.p, o, P.voxel, d, P.rings, K, block_bytes=65536)
    assert_matches_oracle(res, ref, P.extent)
    assert ref.fallbacks[0] > seg.fallbacks[0][0]
    g.free_direct()


def test_direct_layout_errors():
    P = synth.bumpy_pair(seed=44, n=3000, m=2000, voxel=0.05, rings=1, iters=2)
    g = build_grid(dev(P.q), P.voxel, P.rings)
    p = dev(P.p)
    with pytest.raises(VicpError) as e:
        g.build_direct(4096)                   # not dilated yet
    assert e.value.code == ERR_STATE
    g.dilate(P.rings)
    with pytest.raises(VicpError) as e:
        g.register(p, 2, layout="direct")      # not built
    assert e.value.code == ERR_STATE
    for bad in (0, 8, 4100):
        with pytest.raises(VicpError) as e:
            g.build_direct(bad)
        assert e.value.code == ERR_INVALID_ARG
    g.build_direct(4096)
    with pytest.raises(VicpError) as e:
        g.register(p, 2, layout="direct", global_only=True)
    assert e.value.code == ERR_INVALID_ARG
    r1 = g.register(p, 2, layout="direct")
    g.rebuild(dev(P.q)).dilate(P.rings)        # a rebuild invalidates the blocks
    with pytest.raises(VicpError) as e:
        g.register(p, 2, layout="direct")
    assert e.value.code == ERR_STATE
    g.build_direct(4096)
    r2 = g.register(p, 2, layout="direct")
    assert np.array_equal(r1.Rt, r2.Rt)
    g.free_direct()
    with pytest.raises(VicpError) as e:
        g.register(p, 2, layout="direct")
    assert e.value.code == ERR_STATE
    g.free_direct()                            # no-op
    Q = [synth.tiny_cloud(50, 400), synth.tiny_cloud(51, 300)]
    gb = build_grid_batched(dev(np.concatenate(Q, axis=1)), [400, 300], [0.2, 0.2], 1).dilate(1)
    with pytest.raises(VicpError) as e:
        gb.build_direct(4096)
    assert e.value.code == ERR_INVALID_ARG
