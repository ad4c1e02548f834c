"""GPU: the next frame in one call (vicp_rebuild_register) against the three
calls in turn.

The combined call runs each of the refill's count, scan, scatter and order
passes in one launch with the source bucketing's matching pass.  Its results
must equal those of rebuild, dilate and register
run one after the other on a second grid built the same way: the final pose
bit for bit, the RMSE, global-search, candidate and dilated-lookup histories,
the iteration counts and the last iteration's correspondences.  Frames change
the target's pose (same grid shape) and its scale (a new grid shape, so the
voxel buffers and the source workspace are rebuilt inside the call); one
call changes the source's size; batches of 5 and 64 pairs start from a
distinct pose per pair.  One frame is also checked against the
oracle, and the forms that take the plain path (source in index order) and
the argument errors are covered.
"""
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
from paper_2512_04996_amd.api import build_grid, build_grid_batched  # noqa: E402

oracle.set_threads(min(16, len(os.sched_getaffinity(0))))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _rotz(deg):
    a = np.deg2rad(deg)
    return np.array([[np.cos(a), -np.sin(a), 0.0], [np.sin(a), np.cos(a), 0.0], [0.0, 0.0, 1.0]])


def _frames(q):
    """The same target moved by 1 degree and 1 cm (same grid shape), then
    scaled by 1.05 about its centre (more voxels), then moved back."""
    q64 = q.astype(np.float64)
    c = q64.mean(1, keepdims=True)
    moved = (_rotz(1.0) @ (q64 - c) + c + np.array([[0.01], [0.0], [-0.01]])).astype(np.float32)
    scaled = (1.05 * (q64 - c) + c).astype(np.float32)
    return [moved, scaled, moved]


def _same(a, b, B):
    assert np.array_equal(np.asarray(a.Rt), np.asarray(b.Rt))
    assert np.array_equal(a.iters, b.iters)
    for k in range(B):
        assert np.array_equal(a.rmse[k], b.rmse[k]), k
        assert np.array_equal(a.fallbacks[k], b.fallbacks[k]), k
        assert np.array_equal(a.candidates[k], b.candidates[k]), k
        assert np.array_equal(a.dilated_lookups[k], b.dilated_lookups[k]), k
    if a.nn_idx is not None:
        assert torch.equal(a.nn_idx, b.nn_idx)
        assert torch.equal(a.nn_d2.view(torch.int32), b.nn_d2.view(torch.int32))


@pytest.mark.parametrize("mode", [0, 1])
def test_single_pair_frames_match_three_calls(mode):
    P = synth.config("room_226k")
    L, K = P.rings, P.iters
    q0, p = dev(P.q), dev(P.p)
    sched = dict(nns_block=128, lanes_per_query=2, sort_source=True, fallback_grid=1024, search_mode=mode)
    ga = build_grid(q0, P.voxel, L).dilate(L).set_schedule(**sched)
    gb = build_grid(q0, P.voxel, L).dilate(L).set_schedule(**sched)
    for f, q in enumerate(_frames(P.q)):
        qd = dev(q)
        ga.rebuild(qd).dilate(L)
        ra = ga.register(p, K, use_graph=True, correspondences=True)
        rb = gb.rebuild_register(qd, L, p, K, use_graph=True, correspondences=True)
        print(f"[rebuild_register] mode {mode} frame {f}: iters {int(rb.iters[0])}", flush=True)
        _same(ra, rb, 1)
        assert gb.describe()["rings_applied"] == L
    # a source of another size: the source workspace is rebuilt inside the call
    ph = dev(P.p[:, : P.m // 2])
    qd = dev(_frames(P.q)[0])
    ga.rebuild(qd).dilate(L)
    ra = ga.register(ph, K, use_graph=False)
    rb = gb.rebuild_register(qd, L, ph, K, use_graph=False)
    _same(ra, rb, 1)
    ga.free()
    gb.free()


def test_frame_matches_oracle():
    P = synth.config("bumpy_40k")
    q1 = _frames(P.q)[0]
    g = build_grid(dev(P.q), P.voxel, P.rings).dilate(P.rings)
    g.set_schedule(nns_block=256, lanes_per_query=2, sort_source=True, fallback_grid=256, search_mode=0)
    res = g.rebuild_register(dev(q1), P.rings, dev(P.p), P.iters, correspondences=True)
    ref = oracle.register(q1, P.p, P.voxel, P.rings, P.iters)
    assert int(res.iters[0]) == ref.iters
    assert list(res.fallbacks[0]) == list(ref.fallbacks)
    np.testing.assert_allclose(res.rmse[0], ref.rmse, rtol=1e-9, atol=0)
    assert np.array_equal(res.nn_idx.cpu().numpy(), ref.nn_idx)
    assert np.array_equal(res.nn_d2.cpu().numpy().view(np.uint32), ref.nn_d2.view(np.uint32))
    hist, off, vm = g.export()
    og = oracle.dilate(oracle.build_grid(q1, P.voxel, P.rings), P.rings)
    assert np.array_equal(hist, og.hist) and np.array_equal(off, og.off) and np.array_equal(vm, og.vm)
    g.free()


@pytest.mark.parametrize("npairs", [5, 64])
def test_batched_frames_match_three_calls(npairs):
    # 5 pairs: poses and records travel in the start launch; 64 pairs: the
    # poses go up by upload and the records by a separate copy
    pairs = synth.config("batched_64")[:npairs]
    ns, ms, vox = [x.n for x in pairs], [x.m for x in pairs], [x.voxel for x in pairs]
    q0 = np.concatenate([x.q for x in pairs], 1)
    pc = dev(np.concatenate([x.p for x in pairs], 1))
    sched = dict(nns_block=256, lanes_per_query=2, sort_source=True, fallback_grid=512, search_mode=1)
    ga = build_grid_batched(dev(q0), ns, vox, 3).dilate(3).set_schedule(**sched)
    gb = build_grid_batched(dev(q0), ns, vox, 3).dilate(3).set_schedule(**sched)
    frames = [np.concatenate([_frames(x.q)[i] for x in pairs], 1) for i in range(2)]
    # a distinct starting pose per pair (each must reach its own pair's state)
    rt0 = np.stack([np.concatenate([_rotz(0.2 * (b + 1)).reshape(-1), [1e-3 * b, 0.0, -1e-3 * b]])
                    for b in range(npairs)])
    for f, q in enumerate(frames):
        qd = dev(q)
        ga.rebuild(qd).dilate(3)
        ra = ga.register(pc, 30, m_per_pair=ms, use_graph=True, correspondences=True, Rt0=rt0)
        rb = gb.rebuild_register(qd, 3, pc, 30, m_per_pair=ms, use_graph=True, correspondences=True, Rt0=rt0)
        print(f"[rebuild_register] {npairs} pairs, frame {f}", flush=True)
        _same(ra, rb, len(pairs))
    ga.free()
    gb.free()


def test_index_order_source_and_errors():
    P = synth.config("bumpy_40k")
    q0, p = dev(P.q), dev(P.p)
    q1 = dev(_frames(P.q)[0])
    sched = dict(nns_block=256, lanes_per_query=2, sort_source=False, fallback_grid=256, search_mode=0)
    ga = build_grid(q0, P.voxel, P.rings).dilate(P.rings).set_schedule(**sched)
    gb = build_grid(q0, P.voxel, P.rings).dilate(P.rings).set_schedule(**sched)
    ga.rebuild(q1).dilate(P.rings)
    ra = ga.register(p, P.iters)
    rb = gb.rebuild_register(q1, P.rings, p, P.iters)
    _same(ra, rb, 1)
    with pytest.raises(VicpError) as e:
        gb.rebuild_register(q1, P.rings + 1, p, P.iters)   # more rings than the grid was padded for
    assert e.value.code == ERR_INVALID_ARG
    with pytest.raises(VicpError) as e:
        gb.rebuild_register(q1, P.rings, p, -1)
    assert e.value.code == ERR_INVALID_ARG
    # the grid still serves after the refused calls
    rb = gb.rebuild_register(q1, P.rings, p, P.iters)
    _same(ra, rb, 1)
    ga.free()
    gb.free()
