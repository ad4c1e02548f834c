"""Schedules never change a result.

Every build schedule (points per count block; all rings in one launch on
each LDS tile shape, or one launch per ring at each block size) gives the
oracle's histogram, offsets and dilated voxel index word for word, for every
ring count the one-launch form takes, on grids whose edges cut tiles.  The
autotuner, which re-runs the count and the dilation while it times them,
leaves the grid and every correspondence as they were, and stores the
schedule it picks per shape, in the process and in the file named by
VICP_AUTOTUNE_CACHE.
"""
import json
import os
import subprocess
import sys
import time

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

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BUILD_SCHEDULES = ([(cb, True, t, 256) for cb in (256, 512, 1024) for t in range(5)] +
                   [(256, False, 0, rb) for rb in (64, 128, 256)] + [(1024, False, 0, 64)])


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _case(name):
    if name == "tiny_ragged":
        q = synth.tiny_cloud(31, 6000, dup=300)
        return q, 0.13, 4
    P = synth.config(name)
    return P.q, P.voxel, P.rings


@pytest.mark.parametrize("name", ["tiny_ragged", "bumpy_40k", "room_226k"])
def test_every_build_schedule_gives_the_oracle_grid(name):
    q, voxel, L = _case(name)
    og = oracle.build_grid(q, voxel, L)
    hist0, off0 = og.hist.copy(), og.off.copy()
    oracle.dilate(og, L)
    qd = dev(q)
    g = build_grid(qd, voxel, L)
    for sched in BUILD_SCHEDULES:
        g.set_build_schedule(*sched)
        assert g.build_schedule == dict(zip(("count_block", "dilate_fused", "dilate_tile", "ring_block"), sched))
        g.rebuild(qd).dilate(L)
        hist, off, vm = g.export()
        assert np.array_equal(hist, hist0) and np.array_equal(off, off0), sched
        assert np.array_equal(vm, og.vm), sched
        d = g.describe()
        assert d["dilated"] == int(((og.vm[og.off[:-1] + 1] & np.uint32(0x80000000)) != 0).sum())


@pytest.mark.parametrize("rings", [1, 2, 3, 4])
def test_each_tile_shape_for_each_ring_count(rings):
    q = synth.tiny_cloud(32, 2500, dup=100)
    voxel = 0.09                                         # about 23 voxels per axis: tiles cut at every edge
    og = oracle.dilate(oracle.build_grid(q, voxel, 4), rings)
    qd = dev(q)
    g = build_grid(qd, voxel, 4)
    for tile in range(5):
        g.set_build_schedule(256, True, tile, 256)
        g.rebuild(qd).dilate(rings)
        assert np.array_equal(g.export()[2], og.vm), tile


def test_build_schedule_rejects_unsupported_values():
    g = build_grid(dev(synth.tiny_cloud(33, 500)), 0.2, 2)
    for bad in ((128, True, 0, 256), (256, True, 5, 256), (256, False, 0, 512), (2048, True, 0, 256), (256, True, -1, 64)):
        with pytest.raises(VicpError) as e:
            g.set_build_schedule(*bad)
        assert e.value.code == ERR_INVALID_ARG


def test_autotune_leaves_grid_and_correspondences_and_caches_the_schedule():
    P = synth.config("room_226k")
    og = oracle.dilate(oracle.build_grid(P.q, P.voxel, P.rings), P.rings)
    g = build_grid(dev(P.q), P.voxel, P.rings).dilate(P.rings)
    p = dev(P.p)
    Rt = np.array([1, 0, 0, 0, 1, 0, 0, 0, 1, 0.03, -0.02, 0.01], np.float32)
    i0, d0, f0 = (t.cpu().numpy() for t in g.nns(p, Rt))
    r0 = g.register(p, 6, correspondences=True)
    autotune_cache_clear()
    t0 = time.perf_counter()
    g.autotune(p, searches_per_plan=P.iters)
    t_tune = time.perf_counter() - t0
    tuned = (g.schedule, g.build_schedule)
    hist, off, vm = g.export()                           # the count and dilation were re-run while timed
    assert np.array_equal(hist, og.hist) and np.array_equal(off, og.off) and np.array_equal(vm, og.vm)
    i1, d1, f1 = (t.cpu().numpy() for t in g.nns(p, Rt))
    assert np.array_equal(i0, i1) and np.array_equal(d0, d1) and np.array_equal(f0, f1)
    r1 = g.register(p, 6, correspondences=True)
    assert np.array_equal(r0.nn_idx.cpu().numpy(), r1.nn_idx.cpu().numpy())
    assert np.array_equal(r0.fallbacks[0], r1.fallbacks[0]) and np.array_equal(r0.candidates[0], r1.candidates[0])
    assert np.abs(r0.Rt - r1.Rt).max() <= 1e-10 * max(1.0, P.extent)
    # the same shape again: the stored schedule, without timing
    g.set_schedule(512, 1, False, 1024, 0)
    g.set_build_schedule(1024, False, 0, 64)
    t0 = time.perf_counter()
    g.autotune(p, searches_per_plan=P.iters)
    t_cached = time.perf_counter() - t0
    assert (g.schedule, g.build_schedule) == tuned
    assert t_cached < 0.25 * t_tune, (t_cached, t_tune)
    # another searches-per-plan figure is another shape
    g.autotune(p, searches_per_plan=1)
    assert g.build_schedule["count_block"] in (256, 512, 1024)


_SCRIPT = r"""
import json, sys, time
import numpy as np, torch
sys.path.insert(0, sys.argv[1])
from paper_2512_04996_amd import synth
from paper_2512_04996_amd.api import build_grid
P = synth.config("sphere_2k")
g = build_grid(torch.from_numpy(P.q).cuda(), P.voxel, P.rings).dilate(P.rings)
p = torch.from_numpy(P.p).cuda()
if sys.argv[2] == "second":
    g.set_schedule(512, 1, False, 1024, 0)
    g.set_build_schedule(1024, False, 0, 64)
t0 = time.perf_counter()
g.autotune(p, searches_per_plan=P.iters)
print(json.dumps({"schedule": g.schedule, "build": g.build_schedule, "s": time.perf_counter() - t0}))
"""


def test_autotune_file_cache_across_processes(tmp_path):
    cache = tmp_path / "tune.txt"
    env = dict(os.environ, VICP_AUTOTUNE_CACHE=str(cache))
    out = []
    for which in ("first", "second"):
        print(f"[autotune cache] {which} process", flush=True)
        r = subprocess.run([sys.executable, "-c", _SCRIPT, ROOT, which], env=env, capture_output=True, text=True,
                           timeout=100)
        assert r.returncode == 0, r.stderr[-2000:]
        out.append(json.loads(r.stdout.strip().splitlines()[-1]))
    assert out[0]["schedule"] == out[1]["schedule"] and out[0]["build"] == out[1]["build"]
    lines = [line for line in cache.read_text().splitlines() if line.strip()]
    assert len(lines) == 1 and "\t" in lines[0]
