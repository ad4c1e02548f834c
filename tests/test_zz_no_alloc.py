"""The allocation-free search entry point (vicp_nns_noalloc) against vicp_nns.

Both are called through the C ABI on the same grid and inputs; the outputs
must be identical bit for bit (NN indices, float32 distances, global-search
counts), on two calls in a row, the second with fewer source points, at a
pose where every query searches locally and at one that sends queries to the
global search.  The later calls must leave the device's free memory as it
was.  Also checked against the CPU oracle on the small case.
"""
import numpy as np
import pytest

import oracle
from paper_2512_04996_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2512_04996_amd._lib import ERR_INVALID_ARG, NOALLOC_MAX_QUERIES, VicpError  # noqa: E402
from paper_2512_04996_amd.api import build_grid  # noqa: E402

IDENT = np.array([1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0], np.float32)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def shifted(t):
    Rt = IDENT.copy()
    Rt[9:] = t
    return Rt


@pytest.mark.parametrize("name", ["bumpy_40k", "room_226k"])
def test_noalloc_equals_nns_two_calls(name):
    P = synth.config(name)
    g = build_grid(dev(P.q), P.voxel, P.rings).dilate(P.rings)
    p = dev(P.p)
    small = dev(P.p[:, : P.m // 3 + 17])                   # fewer points than the call before
    far = shifted([0.4 * P.extent, 0.0, 0.0])              # sends queries to the global search
    # two calls in a row, the second smaller, at a pose with and without
    # global searches
    cases = [(p, IDENT), (small, far), (p, far), (small, IDENT)]
    refs = []
    for pp, Rt in cases:
        idx, d2, fb = g.nns(pp, Rt)                       # the existing entry point (allocates)
        refs.append((idx.cpu().numpy(), d2.cpu().numpy(), int(fb.cpu()[0])))
    assert refs[1][2] > 0 and refs[2][2] > refs[0][2]
    outs = [(torch.empty(pp.shape[1], dtype=torch.int32, device="cuda"),
             torch.empty(pp.shape[1], dtype=torch.float32, device="cuda"),
             torch.zeros(1, dtype=torch.int32, device="cuda")) for pp, _ in cases]
    g.nns_noalloc(p, IDENT, *outs[0])                      # first use on this device locates the array
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for (pp, Rt), o in zip(cases, outs):
        g.nns_noalloc(pp, Rt, *o)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0           # nothing was allocated
    for (ridx, rd2, rfb), (idx, d2, fb) in zip(refs, outs):
        assert np.array_equal(idx.cpu().numpy(), ridx)
        assert np.array_equal(d2.cpu().numpy().view(np.uint32), rd2.view(np.uint32))
        assert int(fb.cpu()[0]) == rfb


def test_noalloc_matches_oracle_and_limits():
    q = synth.tiny_cloud(41, 5000, dup=200)
    pts = synth.tiny_cloud(42, 3000, scale=1.4)            # some queries land outside the grid
    g = build_grid(dev(q), 0.15, 2).dilate(2)
    og = oracle.dilate(oracle.build_grid(q, 0.15, 2), 2)
    for pp in (pts, pts[:, :1234]):
        m = pp.shape[1]
        idx = torch.empty(m, dtype=torch.int32, device="cuda")
        d2 = torch.empty(m, dtype=torch.float32, device="cuda")
        fb = torch.zeros(1, dtype=torch.int32, device="cuda")
        g.nns_noalloc(dev(pp), IDENT, idx, d2, fb)
        ridx, rd2, rF, _ = oracle.nns(og, q, pp, IDENT)
        assert rF > 0 and int(fb.cpu()[0]) == rF
        assert np.array_equal(idx.cpu().numpy(), ridx)
        assert np.array_equal(d2.cpu().numpy().view(np.uint32), rd2.view(np.uint32))
    # an empty source is a no-op that reports no global search
    fb = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    e = torch.zeros((3, 0), dtype=torch.float32, device="cuda")
    g.nns_noalloc(e, IDENT, torch.empty(1, dtype=torch.int32, device="cuda"),
                  torch.empty(1, dtype=torch.float32, device="cuda"), fb)
    assert int(fb.cpu()[0]) == 0
    # more source points than the fixed array holds: refused on the host
    big = torch.zeros((3, NOALLOC_MAX_QUERIES + 1), dtype=torch.float32, device="cuda")
    with pytest.raises(VicpError) as ex:
        g.nns_noalloc(big, IDENT, torch.empty(NOALLOC_MAX_QUERIES + 1, dtype=torch.int32, device="cuda"),
                      torch.empty(NOALLOC_MAX_QUERIES + 1, dtype=torch.float32, device="cuda"))
    assert ex.value.code == ERR_INVALID_ARG
