"""Python front end of libvicp: argument marshalling over torch device memory.

Every step of the method runs in the HIP library; this module only passes
pointers, sizes and torch's current stream, and converts results.  Point
clouds are float32 CUDA tensors in structure-of-arrays layout, shape (3, k)
(a (k, 3) tensor is accepted and transposed into a contiguous copy).
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import GridDesc, IcpOpts, IcpStats, VicpError, check, lib

__all__ = ["Grid", "build_grid", "build_grid_batched", "IcpResult", "prof_enable", "prof_read", "prof_samples",
           "prof_reset", "autotune_cache_clear"]


_raw_stream = getattr(torch._C, "_cuda_getCurrentRawStream", None)


def _stream():
    # torch's current stream as a raw handle (without building a Stream
    # object when torch exposes the handle directly)
    if _raw_stream is not None:
        return C.c_void_p(_raw_stream(torch.cuda.current_device()))
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _soa(x: torch.Tensor, what: str) -> torch.Tensor:
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{what} must be a CUDA tensor")
    if x.dtype != torch.float32:
        raise TypeError(f"{what} must be float32")
    if x.dim() != 2 or 3 not in x.shape:
        raise ValueError(f"{what} must have shape (3, k) or (k, 3)")
    if x.shape[0] != 3:
        x = x.t()
    return x.contiguous()


def _ptrs(x: torch.Tensor):
    # the three rows of a contiguous (3, k) float32 tensor
    if x.shape[1] == 0:
        return C.c_void_p(0), C.c_void_p(0), C.c_void_p(0)
    base, row = x.data_ptr(), x.stride(0) * x.element_size()
    return C.c_void_p(base), C.c_void_p(base + row), C.c_void_p(base + 2 * row)


def _i64(vals):
    arr = (C.c_int64 * len(vals))(*[int(v) for v in vals])
    return arr


_IDENTITY = np.array([1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0], np.float64)


@dataclass
class IcpResult:
    Rt: np.ndarray            # (12,) float64 or (B, 12): R row-major then t
    iters: np.ndarray         # (B,)
    degenerate: np.ndarray    # (B,)
    rmse: list                # per pair, float64[iters]
    fallbacks: list           # per pair, int64[iters]
    candidates: list          # per pair, int64[iters]: target points scanned by local searches
    dilated_lookups: list     # per pair, int64[iters]: local searches sent to a root voxel
    status: int
    nn_idx: object = None     # with correspondences=True: int32[m] CUDA tensor, the last iteration's targets
    nn_d2: object = None      # ... and their float32 squared distances


class Grid:
    """A built (and possibly dilated) target grid for one or more pairs."""

    def __init__(self, handle: C.c_void_p, q: torch.Tensor, n_per_pair, voxels, pad_rings: int):
        self._h = handle
        self.q = q                       # keeps the target alive for the grid's lifetime
        self.n_per_pair = [int(v) for v in n_per_pair]
        self.voxels = [float(v) for v in voxels]
        self.pad_rings = int(pad_rings)
        self.npairs = len(self.n_per_pair)
        self.n_total = sum(self.n_per_pair)
        self._stats_key = None           # host arrays the registration's statistics land in, per (B, K)
        self._stats = None

    # -- lifetime
    def free(self):
        if self._h is not None and self._h.value:
            lib().vicp_grid_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    @property
    def handle(self):
        if self._h is None:
            raise VicpError(_lib.ERR_STATE, "grid", "freed")
        return self._h

    def rebuild(self, q: torch.Tensor):
        """Refill the grid from a new target with the same per-pair point counts."""
        q = _soa(q, "q")
        if q.shape[1] != self.n_total:
            raise ValueError("rebuild needs the same number of target points")
        qx, qy, qz = _ptrs(q)
        check(lib().vicp_grid_rebuild(self.handle, qx, qy, qz, _stream()), "vicp_grid_rebuild")
        self.q = q
        return self

    def build_direct(self, block_bytes: int = 65536):
        """VANICP's monolithic layout beside this grid, for comparison: a fixed
        block of ``block_bytes`` per voxel (V * block_bytes device bytes) holding
        copies of the voxel's points, or of its root's for a dilated voxel.
        Needs a dilated single-pair grid; ``register(..., layout="direct")``
        then searches it."""
        check(lib().vicp_direct_build(self.handle, int(block_bytes), _stream()), "vicp_direct_build")
        return self

    def free_direct(self):
        """Release the blocks of build_direct."""
        check(lib().vicp_direct_free(self.handle), "vicp_direct_free")

    def set_build_options(self, host_offsets: bool = False, packed_hash: bool = False):
        """The Alg. 1 ablation for later rebuilds: offsets scanned on the host,
        counts with the fused 32-bit LDS hash entry (same grid either way)."""
        check(lib().vicp_set_build_options(self.handle, int(bool(host_offsets)), int(bool(packed_hash))),
              "vicp_set_build_options")
        return self

    @property
    def schedule(self) -> dict:
        a, l, b, c, r = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        check(lib().vicp_get_schedule(self.handle, C.byref(a), C.byref(l), C.byref(b), C.byref(c), C.byref(r)),
              "vicp_get_schedule")
        return {"nns_block": a.value, "lanes_per_query": l.value, "sort_source": bool(b.value),
                "fallback_grid": c.value, "search_mode": r.value}

    def set_schedule(self, nns_block: int = 256, lanes_per_query: int = 4, sort_source: bool = True,
                     fallback_grid: int = 128, search_mode: int = 0):
        check(lib().vicp_set_schedule(self.handle, int(nns_block), int(lanes_per_query), int(bool(sort_source)),
                                      int(fallback_grid), int(search_mode)), "vicp_set_schedule")
        return self

    @property
    def build_schedule(self) -> dict:
        a, b, c, d = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        check(lib().vicp_get_build_schedule(self.handle, C.byref(a), C.byref(b), C.byref(c), C.byref(d)),
              "vicp_get_build_schedule")
        return {"count_block": a.value, "dilate_fused": bool(b.value), "dilate_tile": c.value,
                "ring_block": d.value}

    def set_build_schedule(self, count_block: int = 256, dilate_fused: bool = True, dilate_tile: int = 0,
                           ring_block: int = 256):
        check(lib().vicp_set_build_schedule(self.handle, int(count_block), int(bool(dilate_fused)), int(dilate_tile),
                                            int(ring_block)), "vicp_set_build_schedule")
        return self

    # -- Alg. 3
    def dilate(self, rings: int):
        check(lib().vicp_dilate(self.handle, int(rings), _stream()), "vicp_dilate")
        return self

    # -- Alg. 4
    def nns(self, p: torch.Tensor, Rt, m_per_pair=None):
        """Correspondences of every source point at pose(s) Rt (float32,
        (12,) or (B, 12)).  Returns (nn_idx int32[m], nn_d2 float32[m],
        n_fallback int32[B]) as CUDA tensors."""
        p = _soa(p, "p")
        m = p.shape[1]
        if m_per_pair is None:
            if self.npairs != 1:
                raise ValueError("m_per_pair is required for a batched grid")
            m_per_pair = [m]
        if sum(m_per_pair) != m:
            raise ValueError("m_per_pair does not add up to the source size")
        rt = np.ascontiguousarray(np.asarray(Rt, np.float32).reshape(self.npairs * 12))
        idx = torch.empty(max(m, 1), dtype=torch.int32, device=p.device)
        d2 = torch.empty(max(m, 1), dtype=torch.float32, device=p.device)
        fb = torch.zeros(self.npairs, dtype=torch.int32, device=p.device)
        px, py, pz = _ptrs(p)
        check(lib().vicp_nns_batched(self.handle, px, py, pz, _i64(m_per_pair),
                                     rt.ctypes.data_as(C.POINTER(C.c_float)), C.c_void_p(idx.data_ptr()),
                                     C.c_void_p(d2.data_ptr()), C.c_void_p(fb.data_ptr()), _stream()),
              "vicp_nns_batched")
        return idx[:m], d2[:m], fb

    def nns_noalloc(self, p: torch.Tensor, Rt, nn_idx: torch.Tensor, nn_d2: torch.Tensor,
                    n_fallback: torch.Tensor = None):
        """The search of ``nns`` into caller-allocated outputs (int32[m],
        float32[m], int32[1] or None) through the entry point that allocates
        nothing: its intermediates live in the library's fixed per-GPU
        array, so calls on one GPU must not overlap."""
        p = _soa(p, "p")
        m = p.shape[1]
        rt = np.ascontiguousarray(np.asarray(Rt, np.float32).reshape(12))
        for t, dt in ((nn_idx, torch.int32), (nn_d2, torch.float32)):
            if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dt and t.is_contiguous()
                    and t.numel() >= m):
                raise TypeError("outputs must be contiguous CUDA tensors of m int32 / float32 entries")
        fb = C.c_void_p(n_fallback.data_ptr()) if n_fallback is not None else C.c_void_p(0)
        px, py, pz = _ptrs(p)
        check(lib().vicp_nns_noalloc(self.handle, px, py, pz, m, rt.ctypes.data_as(C.POINTER(C.c_float)),
                                     C.c_void_p(nn_idx.data_ptr()), C.c_void_p(nn_d2.data_ptr()), fb, _stream()),
              "vicp_nns_noalloc")

    # -- the ICP loop
    def register(self, p: torch.Tensor, max_iter: int, rmse_eps: float = 1e-5, early_stop: bool = False,
                 use_graph: bool = True, Rt0=None, m_per_pair=None, raise_degenerate: bool = False,
                 global_only: bool = False, layout: str = "segmented", correspondences: bool = False) -> IcpResult:
        """The ICP loop (Sec. II.A); with correspondences=True the result also
        carries the last iteration's correspondences, written by the
        registration's own kernels."""
        return self._register(p, max_iter, rmse_eps, early_stop, use_graph, Rt0, m_per_pair, raise_degenerate,
                              global_only, layout, correspondences)

    def rebuild_register(self, q: torch.Tensor, rings: int, p: torch.Tensor, max_iter: int, **kw) -> IcpResult:
        """rebuild(q), dilate(rings) and register(p, max_iter, **kw) in one
        call, with the same results; the refill's count, scan, scatter and
        order passes share their launches with the source bucketing's."""
        q = _soa(q, "q")
        if q.shape[1] != self.n_total:
            raise ValueError("rebuild needs the same number of target points")
        res = self._register(p, max_iter, refill=(q, int(rings)), **kw)
        self.q = q
        return res

    def _register(self, p, max_iter, rmse_eps=1e-5, early_stop=False, use_graph=True, Rt0=None, m_per_pair=None,
                  raise_degenerate=False, global_only=False, layout="segmented", correspondences=False,
                  refill=None) -> IcpResult:
        p = _soa(p, "p")
        m = p.shape[1]
        B = self.npairs
        if m_per_pair is None:
            if B != 1:
                raise ValueError("m_per_pair is required for a batched grid")
            m_per_pair = [m]
        if sum(m_per_pair) != m:
            raise ValueError("m_per_pair does not add up to the source size")
        if Rt0 is None:
            rt = np.tile(_IDENTITY, B)
        else:
            rt = np.ascontiguousarray(np.asarray(Rt0, np.float64).reshape(B * 12)).copy()
        K = int(max_iter)
        rm, fbk, cnd, dil, stats = self._stats_arrays(B, K)
        if layout not in ("segmented", "direct"):
            raise ValueError("layout must be 'segmented' or 'direct'")
        out_idx = out_d2 = None
        if correspondences:
            out_idx = torch.full((max(m, 1),), -1, dtype=torch.int32, device=p.device)
            out_d2 = torch.full((max(m, 1),), float("nan"), dtype=torch.float32, device=p.device)
        opts = IcpOpts(K, float(rmse_eps), int(bool(early_stop)), int(bool(use_graph)), int(bool(global_only)),
                       int(layout == "direct"), out_idx.data_ptr() if correspondences else None,
                       out_d2.data_ptr() if correspondences else None)
        px, py, pz = _ptrs(p)
        if refill is None:
            name = "vicp_register_batched"
            rc = lib().vicp_register_batched(self.handle, px, py, pz, _i64(m_per_pair), C.byref(opts),
                                             rt.ctypes.data_as(C.POINTER(C.c_double)), stats, _stream())
        else:
            name = "vicp_rebuild_register"
            qx, qy, qz = _ptrs(refill[0])
            rc = lib().vicp_rebuild_register(self.handle, qx, qy, qz, refill[1], px, py, pz, _i64(m_per_pair),
                                             C.byref(opts), rt.ctypes.data_as(C.POINTER(C.c_double)), stats,
                                             _stream())
        allow = () if raise_degenerate else (_lib.ERR_DEGENERATE,)
        check(rc, name, allow)
        iters = np.array([stats[b].iters for b in range(B)])
        deg = np.array([stats[b].degenerate for b in range(B)])
        return IcpResult(rt.reshape(B, 12) if B > 1 else rt, iters, deg,
                         [rm[b, :iters[b]].copy() for b in range(B)],
                         [fbk[b, :iters[b]].copy() for b in range(B)],
                         [cnd[b, :iters[b]].copy() for b in range(B)],
                         [dil[b, :iters[b]].copy() for b in range(B)], rc,
                         out_idx[:m] if correspondences else None, out_d2[:m] if correspondences else None)

    def _stats_arrays(self, B: int, K: int):
        # reused from call to call (a grid serves one thread at a time); the
        # results returned are copies
        if self._stats_key != (B, K):
            arrs = [np.zeros((B, max(K, 1)), dt) for dt in (np.float64, np.int64, np.int64, np.int64)]
            stats = (IcpStats * B)()
            for b in range(B):
                stats[b].rmse = arrs[0][b].ctypes.data_as(C.POINTER(C.c_double))
                stats[b].fallbacks = arrs[1][b].ctypes.data_as(C.POINTER(C.c_int64))
                stats[b].candidates = arrs[2][b].ctypes.data_as(C.POINTER(C.c_int64))
                stats[b].dilated_lookups = arrs[3][b].ctypes.data_as(C.POINTER(C.c_int64))
            self._stats = (*arrs, stats)
            self._stats_key = (B, K)
        return self._stats

    # -- helpers
    def describe(self, pair: int = 0) -> dict:
        d = GridDesc()
        check(lib().vicp_grid_describe(self.handle, int(pair), C.byref(d)), "vicp_grid_describe")
        return {
            "origin": np.array(d.origin[:], np.float32), "inv": np.float32(d.inv), "voxel": np.float32(d.voxel),
            "dims": np.array(d.dims[:], np.int32), "V": d.V, "n": d.n, "pad_rings": d.pad_rings,
            "rings_applied": d.rings_applied, "occupied": d.occupied, "dilated": d.dilated,
            "max_count": d.max_count, "static_bytes": d.static_bytes, "dynamic_bytes": d.dynamic_bytes,
            "vanicp_bytes": d.vanicp_bytes, "extra_bytes": d.extra_bytes,
        }

    def export(self, pair: int = 0):
        """(hist uint32[V], off uint32[V+1] relative to the pair, vm uint32[n+2V]) as numpy arrays."""
        d = self.describe(pair)
        V, n = d["V"], d["n"]
        dev = self.q.device
        hist = torch.empty(V, dtype=torch.int32, device=dev)
        off = torch.empty(V + 1, dtype=torch.int32, device=dev)
        vm = torch.empty(n + 2 * V, dtype=torch.int32, device=dev)
        check(lib().vicp_grid_export(self.handle, int(pair), C.c_void_p(hist.data_ptr()), C.c_void_p(off.data_ptr()),
                                     C.c_void_p(vm.data_ptr()), _stream()), "vicp_grid_export")
        torch.cuda.current_stream().synchronize()
        u = lambda t: t.cpu().numpy().view(np.uint32)
        return u(hist), u(off), u(vm)

    def autotune(self, p: torch.Tensor, m_per_pair=None, searches_per_plan: int = 1):
        """Pick the fastest search schedule for this source (correspondences and
        counts never change; a pose may change in its last bits)."""
        p = _soa(p, "p")
        if m_per_pair is None:
            m_per_pair = [p.shape[1]]
        px, py, pz = _ptrs(p)
        check(lib().vicp_autotune(self.handle, px, py, pz, _i64(m_per_pair), int(searches_per_plan), _stream()),
              "vicp_autotune")
        return self


def build_grid(q: torch.Tensor, voxel: float, pad_rings: int) -> Grid:
    """Alg. 1 + Alg. 2 on one target cloud (3, n) float32 CUDA."""
    q = _soa(q, "q")
    h = C.c_void_p()
    qx, qy, qz = _ptrs(q)
    check(lib().vicp_build_grid(qx, qy, qz, q.shape[1], C.c_float(voxel), int(pad_rings), None, _stream(),
                                C.byref(h)), "vicp_build_grid")
    return Grid(h, q, [q.shape[1]], [voxel], pad_rings)


def build_grid_fixed(q: torch.Tensor, origin, voxel: float, dims, max_rings: int) -> Grid:
    """Alg. 1 + Alg. 2 on a given grid (``dims`` voxels of edge ``voxel`` from
    ``origin``), e.g. 2^N per axis over [-1, 1)^3 for unit-sphere clouds."""
    q = _soa(q, "q")
    o = (C.c_float * 3)(*[float(v) for v in origin])
    d = (C.c_int32 * 3)(*[int(v) for v in dims])
    h = C.c_void_p()
    qx, qy, qz = _ptrs(q)
    check(lib().vicp_build_grid_fixed(qx, qy, qz, q.shape[1], o, C.c_float(voxel), d, int(max_rings), None,
                                      _stream(), C.byref(h)), "vicp_build_grid_fixed")
    return Grid(h, q, [q.shape[1]], [voxel], max_rings)


def build_grid_batched(q: torch.Tensor, n_per_pair, voxels, pad_rings: int) -> Grid:
    """Alg. 1 + Alg. 2 on several targets concatenated along the point axis."""
    q = _soa(q, "q")
    if sum(int(v) for v in n_per_pair) != q.shape[1]:
        raise ValueError("n_per_pair does not add up to the target size")
    B = len(n_per_pair)
    vox = (C.c_float * B)(*[float(v) for v in voxels])
    h = C.c_void_p()
    qx, qy, qz = _ptrs(q)
    check(lib().vicp_build_grid_batched(qx, qy, qz, _i64(n_per_pair), B, vox, int(pad_rings), None, _stream(),
                                        C.byref(h)), "vicp_build_grid_batched")
    return Grid(h, q, n_per_pair, voxels, pad_rings)


def prof_enable(on: bool = True):
    check(lib().vicp_prof_enable(int(on)), "vicp_prof_enable")


def prof_read(kernel: str):
    n = C.c_int64()
    ms = C.c_double()
    check(lib().vicp_prof_read(kernel.encode(), C.byref(n), C.byref(ms)), "vicp_prof_read")
    return n.value, ms.value


def prof_samples(kernel: str):
    """Each launch's milliseconds, in launch order, since the last reset."""
    n = C.c_int64()
    check(lib().vicp_prof_samples(kernel.encode(), None, 0, C.byref(n)), "vicp_prof_samples")
    out = (C.c_double * max(n.value, 1))()
    check(lib().vicp_prof_samples(kernel.encode(), out, n.value, C.byref(n)), "vicp_prof_samples")
    return [out[i] for i in range(n.value)]


def autotune_cache_clear():
    """Forget the schedules the autotuner stored in this process."""
    check(lib().vicp_autotune_cache_clear(), "vicp_autotune_cache_clear")


def prof_reset():
    check(lib().vicp_prof_reset(), "vicp_prof_reset")
