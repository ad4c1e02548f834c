"""ctypes front end of the CPU oracle (``vicp_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg are its only users.  It never imports the GPU
package, and the GPU package never imports it.

All inputs are numpy arrays; coordinates are float32 structure-of-arrays of
shape (3, k).  Each function names the part of the paper it follows; the C
file carries the details and the readings of the paper.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "vicp_oracle.c")
LIB = os.path.join(HERE, "libvicp_oracle.so")

OK, ERR_ARG, ERR_TOO_LARGE, ERR_OOM, ERR_NONFINITE, ERR_INTERNAL = 0, -1, -2, -3, -4, -5
MASK_BIT = 0x80000000


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: oracle error {code}")
        self.code = code


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no contraction, so float32 rounds as written)."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.run(cmd, check=True, cwd=HERE)
        os.replace(LIB + ".tmp", LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        f32p, f64p = C.POINTER(C.c_float), C.POINTER(C.c_double)
        u32p, i32p, i64p = C.POINTER(C.c_uint32), C.POINTER(C.c_int32), C.POINTER(C.c_int64)
        i64, i32 = C.c_int64, C.c_int32
        L.vicpo_set_threads.argtypes = [i32]
        L.vicpo_set_threads.restype = C.c_int
        L.vicpo_grid_spec.argtypes = [f32p, f32p, f32p, i64, C.c_float, i32, f32p, f32p, i32p, i64p]
        L.vicpo_voxel_ids.argtypes = [f32p, f32p, f32p, i64, f32p, C.c_float, i32p, i64p]
        L.vicpo_build.argtypes = [f32p, f32p, f32p, i64, f32p, C.c_float, i32p, i64, u32p, u32p, u32p]
        L.vicpo_dilate.argtypes = [i32p, i64, u32p, u32p, i32, u32p, u32p]
        L.vicpo_nns.argtypes = [f32p, f32p, f32p, i64, f32p, C.c_float, i32p, u32p, u32p,
                                f32p, f32p, f32p, i64, f32p, i32p, f32p, i64p, i64p, i64p]
        L.vicpo_nns_cap.argtypes = [f32p, f32p, f32p, i64, f32p, C.c_float, i32p, u32p, u32p,
                                    f32p, f32p, f32p, i64, f32p, i64, i32p, f32p, i64p, i64p, i64p]
        L.vicpo_solve.argtypes = [f32p, f32p, f32p, f32p, f32p, f32p, i32p, i64, f64p, f64p, f64p, i32p]
        L.vicpo_register.argtypes = [f32p, f32p, f32p, i64, f32p, f32p, f32p, i64, C.c_float, i32, i32,
                                     C.c_double, i32, f64p, f64p, i64p, i32p, i32p, i32p, f32p]
        L.vicpo_register_spec.argtypes = [f32p, f32p, f32p, i64, f32p, f32p, f32p, i64, f32p, C.c_float, i32p, i64,
                                          i32, i32, C.c_double, i32, f64p, f64p, i64p, i32p, i32p, i32p, f32p]
        L.vicpo_register_cap.argtypes = [f32p, f32p, f32p, i64, f32p, f32p, f32p, i64, f32p, C.c_float, i32p, i64,
                                         i32, i64, i32, C.c_double, i32, f64p, f64p, i64p, i32p, i32p, i32p, f32p]
        L.vicpo_se3_exp.argtypes = [f64p, f64p, f64p, f64p]
        L.vicpo_se3_exp.restype = None
        L.vicpo_p2p_loss_fixed.argtypes = [f32p, f32p, f32p, f64p, f64p, f64p, i64, i32p, f64p]
        L.vicpo_p2p_loss_fixed.restype = C.c_double
        L.vicpo_p2p.argtypes = [f32p, f32p, f32p, i64, f32p, C.c_float, i32p, u32p, u32p,
                                f32p, f32p, f32p, i64, f64p, f64p, f64p, f64p, f64p, f64p, i32p]
        _lib = L
    return _lib


def set_threads(k: int) -> int:
    """Threads of Alg. 4's per-query loop (default 1); returns the count in
    force.  Results do not depend on it."""
    return int(lib().vicpo_set_threads(int(k)))


def _p(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _soa(x: np.ndarray, dtype=np.float32):
    x = np.ascontiguousarray(x, dtype=dtype)
    assert x.ndim == 2 and x.shape[0] == 3, x.shape
    return x


def _rows(x):
    return [np.ascontiguousarray(x[a]) for a in range(3)]


def _check(rc: int, what: str):
    if rc != OK:
        raise OracleError(rc, what)


@dataclass
class Grid:
    """Target grid: specification (Sec. II.A Step 1) and segmented memory (Alg. 1-3)."""
    origin: np.ndarray   # (3,) float32
    inv: np.float32
    voxel: np.float32
    dims: np.ndarray     # (3,) int32
    V: int
    n: int
    hist: np.ndarray     # uint32[V]
    off: np.ndarray      # uint32[V+1]
    vm: np.ndarray       # uint32[n+2V]
    roots: np.ndarray | None = None   # uint32[V] after dilation (0xFFFFFFFF = none)


def grid_spec(q: np.ndarray, voxel: float, rings: int):
    """Origin, 1/voxel, dims and V of the target grid padded by ``rings`` voxels."""
    q = _soa(q)
    qx, qy, qz = _rows(q)
    origin = np.zeros(3, np.float32)
    inv = np.zeros(1, np.float32)
    dims = np.zeros(3, np.int32)
    V = np.zeros(1, np.int64)
    rc = lib().vicpo_grid_spec(_p(qx, C.c_float), _p(qy, C.c_float), _p(qz, C.c_float), q.shape[1],
                               C.c_float(voxel), rings, _p(origin, C.c_float), _p(inv, C.c_float),
                               _p(dims, C.c_int32), _p(V, C.c_int64))
    _check(rc, "grid_spec")
    return origin, inv[0], dims, int(V[0])


def voxel_ids(x: np.ndarray, origin, inv, dims) -> np.ndarray:
    """Linear voxel id of each point, -1 when outside the grid."""
    x = _soa(x)
    xs = _rows(x)
    out = np.zeros(x.shape[1], np.int64)
    lib().vicpo_voxel_ids(*(_p(a, C.c_float) for a in xs), x.shape[1], _p(np.asarray(origin, np.float32), C.c_float),
                          C.c_float(inv), _p(np.asarray(dims, np.int32), C.c_int32), _p(out, C.c_int64))
    return out


def build_grid(q: np.ndarray, voxel: float, rings: int) -> Grid:
    """Counts (Alg. 1 GPU part), offsets (Alg. 1 CPU part) and segments (Alg. 2)."""
    q = _soa(q)
    origin, inv, dims, V = grid_spec(q, voxel, rings)
    n = q.shape[1]
    hist = np.zeros(V, np.uint32)
    off = np.zeros(V + 1, np.uint32)
    vm = np.zeros(n + 2 * V, np.uint32)
    qx, qy, qz = _rows(q)
    rc = lib().vicpo_build(_p(qx, C.c_float), _p(qy, C.c_float), _p(qz, C.c_float), n,
                           _p(origin, C.c_float), C.c_float(inv), _p(dims, C.c_int32), V,
                           _p(hist, C.c_uint32), _p(off, C.c_uint32), _p(vm, C.c_uint32))
    _check(rc, "build")
    return Grid(origin, np.float32(inv), np.float32(voxel), dims, V, n, hist, off, vm)


def fixed_spec(origin, voxel: float, dims):
    """A given grid (not the target's padded box): origin and dims as given,
    1/voxel rounded once to float32 as for every grid."""
    origin = np.ascontiguousarray(origin, np.float32).reshape(3)
    dims = np.ascontiguousarray(dims, np.int32).reshape(3)
    inv = np.float32(1.0) / np.float32(voxel)
    return origin, inv, dims, int(np.prod(dims.astype(np.int64)))


def build_grid_fixed(q: np.ndarray, origin, voxel: float, dims) -> Grid:
    """build_grid on a given grid, e.g. the 2^N voxels per axis over the unit
    sphere's cube of Sec. IV.A.  Every target point must lie inside it."""
    q = _soa(q)
    origin, inv, dims, V = fixed_spec(origin, voxel, dims)
    n = q.shape[1]
    hist = np.zeros(V, np.uint32)
    off = np.zeros(V + 1, np.uint32)
    vm = np.zeros(n + 2 * V, np.uint32)
    qx, qy, qz = _rows(q)
    rc = lib().vicpo_build(_p(qx, C.c_float), _p(qy, C.c_float), _p(qz, C.c_float), n,
                           _p(origin, C.c_float), C.c_float(inv), _p(dims, C.c_int32), V,
                           _p(hist, C.c_uint32), _p(off, C.c_uint32), _p(vm, C.c_uint32))
    if rc == -5:   # VICPO_ERR_INTERNAL: a target point outside the given grid
        raise ValueError("a target point lies outside the given grid")
    _check(rc, "build")
    return Grid(origin, inv, np.float32(voxel), dims, V, n, hist, off, vm)


def dilate(g: Grid, rings: int) -> Grid:
    """L synchronous dilation rings (Alg. 3), in place on ``g.vm``."""
    roots = np.zeros(g.V, np.uint32)
    rc = lib().vicpo_dilate(_p(g.dims, C.c_int32), g.V, _p(g.hist, C.c_uint32), _p(g.off, C.c_uint32),
                            rings, _p(g.vm, C.c_uint32), _p(roots, C.c_uint32))
    _check(rc, "dilate")
    g.roots = roots
    return g


def nns(g: Grid, q: np.ndarray, p: np.ndarray, Rt: np.ndarray, capacity: int = 0):
    """Alg. 4 for every source point; ``Rt`` = float32 row-major R then t.
    ``capacity`` > 0: VANICP's per-voxel block capacity (see direct_capacity);
    a query whose points would not fit one block takes the global search.

    Returns (idx int32[m], d2 float32[m], n_fallback, candidates_total).
    """
    idx, d2, F, Ct, _ = _nns(g, q, p, Rt, capacity)
    return idx, d2, F, Ct


def nns_counts(g: Grid, q: np.ndarray, p: np.ndarray, Rt: np.ndarray, capacity: int = 0):
    """Counts of one Alg. 4 pass: (queries sent to the global search,
    candidates scanned by the local searches, queries resolved through a
    dilated voxel, i.e. one whose count word holds Mask(root))."""
    q, p = _soa(q), _soa(p)
    _, _, F, Ct, Dl = _nns(g, q, p, Rt, capacity)
    return F, Ct - F * q.shape[1], Dl


def _nns(g: Grid, q: np.ndarray, p: np.ndarray, Rt: np.ndarray, capacity: int = 0):
    q, p = _soa(q), _soa(p)
    Rt = np.ascontiguousarray(Rt, np.float32).reshape(12)
    m = p.shape[1]
    idx = np.zeros(max(m, 1), np.int32)
    d2 = np.zeros(max(m, 1), np.float32)
    F = np.zeros(1, np.int64)
    Ct = np.zeros(1, np.int64)
    Dl = np.zeros(1, np.int64)
    qs, ps = _rows(q), _rows(p)
    rc = lib().vicpo_nns_cap(*(_p(a, C.c_float) for a in qs), q.shape[1], _p(g.origin, C.c_float),
                             C.c_float(g.inv), _p(g.dims, C.c_int32), _p(g.off, C.c_uint32), _p(g.vm, C.c_uint32),
                             *(_p(a, C.c_float) for a in ps), m, _p(Rt, C.c_float), int(capacity),
                             _p(idx, C.c_int32), _p(d2, C.c_float), _p(F, C.c_int64), _p(Ct, C.c_int64),
                             _p(Dl, C.c_int64))
    _check(rc, "nns")
    return idx[:m], d2[:m], int(F[0]), int(Ct[0]), int(Dl[0])


def solve(p: np.ndarray, q: np.ndarray, idx: np.ndarray, Rt_prev=None):
    """Least-squares rigid transform of Eq. 1 for pairs (p_i, q_idx[i]).

    Returns (Rt float64[12], singular values of the cross-covariance, degenerate).
    """
    p, q = _soa(p), _soa(q)
    idx = np.ascontiguousarray(idx, np.int32)
    prev = np.ascontiguousarray(Rt_prev if Rt_prev is not None else identity_rt(), np.float64).reshape(12)
    out = np.zeros(12, np.float64)
    sv = np.zeros(3, np.float64)
    deg = np.zeros(1, np.int32)
    ps, qs = _rows(p), _rows(q)
    rc = lib().vicpo_solve(*(_p(a, C.c_float) for a in ps), *(_p(a, C.c_float) for a in qs), _p(idx, C.c_int32),
                           p.shape[1], _p(prev, C.c_double), _p(out, C.c_double), _p(sv, C.c_double),
                           _p(deg, C.c_int32))
    _check(rc, "solve")
    return out, sv, bool(deg[0])


def identity_rt() -> np.ndarray:
    return np.array([1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0], np.float64)


@dataclass
class IcpResult:
    Rt: np.ndarray        # float64[12]
    rmse: np.ndarray      # float64[iters]
    fallbacks: np.ndarray  # int64[iters]
    degenerate: np.ndarray  # int32[iters]
    iters: int
    nn_idx: np.ndarray    # int32[m] of the last iteration
    nn_d2: np.ndarray     # float32[m] of the last iteration


def register(q, p, voxel: float, rings: int, iters: int, rmse_eps: float = 1e-5,
             early_stop: bool = False, Rt0=None) -> IcpResult:
    """Full dilation-based ICP (grid, dilation, then NNS + solve per iteration)."""
    q, p = _soa(q), _soa(p)
    Rt = np.ascontiguousarray(Rt0 if Rt0 is not None else identity_rt(), np.float64).reshape(12).copy()
    K = max(iters, 1)
    rmse = np.zeros(K, np.float64)
    fb = np.zeros(K, np.int64)
    deg = np.zeros(K, np.int32)
    done = np.zeros(1, np.int32)
    m = p.shape[1]
    idx = np.zeros(max(m, 1), np.int32)
    d2 = np.zeros(max(m, 1), np.float32)
    qs, ps = _rows(q), _rows(p)
    rc = lib().vicpo_register(*(_p(a, C.c_float) for a in qs), q.shape[1], *(_p(a, C.c_float) for a in ps), m,
                              C.c_float(voxel), rings, iters, C.c_double(rmse_eps), int(early_stop),
                              _p(Rt, C.c_double), _p(rmse, C.c_double), _p(fb, C.c_int64), _p(done, C.c_int32),
                              _p(deg, C.c_int32), _p(idx, C.c_int32), _p(d2, C.c_float))
    _check(rc, "register")
    k = int(done[0])
    return IcpResult(Rt, rmse[:k], fb[:k], deg[:k], k, idx[:m], d2[:m])


def register_fixed(q, p, origin, voxel: float, dims, rings: int, iters: int, rmse_eps: float = 1e-5,
                   early_stop: bool = False, Rt0=None, block_bytes: int = 0) -> IcpResult:
    """register on a given grid (see build_grid_fixed); ``block_bytes`` > 0
    adds VANICP's per-voxel block capacity (see register_direct)."""
    q, p = _soa(q), _soa(p)
    origin, inv, dims, V = fixed_spec(origin, voxel, dims)
    Rt = np.ascontiguousarray(Rt0 if Rt0 is not None else identity_rt(), np.float64).reshape(12).copy()
    K = max(iters, 1)
    rmse = np.zeros(K, np.float64)
    fb = np.zeros(K, np.int64)
    deg = np.zeros(K, np.int32)
    done = np.zeros(1, np.int32)
    m = p.shape[1]
    idx = np.zeros(max(m, 1), np.int32)
    d2 = np.zeros(max(m, 1), np.float32)
    qs, ps = _rows(q), _rows(p)
    rc = lib().vicpo_register_cap(*(_p(a, C.c_float) for a in qs), q.shape[1], *(_p(a, C.c_float) for a in ps), m,
                                  _p(origin, C.c_float), C.c_float(inv), _p(dims, C.c_int32), V, rings,
                                  direct_capacity(block_bytes), iters, C.c_double(rmse_eps), int(early_stop),
                                  _p(Rt, C.c_double), _p(rmse, C.c_double), _p(fb, C.c_int64), _p(done, C.c_int32),
                                  _p(deg, C.c_int32), _p(idx, C.c_int32), _p(d2, C.c_float))
    _check(rc, "register")
    k = int(done[0])
    return IcpResult(Rt, rmse[:k], fb[:k], deg[:k], k, idx[:m], d2[:m])


# A block record is three float32 coordinates and the point index.
RECORD_BYTES = 16


def direct_capacity(block_bytes: int) -> int:
    """Points one voxel's block holds in VANICP's layout (a fixed memory
    block per voxel, Sec. II.B; 64 KiB there, so 4096 points)."""
    return int(block_bytes) // RECORD_BYTES


def register_direct(q, p, voxel: float, rings: int, iters: int, block_bytes: int = 65536,
                    rmse_eps: float = 1e-5, early_stop: bool = False, Rt0=None) -> IcpResult:
    """register with VANICP's per-voxel block capacity: a query whose voxel,
    or whose dilated voxel's root, holds more points than one block does
    takes the global search (Sec. IV.B)."""
    q, p = _soa(q), _soa(p)
    origin, inv, dims, V = grid_spec(q, voxel, rings)
    Rt = np.ascontiguousarray(Rt0 if Rt0 is not None else identity_rt(), np.float64).reshape(12).copy()
    K = max(iters, 1)
    rmse = np.zeros(K, np.float64)
    fb = np.zeros(K, np.int64)
    deg = np.zeros(K, np.int32)
    done = np.zeros(1, np.int32)
    m = p.shape[1]
    idx = np.zeros(max(m, 1), np.int32)
    d2 = np.zeros(max(m, 1), np.float32)
    qs, ps = _rows(q), _rows(p)
    rc = lib().vicpo_register_cap(*(_p(a, C.c_float) for a in qs), q.shape[1], *(_p(a, C.c_float) for a in ps), m,
                                  _p(origin, C.c_float), C.c_float(inv), _p(dims, C.c_int32), V, rings,
                                  direct_capacity(block_bytes), iters, C.c_double(rmse_eps), int(early_stop),
                                  _p(Rt, C.c_double), _p(rmse, C.c_double), _p(fb, C.c_int64), _p(done, C.c_int32),
                                  _p(deg, C.c_int32), _p(idx, C.c_int32), _p(d2, C.c_float))
    _check(rc, "register")
    k = int(done[0])
    return IcpResult(Rt, rmse[:k], fb[:k], deg[:k], k, idx[:m], d2[:m])


def register_global(q, p, iters: int, rmse_eps: float = 1e-5, early_stop: bool = False, Rt0=None) -> IcpResult:
    """ICP with the exact global search for every query, the exhaustive-NNS
    ("Brute") comparator of Table 2: the loop of register with Alg. 4 given
    a one-voxel grid that no point reaches, so every query takes the exact
    global search (same float32 distance, lowest index on ties)."""
    q, p = _soa(q), _soa(p)
    n, m = q.shape[1], p.shape[1]
    far = np.float32(1e30)
    g = Grid(np.array([far, far, far], np.float32), np.float32(1.0), np.float32(1.0), np.ones(3, np.int32), 1, n,
             np.zeros(1, np.uint32), np.array([0, 2], np.uint32), np.zeros(n + 2, np.uint32))
    Rt = np.ascontiguousarray(Rt0 if Rt0 is not None else identity_rt(), np.float64).reshape(12).copy()
    rmse, fb, deg = [], [], []
    idx = np.zeros(0, np.int32)
    d2 = np.zeros(0, np.float32)
    prev = 0.0
    for k in range(iters):
        idx, d2, F, _ = nns(g, q, p, Rt.astype(np.float32))
        acc = 0.0
        for v in d2.astype(np.float64):   # sequential, as the C loop
            acc += v
        r = math.sqrt(acc / m)
        Rt, _, dg = solve(p, q, idx, Rt)
        rmse.append(r)
        fb.append(F)
        deg.append(int(dg))
        if early_stop and k >= 1 and abs(r - prev) < rmse_eps:
            break
        prev = r
    k = len(rmse)
    return IcpResult(Rt, np.array(rmse), np.array(fb, np.int64), np.array(deg, np.int32), k, idx, d2)


def se3_exp(xi):
    """SE(3) exponential of xi = (rho, phi): (R (3,3), t (3,), 6x6 left Jacobian)."""
    xi = np.ascontiguousarray(xi, np.float64).reshape(6)
    R = np.zeros(9)
    t = np.zeros(3)
    J = np.zeros(36)
    lib().vicpo_se3_exp(_p(xi, C.c_double), _p(R, C.c_double), _p(t, C.c_double), _p(J, C.c_double))
    return R.reshape(3, 3), t, J.reshape(6, 6)


def p2p_loss_fixed(q, p64: np.ndarray, idx: np.ndarray, xi) -> float:
    """(1/m) sum |T(xi) p_i - q_idx[i]|^2 in float64, correspondences given."""
    q = _soa(q)
    p64 = np.ascontiguousarray(p64, np.float64)
    idx = np.ascontiguousarray(idx, np.int32)
    xi = np.ascontiguousarray(xi, np.float64).reshape(6)
    qs = _rows(q)
    pr = [np.ascontiguousarray(p64[a]) for a in range(3)]
    return float(lib().vicpo_p2p_loss_fixed(*(_p(a, C.c_float) for a in qs), *(_p(a, C.c_double) for a in pr),
                                            p64.shape[1], _p(idx, C.c_int32), _p(xi, C.c_double)))


def p2p(g: Grid, q, p, xi):
    """Point-to-point loss at pose xi, correspondences from Alg. 4 at the
    float32-rounded pose, and its float64 gradients.

    Returns (loss, dP (3, m) float64, dxi (6,) float64, idx int32[m]).
    """
    q, p = _soa(q), _soa(p)
    xi = np.ascontiguousarray(xi, np.float64).reshape(6)
    m = p.shape[1]
    dp = [np.zeros(max(m, 1)) for _ in range(3)]
    dxi = np.zeros(6)
    loss = np.zeros(1)
    idx = np.zeros(max(m, 1), np.int32)
    qs, ps = _rows(q), _rows(p)
    rc = lib().vicpo_p2p(*(_p(a, C.c_float) for a in qs), q.shape[1], _p(g.origin, C.c_float), C.c_float(g.inv),
                         _p(g.dims, C.c_int32), _p(g.off, C.c_uint32), _p(g.vm, C.c_uint32),
                         *(_p(a, C.c_float) for a in ps), m, _p(xi, C.c_double), _p(loss, C.c_double),
                         *(_p(a, C.c_double) for a in dp), _p(dxi, C.c_double), _p(idx, C.c_int32))
    _check(rc, "p2p")
    return float(loss[0]), np.stack([a[:m] for a in dp]), dxi, idx[:m]


# ----------------------------------------------------------------------------
# memory accounting (Table 1 and its footnote)
# ----------------------------------------------------------------------------

VANICP_BYTES_PER_VOXEL = 64 * 1024   # fixed 64 KB block per voxel (Sec. II.B)


def paper_static_bytes(V: int) -> int:
    """Histogram + address offsets, one 32-bit word each per voxel (Table 1, note 1)."""
    return 2 * 4 * V


def dynamic_bytes(n: int, V: int) -> int:
    """Dilated voxel index: count + 2 words per voxel (Alg. 1 CPU part)."""
    return 4 * (n + 2 * V)


def vanicp_bytes(V: int) -> int:
    """Monolithic per-voxel allocation of the original VANICP (Sec. II.B)."""
    return VANICP_BYTES_PER_VOXEL * V


def saving(ours: float, theirs: float) -> float:
    """Fractional memory saving as Table 1 reports it: 1 - ours / theirs."""
    return 1.0 - ours / theirs
