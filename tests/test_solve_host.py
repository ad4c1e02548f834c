"""The GPU path's float64 rigid-transform solve, compiled for the host with
hipcc, against the textbook SVD solution (numpy) on random correspondences,
reflections, planar and far-from-origin clouds, and against the rank test on
degenerate inputs (one target point, exactly collinear targets) and on
nearly collinear targets (refused, or solved with the SVD's objective).  The polar
factor refined from a starting rotation (the previous pose in the ICP loop)
must give the same answer from near, far, identity and non-orthogonal
starts (the last two fall back to the Newton or SVD path)."""
import ctypes as C
import os
import shutil
import subprocess

import numpy as np
import pytest

from bruteforce import kabsch_svd
from paper_2512_04996_amd.synth import random_rotation

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def solve_lib(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("solve") / "libsolve.so")
    cmd = [hipcc, "-x", "hip", "--offload-arch=gfx950", "-O2", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2512_04996_amd", "csrc"),
           os.path.join(HERE, "solve_harness.cpp"), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    L = C.CDLL(out)
    L.vicp_test_kabsch.argtypes = [C.POINTER(C.c_double)] * 3
    L.vicp_test_kabsch_from.argtypes = [C.POINTER(C.c_double)] * 4
    return L


def _p(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def moments(p, q, c):
    pc = p - c[:, None]
    qc = q - c[:, None]
    mom = np.zeros(19)
    mom[0:3] = pc.sum(1)
    mom[3:6] = qc.sum(1)
    mom[6:15] = (pc @ qc.T).reshape(9)
    mom[15] = (pc * pc).sum()
    mom[16] = (qc * qc).sum()
    mom[18] = p.shape[1]
    return mom


def test_solve_matches_svd_and_detects_rank(solve_lib):
    rng = np.random.default_rng(0)
    for trial in range(1600):
        kind = trial % 8
        n = int(rng.integers(3, 300))
        p = rng.standard_normal((3, n)) * rng.uniform(0.01, 10)
        if kind == 1:
            p[2] *= 1e-3
        if kind == 2:
            p[2] = 0
        R = random_rotation(rng.standard_normal(3), rng.uniform(0, np.pi))
        q = R @ p + rng.standard_normal((3, 1)) + rng.standard_normal((3, n)) * rng.uniform(0, 0.5)
        if kind == 3:
            q[0] *= -1                     # mirror image: needs the reflection fix
        if kind == 4:
            q = rng.standard_normal((3, n))
        if kind == 5:
            p, q = p + 100.0, q + 100.0    # far from the origin
        if kind == 6:
            q = np.repeat(rng.standard_normal((3, 1)) * 50, n, 1)   # one target point
        if kind == 7:
            q = np.zeros((3, n))
            q[0] = rng.standard_normal(n) * 5
            q[1], q[2] = 1.25, -7.5         # exactly collinear targets
        p = p.astype(np.float32).astype(np.float64)
        q = q.astype(np.float32).astype(np.float64)
        c = np.round(q.mean(1), 1)
        out = np.zeros(12)
        ok = solve_lib.vicp_test_kabsch(_p(moments(p, q, c)), _p(c), _p(out))
        if kind in (6, 7):
            assert not ok, (trial, kind)
            continue
        assert ok, (trial, kind)
        Rk, tk, _ = kabsch_svd(p, q)
        assert np.abs(out[:9].reshape(3, 3) - Rk).max() < 1e-11, (trial, kind)
        assert np.abs(out[9:] - tk).max() < 1e-11 * max(1.0, np.abs(tk).max()), (trial, kind)


def test_refined_solve_matches_svd_from_any_start(solve_lib):
    rng = np.random.default_rng(1)
    for trial in range(1200):
        kind = trial % 6
        n = int(rng.integers(3, 300))
        p = rng.standard_normal((3, n)) * rng.uniform(0.01, 10)
        if kind == 1:
            p[2] *= 1e-3
        R = random_rotation(rng.standard_normal(3), rng.uniform(0, np.pi))
        q = R @ p + rng.standard_normal((3, 1)) + rng.standard_normal((3, n)) * rng.uniform(0, 0.5)
        if kind == 2:
            q[0] *= -1                     # mirror image: needs the reflection fix
        if kind == 3:
            p, q = p + 100.0, q + 100.0
        p = p.astype(np.float32).astype(np.float64)
        q = q.astype(np.float32).astype(np.float64)
        c = np.round(q.mean(1), 1)
        Rk, tk, _ = kabsch_svd(p, q)
        start = trial % 4
        if start == 0:     # near: within 0.3 rad of the answer
            R0 = random_rotation(rng.standard_normal(3), rng.uniform(0, 0.3)) @ Rk
        elif start == 1:
            R0 = np.eye(3)
        elif start == 2:   # anywhere
            R0 = random_rotation(rng.standard_normal(3), rng.uniform(0, np.pi))
        else:              # not orthogonal: the refinement must refuse it
            R0 = Rk + rng.standard_normal((3, 3)) * 1e-6
        out = np.zeros(12)
        ok = solve_lib.vicp_test_kabsch_from(_p(moments(p, q, c)), _p(c), _p(np.ascontiguousarray(R0).reshape(9)),
                                             _p(out))
        assert ok, (trial, kind, start)
        assert np.abs(out[:9].reshape(3, 3) - Rk).max() < 1e-11, (trial, kind, start)
        assert np.abs(out[9:] - tk).max() < 1e-11 * max(1.0, np.abs(tk).max()), (trial, kind, start)


def test_nearly_collinear_targets_refused_or_optimal(solve_lib):
    """Targets on a line up to a transverse spread eps: the rotation about the
    line is then barely determined, so the solve may refuse (rank test) or
    answer; an answer must be a proper rotation whose Eq. 1 objective is the
    SVD solution's (the objective stays well determined when R is not).  A
    spread of 1e-2 of the extent is well conditioned and must be solved."""
    rng = np.random.default_rng(5)
    for trial in range(200):
        eps = [1e-2, 1e-4, 1e-6, 1e-8][trial % 4]
        n = int(rng.integers(8, 200))
        t = rng.standard_normal(n) * 5
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        q = np.outer(d, t) + rng.standard_normal((3, 1)) + rng.standard_normal((3, n)) * (5 * eps)
        R = random_rotation(rng.standard_normal(3), rng.uniform(0, np.pi))
        p = R.T @ (q - rng.standard_normal((3, 1))) + rng.standard_normal((3, n)) * 1e-3
        p = p.astype(np.float32).astype(np.float64)
        q = q.astype(np.float32).astype(np.float64)
        c = np.round(q.mean(1), 1)
        out = np.zeros(12)
        ok = solve_lib.vicp_test_kabsch(_p(moments(p, q, c)), _p(c), _p(out))
        if eps == 1e-2:
            assert ok, trial
        if not ok:
            continue
        Ro, to = out[:9].reshape(3, 3), out[9:]
        assert np.abs(Ro @ Ro.T - np.eye(3)).max() < 1e-12 and np.linalg.det(Ro) > 0, trial
        Rk, tk, _ = kabsch_svd(p, q)
        e_out = float(((Ro @ p + to[:, None] - q) ** 2).sum())
        e_svd = float(((Rk @ p + tk[:, None] - q) ** 2).sum())
        assert e_out <= e_svd * (1 + 1e-9) + 1e-18, (trial, eps, e_out, e_svd)
