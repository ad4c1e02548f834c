"""ctypes declarations of libvicp.so (the C ABI in include/vicp.h).

Loading fails loudly when the library has not been built: there is no
fallback implementation of any kernel in Python.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvicp.so")

OK = 0
ERR_INVALID_ARG = -1
ERR_GRID_TOO_LARGE = -2
ERR_OOM = -3
ERR_HIP = -4
ERR_STATE = -5
ERR_NONFINITE = -6
ERR_DEGENERATE = -7
MASK_BIT = 0x80000000
NOALLOC_MAX_QUERIES = 1 << 20


class VicpError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: {msg} (code {code})")
        self.code = code


class GridDesc(C.Structure):
    _fields_ = [
        ("origin", C.c_float * 3), ("inv", C.c_float), ("voxel", C.c_float), ("dims", C.c_int32 * 3),
        ("V", C.c_int64), ("n", C.c_int64), ("pad_rings", C.c_int32), ("rings_applied", C.c_int32),
        ("occupied", C.c_int64), ("dilated", C.c_int64), ("max_count", C.c_uint32),
        ("static_bytes", C.c_int64), ("dynamic_bytes", C.c_int64), ("vanicp_bytes", C.c_int64),
        ("extra_bytes", C.c_int64),
    ]


class IcpOpts(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("rmse_eps", C.c_double), ("early_stop", C.c_int32),
                ("use_graph", C.c_int32), ("global_only", C.c_int32), ("layout", C.c_int32),
                ("nn_idx", C.c_void_p), ("nn_d2", C.c_void_p)]


class IcpStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("degenerate", C.c_int32), ("rmse", C.POINTER(C.c_double)),
                ("fallbacks", C.POINTER(C.c_int64)), ("candidates", C.POINTER(C.c_int64)),
                ("dilated_lookups", C.POINTER(C.c_int64))]


SYMBOLS = {
    "vicp_build_grid": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_float, C.c_int32, C.c_void_p,
                                  C.c_void_p, C.POINTER(C.c_void_p)]),
    "vicp_build_grid_batched": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_int64), C.c_int32,
                                          C.POINTER(C.c_float), C.c_int32, C.c_void_p, C.c_void_p,
                                          C.POINTER(C.c_void_p)]),
    "vicp_build_grid_fixed": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(C.c_float),
                                        C.c_float, C.POINTER(C.c_int32), C.c_int32, C.c_void_p, C.c_void_p,
                                        C.POINTER(C.c_void_p)]),
    "vicp_grid_rebuild": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "vicp_set_build_options": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    "vicp_dilate": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    "vicp_direct_build": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p]),
    "vicp_direct_free": (C.c_int, [C.c_void_p]),
    "vicp_nns": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(C.c_float),
                           C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "vicp_nns_batched": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_int64),
                                   C.POINTER(C.c_float), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "vicp_nns_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(C.c_float),
                                   C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "vicp_register": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(IcpOpts),
                                C.POINTER(C.c_double), C.POINTER(IcpStats), C.c_void_p]),
    "vicp_register_batched": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_int64),
                                        C.POINTER(IcpOpts), C.POINTER(C.c_double), C.POINTER(IcpStats), C.c_void_p]),
    "vicp_rebuild_register": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.POINTER(C.c_int64), C.POINTER(IcpOpts),
                                        C.POINTER(C.c_double), C.POINTER(IcpStats), C.c_void_p]),
    "vicp_p2p_loss_fwd": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_int64),
                                    C.c_void_p, C.c_void_p, C.c_void_p]),
    "vicp_p2p_loss_bwd": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_int64),
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_void_p]),
    "vicp_grid_npairs": (C.c_int, [C.c_void_p]),
    "vicp_grid_describe": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(GridDesc)]),
    "vicp_grid_export": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "vicp_grid_free": (C.c_int, [C.c_void_p]),
    "vicp_autotune": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_int64), C.c_int32,
                                C.c_void_p]),
    "vicp_get_schedule": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "vicp_set_schedule": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    "vicp_get_build_schedule": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                          C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "vicp_set_build_schedule": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    "vicp_autotune_cache_clear": (C.c_int, []),
    "vicp_prof_enable": (C.c_int, [C.c_int32]),
    "vicp_prof_samples": (C.c_int, [C.c_char_p, C.POINTER(C.c_double), C.c_int64, C.POINTER(C.c_int64)]),
    "vicp_prof_read": (C.c_int, [C.c_char_p, C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
    "vicp_prof_reset": (C.c_int, []),
    "vicp_status_str": (C.c_char_p, [C.c_int]),
    "vicp_last_error": (C.c_char_p, []),
    "vicp_version": (C.c_char_p, []),
}

_lib = None


def lib():
    """The loaded library; raises ImportError when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libvicp.so is not built ({LIB_PATH}); run "
                              "`python -m paper_2512_04996_amd.build` or __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SYMBOLS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(rc: int, where: str, allow=()):
    if rc != OK and rc not in allow:
        msg = lib().vicp_last_error().decode(errors="replace")
        raise VicpError(rc, where, msg)
    return rc
