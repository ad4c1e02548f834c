"""Dilation-based ICP with segmented, offset-addressed dilation memory on
AMD Instinct MI355X (gfx950): the method of Chang, Wang, Zhong and Miyazaki,
arXiv 2512.04996, as hand-written HIP kernels behind the C ABI of
include/vicp.h, with a thin torch binding.

Submodules load lazily so that ``paper_2512_04996_amd.synth`` (input
generation) imports without the built library.
"""
import importlib

__all__ = ["build_grid", "build_grid_batched", "build_grid_fixed", "Grid", "p2p_loss", "P2PLoss", "prof_enable", "prof_read",
           "prof_reset", "synth", "VicpError"]

_LAZY = {
    "build_grid": "api", "build_grid_batched": "api", "build_grid_fixed": "api", "Grid": "api", "prof_enable": "api", "prof_read": "api",
    "prof_reset": "api", "p2p_loss": "autograd", "P2PLoss": "autograd", "VicpError": "_lib",
}


def __getattr__(name):
    if name in _LAZY:
        mod = importlib.import_module(f".{_LAZY[name]}", __name__)
        return getattr(mod, name)
    if name == "synth":
        return importlib.import_module(".synth", __name__)
    raise AttributeError(name)
