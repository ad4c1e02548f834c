"""Host-side checks that need no GPU: the C-ABI library loads and exports
every entry point include/vicp.h declares, and its pure-host helpers answer."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    txt = open(os.path.join(ROOT, "include", "vicp.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(vicp_\w+)\s*\(", txt, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2512_04996_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return _lib.lib()


def test_header_declares_the_boundary():
    names = declared()
    for must in ("vicp_build_grid", "vicp_dilate", "vicp_nns", "vicp_register"):
        assert must in names
    assert len(names) >= 20


def test_every_declared_symbol_is_exported(lib):
    import subprocess
    from paper_2512_04996_amd import _lib
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (vicp_\w+)", out))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing
    for n in declared():
        assert hasattr(lib, n)
    # the binding declares exactly the header's entry points
    assert set(_lib.SYMBOLS) == set(declared())


def test_host_helpers(lib):
    assert lib.vicp_version().startswith(b"vicp")
    assert lib.vicp_status_str(0) == b"ok"
    assert lib.vicp_status_str(-6) == b"non-finite coordinates"
    assert lib.vicp_status_str(-2) == b"grid too large"


def test_error_codes_match_header():
    from paper_2512_04996_amd import _lib
    txt = open(os.path.join(ROOT, "include", "vicp.h")).read()
    codes = dict((k, int(v)) for k, v in re.findall(r"#define VICP_(\w+) \((-?\d+)\)", txt))
    assert codes["ERR_INVALID_ARG"] == _lib.ERR_INVALID_ARG
    assert codes["ERR_GRID_TOO_LARGE"] == _lib.ERR_GRID_TOO_LARGE
    assert codes["ERR_NONFINITE"] == _lib.ERR_NONFINITE
    assert codes["ERR_DEGENERATE"] == _lib.ERR_DEGENERATE
    assert codes["ERR_STATE"] == _lib.ERR_STATE


def test_product_path_never_imports_the_oracle():
    pkg = os.path.join(ROOT, "paper_2512_04996_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src and "vicp_oracle" not in src, f


def test_missing_library_fails_loudly(monkeypatch):
    # the product path has no CPU fallback: without the HIP library every
    # entry point raises
    from paper_2512_04996_amd import _lib, api
    monkeypatch.setattr(_lib, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libvicp.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.lib()
    # and host tensors are refused, never computed on the CPU
    import torch
    with pytest.raises(TypeError):
        api.build_grid(torch.zeros(3, 8), 0.1, 1)


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout
