"""The C ABI library loads and exports every entry point include/*.h
declares (no compute calls: this runs without a GPU)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))


def declared_functions():
    names = set()
    for h in HEADERS:
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(ugkwp_[a-z_0-9]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_step_api():
    names = declared_functions()
    for required in ("ugkwp_init", "ugkwp_step", "ugkwp_residual", "ugkwp_surface"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_2607_09552_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        pytest.fail("libugkwp.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(pkg.LIB_PATH)
    names = declared_functions()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(pkg.ABI_SYMBOLS) == names


def test_solver_fails_loudly_without_library(tmp_path, monkeypatch):
    import paper_2607_09552_amd as pkg
    monkeypatch.setattr(pkg, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        pkg.load_library(str(tmp_path / "nope.so"))


def test_library_exports_no_other_c_symbols():
    """Only the declared entry points are exported with C linkage."""
    import shutil
    import subprocess
    import paper_2607_09552_amd as pkg
    if shutil.which("nm") is None or not os.path.exists(pkg.LIB_PATH):
        pytest.skip("nm or the library is not available")
    out = subprocess.run(["nm", "-D", "--defined-only", pkg.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    syms = {ln.split()[-1] for ln in out.splitlines() if ln.split() and ln.split()[1] in "TW"}
    c_syms = {x for x in syms if not x.startswith("_")}
    assert c_syms == set(declared_functions()), sorted(c_syms ^ set(declared_functions()))
