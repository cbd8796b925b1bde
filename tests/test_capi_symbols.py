"""The C-ABI library exports every entry point that include/bemfmm.h
declares, and loads in a fresh process (no GPU work is done here)."""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bemfmm.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bemfmm_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def libpath():
    sys.path.insert(0, ROOT)
    from paper_1007_4591_amd import build
    return build.ensure_built()


def test_header_declares_the_boundary():
    names = declared()
    for n in ("bemfmm_build_tree", "bemfmm_fmm_matvec", "bemfmm_solve_bem", "bemfmm_bibee_energy",
              "bemfmm_solvation_energy", "bemfmm_adjoint_grad", "bemfmm_set_charges", "bemfmm_tree_destroy",
              "bemfmm_last_error"):
        assert n in names


def test_exports_every_declared_symbol(libpath):
    out = subprocess.run(["nm", "-D", "--defined-only", libpath], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(\w+)$", out, flags=re.M))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing


def test_loads_in_fresh_process(libpath):
    code = ("import ctypes, sys; lib = ctypes.CDLL(sys.argv[1]); "
            "lib.bemfmm_last_error.restype = ctypes.c_char_p; "
            "assert lib.bemfmm_tree_destroy(None) == 5; print(lib.bemfmm_last_error().decode())")
    r = subprocess.run([sys.executable, "-c", code, libpath], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert "tree" in r.stdout


def test_python_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import paper_1007_4591_amd as B
    monkeypatch.setattr(B._build, "LIB", str(tmp_path / "missing.so"))
    monkeypatch.setattr(B, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        B._load()
