"""CPU checks of the boundary: the shared library loads and exports every
entry point that include/rhqr.h declares (no compute calls without a GPU),
and the binding refuses to run without the library."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rhqr.h")
LIB = os.path.join(ROOT, "paper_2405_10923_amd", "librhqr.so")


def declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^RHQR_API\s+\w+\s+\**\s*((?:rhqr|recrhqr)_\w+)\s*\(", src, re.M)))


def test_header_declares_the_paper_entry_points():
    names = declared()
    for must in ("rhqr_sketch", "rhqr_factor", "recrhqr_factor", "rhqr_arnoldi_step"):
        assert must in names
    assert len(names) >= 20


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_nothing_else():
    out = os.popen(f"nm -D --defined-only {LIB}").read()
    exported = sorted(set(l.split()[-1] for l in out.splitlines() if " T " in l))
    assert exported == declared()


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2405_10923_amd import rhqr
    monkeypatch.setattr(rhqr, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(rhqr, "_lib", None)
    with pytest.raises(RuntimeError):
        rhqr.lib()
