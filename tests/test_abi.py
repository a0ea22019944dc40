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


# ---------------------------------------------------------------- error contract
# Argument errors are returned as -i (i the 1-based position of the offending
# argument) before anything touches the GPU, so they are checked here on the
# CPU.  A fake non-null pointer stands for a device buffer: validation never
# dereferences it.
FAKE = ctypes.c_void_p(0x1000)


def _lib():
    from paper_2405_10923_amd import rhqr
    return rhqr.lib()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_sketch_create_argument_errors():
    L = _lib()
    h = ctypes.c_void_p()
    bh = ctypes.byref(h)
    assert L.rhqr_sketch_create(7, 100, 4, 8, 0, None, 0, None, bh) == -1
    assert L.rhqr_sketch_create(0, 1, 4, 8, 0, None, 0, None, bh) == -2
    assert L.rhqr_sketch_create(0, 100, -1, 8, 0, None, 0, None, bh) == -3
    assert L.rhqr_sketch_create(0, 100, 100, 8, 0, None, 0, None, bh) == -3
    assert L.rhqr_sketch_create(0, 100, 4, 0, 0, None, 0, None, bh) == -4
    assert L.rhqr_sketch_create(0, 100, 4, 129, 0, None, 0, None, bh) == -4      # l > N = 128
    assert L.rhqr_sketch_create(0, 1 << 20, 4, 4097, 0, None, 0, None, bh) == -4  # l > 4096
    assert L.rhqr_sketch_create(1, 100, 4, 8, 0, FAKE, 7, None, bh) == -7        # ld_omega < l
    assert L.rhqr_sketch_create(0, 100, 4, 8, 0, None, 0, None, None) == -9
    assert h.value is None


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_null_handle_errors():
    L = _lib()
    assert L.rhqr_sketch_workspace_size(None, 4) == 0
    assert L.rhqr_factor_workspace_size(None, 0, 4) == 0
    assert L.recrhqr_workspace_size(None, 0, 4) == 0
    assert L.rhqr_trim_workspace_size(None, 0, 4) == 0
    assert L.rhqr_trim_factor(None, 0, 100, 4, FAKE, 100, FAKE, 8, FAKE, 4, FAKE, 4, FAKE, 4,
                              None, 0, 0, FAKE, 1 << 20, None) == -1
    assert L.rhqr_sketch(None, 0, 100, 4, FAKE, 100, FAKE, 12, FAKE, 1 << 20, None) == -1
    assert L.rhqr_factor(None, 0, 100, 4, FAKE, 100, FAKE, 12, FAKE, 4, FAKE, 4, None, 0, 0,
                         FAKE, 1 << 20, None) == -1
    assert L.recrhqr_factor(None, 0, 100, 4, FAKE, 100, FAKE, 100, FAKE, 12, FAKE, 4, FAKE, 4,
                            None, 0, 0, FAKE, 1 << 20, None) == -1
    info = ctypes.c_int32()
    assert L.rhqr_status(None, None, ctypes.byref(info)) == -1
    assert L.rhqr_status(FAKE, None, None) == -3
    assert L.rhqr_sketch_destroy(None) == -1
    a = ctypes.c_void_p()
    assert L.rhqr_arnoldi_create(None, 0, 100, 4, None, ctypes.byref(a)) == -1
    assert L.rhqr_arnoldi_destroy(None) == -1
    assert L.rhqr_arnoldi_start(None, FAKE, FAKE, None, None) == -1
    assert L.rhqr_arnoldi_step(None, FAKE, FAKE, FAKE, None) == -1
    assert L.rhqr_arnoldi_solution(None, 1, FAKE, FAKE, None) == -1
    assert L.rhqr_arnoldi_basis(None, None, None, None) == -1


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_spmv_colscale_profile_argument_errors():
    L = _lib()
    assert L.rhqr_spmv_csr(9, 10, FAKE, FAKE, FAKE, FAKE, FAKE, None) == -1
    assert L.rhqr_spmv_csr(0, 0, FAKE, FAKE, FAKE, FAKE, FAKE, None) == -2
    assert L.rhqr_spmv_csr(0, 10, None, FAKE, FAKE, FAKE, FAKE, None) == -3
    assert L.rhqr_spmv_csr(0, 10, FAKE, None, FAKE, FAKE, FAKE, None) == -4
    assert L.rhqr_spmv_csr(0, 10, FAKE, FAKE, None, FAKE, FAKE, None) == -5
    assert L.rhqr_spmv_csr(0, 10, FAKE, FAKE, FAKE, None, FAKE, None) == -6
    assert L.rhqr_spmv_csr(0, 10, FAKE, FAKE, FAKE, FAKE, None, None) == -7
    assert L.rhqr_colscale(4, 10, 2, FAKE, 10, FAKE, 10, FAKE, None) == -1
    assert L.rhqr_colscale(0, 0, 2, FAKE, 10, FAKE, 10, FAKE, None) == -2
    assert L.rhqr_colscale(0, 10, 0, FAKE, 10, FAKE, 10, FAKE, None) == -3
    assert L.rhqr_colscale(0, 10, 2, None, 10, FAKE, 10, FAKE, None) == -4
    assert L.rhqr_colscale(0, 10, 2, FAKE, 9, FAKE, 10, FAKE, None) == -5
    assert L.rhqr_colscale(0, 10, 2, FAKE, 10, None, 10, FAKE, None) == -6
    assert L.rhqr_colscale(0, 10, 2, FAKE, 10, FAKE, 9, FAKE, None) == -7
    assert L.rhqr_colscale(0, 10, 2, FAKE, 10, FAKE, 10, None, None) == -8
    assert L.rhqr_scale_r(0, FAKE, 4, FAKE, None) == -1
    assert L.rhqr_scale_r(4, None, 4, FAKE, None) == -2
    assert L.rhqr_scale_r(4, FAKE, 3, FAKE, None) == -3
    assert L.rhqr_scale_r(4, FAKE, 4, None, None) == -4
    ncls = 11  # RHQR_PROF_NCLASS
    ms = (ctypes.c_double * (ncls + 1))()
    cnt = (ctypes.c_int64 * (ncls + 1))()
    assert L.rhqr_profile_end(-1, ms, cnt) == -1
    assert L.rhqr_profile_end(ncls + 1, ms, cnt) == -1
    assert L.rhqr_profile_end(2, None, cnt) == -2
    assert L.rhqr_profile_end(2, ms, None) == -3
    assert L.rhqr_profile_begin() == 0
    assert L.rhqr_profile_end(ncls, ms, cnt) == 0   # an empty window
    assert list(cnt) == [0] * (ncls + 1)


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_batch_argument_errors():
    from paper_2405_10923_amd import rhqr
    L = _lib()
    b = ctypes.c_void_p()
    assert L.rhqr_batch_workspace_size(None, 1, 0) == 0
    assert L.rhqr_batch_create(None, 1, 0, 0, FAKE, 1 << 20, None, ctypes.byref(b)) == -1
    arr = (rhqr._Problem * 1)()
    assert L.rhqr_batch_create(arr, 0, 0, 0, FAKE, 1 << 20, None, ctypes.byref(b)) == -2
    assert L.rhqr_batch_create(arr, 1, 0, 0, FAKE, 1 << 20, None, ctypes.byref(b)) == -1  # null sketch
    assert L.rhqr_batch_factor(None, 0, None) == -1
    assert L.rhqr_batch_status(None, None, None) == -1
    assert L.rhqr_batch_thin_q(None, None, None, None) == -1
    assert L.rhqr_batch_destroy(None) == -1
