"""The C-ABI library without a GPU: it loads, exports every symbol the header
declares, and rejects bad arguments before touching the device."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gko.h")
LIB = os.path.join(ROOT, "paper_2011_08879_amd", "libgko_mi355x.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gko_[a-z0-9_]+)\s*\(", text)) - {"gko_alloc_fn", "gko_dealloc_fn"})


@pytest.fixture(scope="module")
def lib():
    import torch  # noqa: F401  (bind to torch's HIP runtime, as the binding does)
    if not os.path.exists(LIB):
        import __graft_entry__
        __graft_entry__._lib_builder().build()
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert len(names) >= 20
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\sT\s(gko_[a-z0-9_]+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        getattr(lib, n)


def test_binding_covers_the_header(lib):
    import paper_2011_08879_amd as g
    assert set(declared()) <= set(g.EXPORTED)


def test_argument_errors_without_device(lib):
    lib.gko_status_string.restype = ctypes.c_char_p
    lib.gko_last_error.restype = ctypes.c_char_p
    assert lib.gko_status_string(0) == b"ok"
    assert lib.gko_status_string(8) == b"matrix not SPD"
    # null output handle: rejected before any HIP call
    assert lib.gko_context_create(None, None) == 1
    assert b"null" in lib.gko_last_error()
    assert lib.gko_matrix_destroy(None) == 0
    assert lib.gko_spmv(None, ctypes.c_double(1.0), None, ctypes.c_double(0.0), None) == 1
    assert lib.gko_convert(None, 0) == 1
    assert lib.gko_cg_solve(None, None, None, ctypes.c_double(1e-10), 10) == 1
    assert lib.gko_matrix_create_csr(None, 0, 0, 0, 0, None, 0, None, None, None) == 1
    assert lib.gko_dot(None, 0, 0, None, None, None) == 1


def test_missing_library_fails_loudly(tmp_path):
    """Importing the binding from a copy without the built library raises."""
    import shutil
    import sys
    pkg = tmp_path / "paper_2011_08879_amd"
    pkg.mkdir()
    shutil.copy(os.path.join(ROOT, "paper_2011_08879_amd", "__init__.py"), pkg / "__init__.py")
    code = "import sys; sys.path.insert(0, %r)\ntry:\n import paper_2011_08879_amd\nexcept ImportError as e:\n print('IMPORTERROR', e)\n" % str(tmp_path)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True).stdout
    assert "IMPORTERROR" in out
