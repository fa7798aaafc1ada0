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


def test_null_handles_rejected(lib):
    """Every call that takes a handle rejects a null one with INVALID_ARG and a
    message, before any device work; destroying a null handle is a no-op."""
    d, f = ctypes.c_double, ctypes.c_float
    calls = {
        "gko_context_destroy": (None,),
        "gko_context_set_stream": (None, None),
        "gko_context_set_allocator": (None, None, None, None),
        "gko_matrix_clone": (None, None),
        "gko_matrix_describe": (None, None),
        "gko_matrix_export_csr": (None, None, None, None),
        "gko_matrix_export_storage": (None, None, None, None, None, None),
        "gko_matrix_export_sellp": (None, None, None, None, None),
        "gko_spmv": (None, d(1.0), None, d(0.0), None),
        "gko_convert": (None, 0),
        "gko_dot": (None, 0, 0, None, None, None),
        "gko_norm2": (None, 0, 0, None, None),
        "gko_stream": (None, 0, 0, None, None, d(1.0), None),
        "gko_gather_probe": (None, 0, None, 1, None, None),
        "gko_context_set_solver_opts": (None, None),
        "gko_context_get_solver_opts": (None, None),
        "gko_context_get_solve_info": (None, None),
        "gko_cg_solve": (None, None, None, d(1e-10), 10),
        "gko_cg_solve_noalloc": (None, None, None, d(1e-10), 10),
        "gko_fcg_solve": (None, None, None, d(1e-10), 10),
        "gko_pipecg_solve": (None, None, None, d(1e-10), 10),
        "gko_bicgstab_solve": (None, None, None, d(1e-10), 10),
        "gko_cgs_solve": (None, None, None, d(1e-10), 10),
        "gko_gmres_solve": (None, None, None, d(1e-10), 10),
        "gko_batch_create_csr": (None, 0, None, None, None, None, None, 0, None),
        "gko_batch_cg_solve": (None, None, None, d(1e-10), 10, None, None),
        "gko_batch_set_block": (None, 256),
        "gko_batch_get_block": (None, None),
        "gko_batch_autotune": (None, None, None, d(1e-10), 10, None, None, None, None),
        "gko_batch_launch_info": (None, None, None),
        "gko_batch_set_lds_mode": (None, 0),
        "gko_batch_get_lds_mode": (None, None),
        "gko_matrix_features": (None, None),
        "gko_autotune_format": (None, None, None),
        "gko_mlp_create": (None, None, None),
        "gko_mlp_get_params": (None, None, None),
        "gko_mlp_fit_normalization": (None, 0, None),
        "gko_mlp_forward": (None, 0, None, None),
        "gko_mlp_loss_grad": (None, 0, None, None, None, None, None),
        "gko_mlp_train": (None, 0, None, None, None, 1, f(1e-3), None),
        "gko_mlp_save": (None, b"/nonexistent"),
        "gko_mlp_load": (None, b"/nonexistent", None),
        "gko_select_format": (None, None, None, None),
        "gko_context_set_selector": (None, None),
    }
    lib.gko_last_error.restype = ctypes.c_char_p
    for name, args in calls.items():
        st = getattr(lib, name)(*args)
        if name == "gko_context_destroy":
            assert st == 0, name
            continue
        assert st == 1, (name, st)
        assert lib.gko_last_error(), name
    for name in ("gko_batch_destroy", "gko_mlp_destroy", "gko_matrix_destroy"):
        assert getattr(lib, name)(None) == 0, name
    handled = set(calls) | {"gko_batch_destroy", "gko_mlp_destroy", "gko_matrix_destroy",
                            "gko_context_create", "gko_matrix_create_csr", "gko_status_string",
                            "gko_last_error"}
    assert set(declared()) <= handled, sorted(set(declared()) - handled)


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


def test_binding_checks_vectors_before_the_library(lib):
    """The C-ABI sees bare pointers, so the binding rejects host tensors, wrong
    element types and short outputs before any library call."""
    import torch
    import paper_2011_08879_amd as g
    x = torch.zeros(8, dtype=torch.float64)
    idx = torch.zeros(8, dtype=torch.int32)
    with pytest.raises(ValueError, match="CUDA"):
        g.gather_probe(x, idx, x)                      # host tensors
    with pytest.raises(ValueError, match="CUDA"):
        g.stream(g.STREAM_COPY, x, x)
    with pytest.raises(ValueError):
        g.dot(x, x)
    with pytest.raises(ValueError):
        g.norm2(x)
    with pytest.raises(ValueError, match="required"):
        g._vec(None, 1, torch.float64, "y")
    # the element-type and length checks, on a stand-in for a contiguous device tensor
    class Dev:
        def __init__(self, n, dtype):
            self.is_cuda, self.dtype, self._n = True, dtype, n

        def is_contiguous(self):
            return True

        def numel(self):
            return self._n
    with pytest.raises(TypeError):
        g._vec(Dev(8, torch.float32), 8, torch.float64, "x")
    with pytest.raises(ValueError, match="at least 9"):
        g._vec(Dev(8, torch.float64), 9, torch.float64, "y")
    g._vec(Dev(9, torch.float64), 9, torch.float64, "y")
