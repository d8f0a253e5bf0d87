"""The C-ABI library loads and exports every entry point include/osscir.h declares
(no compute: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "osscir.h")
LIB = os.path.join(ROOT, "paper_1801_06263_amd", "libosscir.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(osscir_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("osscir_forward_project", "osscir_back_project", "osscir_spectral_model",
                     "osscir_block_spc_steps", "osscir_diag_spc_steps", "osscir_mocca_iterate",
                     "osscir_plan_create", "osscir_plan_destroy", "osscir_dtpl"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libosscir.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name
    from paper_1801_06263_amd import osscir
    assert set(osscir.SIGNATURES) == set(declared_functions())


@pytest.mark.skipif(not os.path.exists(LIB), reason="libosscir.so not built")
def test_errors_are_reported_without_a_device():
    from paper_1801_06263_amd import osscir
    lib = osscir.load_library()
    assert lib.osscir_version().decode().startswith("osscir")
    # null plan: EINVAL, message set
    assert lib.osscir_plan_destroy(None) == 0
    rc = lib.osscir_forward_project(None, None, 3, None, None)
    assert rc == -1 and b"plan" in lib.osscir_last_error()
    nb = ctypes.c_size_t()
    assert lib.osscir_workspace_bytes(None, ctypes.byref(nb)) == -1
    assert lib.osscir_batch_workspace_bytes(None, ctypes.byref(nb)) == -1
    # batch entry points: argument errors are reported before any device work
    assert lib.osscir_batch_destroy(None) == 0
    h = ctypes.c_void_p()
    assert lib.osscir_batch_create(None, 4, ctypes.byref(h)) == -1 and not h.value
    assert lib.osscir_batch_iterate(None, 1, 1, None) == -1
    assert lib.osscir_batch_clear_slot(None, 0) == -1
    assert lib.osscir_batch_get_config(None, None) == -1


@pytest.mark.skipif(not os.path.exists(LIB), reason="libosscir.so not built")
def test_spectral_struct_layout_matches_header():
    """The binding's osscir_spectral has the header's fields in order."""
    from paper_1801_06263_amd import osscir
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct \{([^}]*)\} osscir_spectral;", src).group(1)
    names = re.findall(r"\*?\s*(\w+)\s*[,;]", body)
    assert names == [n for n, _ in osscir._Spectral._fields_]
