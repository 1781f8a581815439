"""The C-ABI library loads, exports every entry point that include/genga.h declares, and its
host-side argument checks answer without touching a GPU.  CPU only."""
import ctypes
import os
import re

import pytest

import paper_2309_08217_amd as genga

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "genga.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(genga_\w+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    assert set(names) == set(genga.ENTRY_POINTS), names


def test_library_exports_every_declared_symbol():
    lib = genga.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), f"{name} not exported"
        assert ctypes.cast(getattr(lib, name), ctypes.c_void_p).value


def test_host_side_argument_errors_without_gpu():
    lib = genga.load_library()
    assert lib.genga_destroy(None) == genga.GENGA_OK
    assert lib.genga_poll_status(None) == genga.GENGA_ERR_ARG
    assert lib.genga_kick(None, None, 0.1, 1, None) == genga.GENGA_ERR_ARG
    assert b"null context" in lib.genga_last_error()
    assert lib.genga_set_systems(None, 1, None, None, 0) == genga.GENGA_ERR_ARG
    assert lib.genga_set_kick_shape(None, 1, 8, 1) == genga.GENGA_ERR_ARG
    assert lib.genga_create(None, 0) == genga.GENGA_ERR_ARG


def test_python_binding_refuses_cpu_tensors():
    torch = pytest.importorskip("torch")
    with pytest.raises(TypeError):
        genga.Bodies(x=torch.zeros(3, dtype=torch.float64))
