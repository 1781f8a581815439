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
    assert lib.genga_kick(None, None, 0.1, 1, 0, None) == genga.GENGA_ERR_ARG
    assert lib.genga_encounter_list(None, None, None, 0, None, None) == genga.GENGA_ERR_ARG
    assert lib.genga_drift(None, None, 0.1, None, None, None) == genga.GENGA_ERR_ARG
    assert lib.genga_autotune(None, None, 1, None, None) == genga.GENGA_ERR_ARG
    assert lib.genga_sort_bodies(None, None, None, None) == genga.GENGA_ERR_ARG
    assert b"null context" in lib.genga_last_error()
    assert lib.genga_set_systems(None, 1, None, None, 0) == genga.GENGA_ERR_ARG
    assert lib.genga_set_kick_shape(None, 1, 8, 1) == genga.GENGA_ERR_ARG
    assert lib.genga_create(None, 0) == genga.GENGA_ERR_ARG


def declared_signatures():
    """name -> parameter list of every function the header declares"""
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    out = {}
    for m in re.finditer(r"\b(genga_\w+)\s*\(([^)]*)\)\s*;", src):
        params = [p.strip() for p in m.group(2).split(",") if p.strip() and p.strip() != "void"]
        out[m.group(1)] = params
    return out


def test_binding_argument_lists_match_the_header():
    """The binding declares every C function with the header's number of parameters, and the
    kick path takes the precision and accumulator selectors, the drift a caller's pair list and
    the encounter list the bodies (NULL: the last kick's list)."""
    lib = genga.load_library()
    sigs = declared_signatures()
    for name, params in sigs.items():
        if name == "genga_last_error":
            continue
        assert len(getattr(lib, name).argtypes) == len(params), (name, params)
    assert [p.split()[-1] for p in sigs["genga_accel"]][-3:] == ["prec", "acc", "*stream"]
    assert [p.split()[-1] for p in sigs["genga_kick"]][-3:] == ["prec", "acc", "*stream"]
    assert [p.split()[-1] for p in sigs["genga_step"]][4:6] == ["prec", "acc"]
    assert [p.split()[-1] for p in sigs["genga_drift"]][3:5] == ["*pairs", "*d_count"]
    assert sigs["genga_encounter_list"][1].startswith("const genga_bodies")
    assert [p.split()[-1] for p in sigs["genga_autotune"]][3] == "*cache_path"
    assert genga.GENGA_ACC_FP64 == 0 and genga.GENGA_ACC_KAHAN32 == 1
    src = open(HEADER).read()
    assert "GENGA_ACC_FP64 = 0, GENGA_ACC_KAHAN32 = 1" in src


def test_python_binding_refuses_cpu_tensors():
    torch = pytest.importorskip("torch")
    with pytest.raises(TypeError):
        genga.Bodies(x=torch.zeros(3, dtype=torch.float64))
