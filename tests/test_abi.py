"""Host-side checks of the C ABI: the library loads and exports every
function that include/flr.h declares, and the header and the binding agree.
No compute calls (these run without a GPU)."""
import ctypes
import os
import re

import paper_1306_1970_amd as flr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "flr.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(flr_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("flr_create", "flr_solve", "flr_solve_ex", "flr_solve_grid", "flr_server_submit",
                 "flr_server_poll"):
        assert must in names


def test_library_exports_every_declared_symbol():
    L = flr.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
        assert isinstance(getattr(L, name), ctypes._CFuncPtr)


def test_binding_lists_every_declared_symbol():
    assert sorted(flr.EXPORTS) == declared_functions()


def test_status_strings_without_gpu():
    assert flr.status_name(flr.FLR_OK) == "ok"
    assert "argument" in flr.status_name(flr.FLR_ERR_INVALID_ARG)


def test_struct_layouts_match_header():
    # flr_solve_opts: 2 doubles, 4 int32, a pointer, 2 int32 -> 48 bytes; flr_result: 4 doubles + int64 + 2 int32
    assert ctypes.sizeof(flr.flr_solve_opts) == 48
    assert ctypes.sizeof(flr.flr_result) == 48
    o = flr.default_opts()
    assert o.eps == 1e-8 and o.max_iter == 0 and o.precision == flr.FLR_PREC_FP64


def test_every_export_declares_argtypes():
    # a function called without argtypes gets its pointer arguments truncated to C int
    lib = flr.lib()
    for name in flr.EXPORTS:
        if name in ("flr_last_error",):
            continue
        assert getattr(lib, name).argtypes is not None, name
