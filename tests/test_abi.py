"""CPU checks of the C ABI: the library loads and exports every symbol mf.h declares."""
import os
import re
import subprocess

import paper_2111_03541_amd as mf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "mf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mf_[a-z_]+)\s*\(", src)))


def test_library_loads_and_exports_every_declared_symbol():
    lib = mf.load()
    names = declared_functions()
    assert "mf_pattern" in names and "mf_assemble" in names
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", mf.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (mf_\w+)", out))
    assert set(names) <= exported
    assert set(mf.EXPORTS) == set(names)


def test_version_and_error_string_without_gpu():
    assert "gfx950" in mf.version()
    assert isinstance(mf.load().mf_last_error(), bytes)


def test_argument_errors_are_reported_synchronously():
    import ctypes as C
    lib = mf.load()
    h = C.c_void_p()
    # NULL mesh -> MF_ERR_ARG, no device work
    st = lib.mf_pattern(None, mf.HEX8, 1, None, None, C.byref(h))
    assert st == mf.ERR_ARG and not h.value
    assert b"NULL" in lib.mf_last_error()
    mesh = mf._Mesh(3, 8, 1, None)
    dofs = mf._Dofs(1, None, mf.NODE_MAJOR)
    assert lib.mf_pattern(C.byref(mesh), mf.HEX8, 2, C.byref(dofs), None, C.byref(h)) == mf.ERR_UNSUPPORTED
    assert lib.mf_pattern(C.byref(mesh), mf.QUAD4, 1, C.byref(dofs), None, C.byref(h)) == mf.ERR_ARG
    dofs5 = mf._Dofs(5, None, mf.NODE_MAJOR)
    assert lib.mf_pattern(C.byref(mesh), mf.HEX8, 1, C.byref(dofs5), None, C.byref(h)) == mf.ERR_ARG
    assert lib.mf_assemble(None, None, None, None, None, 0, None, None, None) == mf.ERR_ARG
