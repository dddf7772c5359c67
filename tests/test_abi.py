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


def _fake_pattern(n_nodes=8, n_elems=1, dim=3, nf=3, nnz=576):
    """A binding Pattern object without a device handle: the argument checks run before
    any library call, so host tensors and short arrays can be rejected on the CPU."""
    p = mf.Pattern.__new__(mf.Pattern)
    p.dim, p.n_fields, p.numbering = dim, nf, mf.NODE_MAJOR
    p.n_nodes, p.n_elems, p.n_rows, p.nnz = n_nodes, n_elems, n_nodes * nf, nnz
    p.elem, p._h = mf.HEX8, None
    return p


def test_binding_rejects_host_and_short_arrays():
    import pytest
    import torch
    p = _fake_pattern()
    coords = torch.zeros(3 * 8, dtype=torch.float64)  # a host tensor
    with pytest.raises(ValueError, match="CUDA"):
        p.assemble(mf.Form(mf.ELASTICITY, coef=1.0, nu=0.3), coords)
    with pytest.raises(ValueError, match="CUDA"):
        p.assemble_boundary(mf.BFORM_PENALTY, coords, torch.zeros(2, dtype=torch.int32),
                            torch.zeros(1, dtype=torch.uint8))
    with pytest.raises(ValueError, match="CUDA"):
        mf.ns_newton(p, mf.Form(mf.NS_SUPG), coords, torch.zeros(4 * 8, dtype=torch.float64))
    with pytest.raises(ValueError, match="required"):
        mf._require(None, "coords", torch.float64, 24, optional=False)


def test_binding_require_checks_dtype_layout_and_size():
    import pytest
    import torch

    class FakeCuda:  # stands for a device tensor: only the attributes the check reads
        def __init__(self, t):
            self.t, self.is_cuda, self.dtype = t, True, t.dtype

        def is_contiguous(self):
            return self.t.is_contiguous()

        def numel(self):
            return self.t.numel()

    mf._require(FakeCuda(torch.zeros(6, dtype=torch.int32)), "face_elem", torch.int32, 6)
    with pytest.raises(ValueError, match="elements"):
        mf._require(FakeCuda(torch.zeros(5, dtype=torch.uint8)), "face_id", torch.uint8, 6)
    with pytest.raises(ValueError, match="float64"):
        mf._require(FakeCuda(torch.zeros(6, dtype=torch.float32)), "coords", torch.float64, 6)
    with pytest.raises(ValueError, match="contiguous"):
        mf._require(FakeCuda(torch.zeros(4, 6, dtype=torch.float64).t()), "state", torch.float64, 24)


STRUCTS = {  # binding structure -> C type in mf.h
    "_Mesh": "mf_mesh", "_Dofs": "mf_dofs", "_Form": "mf_form", "_Fields": "mf_fields",
    "_Quad": "mf_quadrature", "_CSR": "mf_csr", "_PcgOpts": "mf_pcg_opts", "_PcgResult": "mf_pcg_result",
    "_TransientOpts": "mf_transient_opts", "_TransientResult": "mf_transient_result", "_BForm": "mf_bform",
    "_BSet": "mf_bset", "_NewtonOpts": "mf_newton_opts", "_NewtonResult": "mf_newton_result",
    "_BatchProblem": "mf_batch_problem", "_MgOpts": "mf_mg_opts",
}


def test_binding_structures_match_the_header_layout(tmp_path):
    """Every ctypes structure of the binding has the size and field offsets of its C type
    (a C probe compiled against include/mf.h prints them)."""
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "mf.h"', "int main(void) {"]
    for py, c in STRUCTS.items():
        lines.append(f'printf("{py} size %zu\\n", sizeof({c}));')
        for name, _ in getattr(mf, py)._fields_:
            lines.append(f'printf("{py} {name} %zu\\n", offsetof({c}, {name}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for py in STRUCTS:
        S = getattr(mf, py)
        assert got[(py, "size")] == C_sizeof(S), py
        for name, _ in S._fields_:
            assert got[(py, name)] == getattr(S, name).offset, (py, name)


def C_sizeof(S):
    import ctypes
    return ctypes.sizeof(S)
