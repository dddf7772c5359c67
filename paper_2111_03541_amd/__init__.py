"""Python binding of libmf.so, the MI355X finite-element assembly library (include/mf.h).

Argument marshalling only: torch tensors supply device memory and the HIP stream, and
every step of the path runs in the library's kernels.  There is no fallback: if the
library is missing or fails to load, every call raises.

    import paper_2111_03541_amd as mf
    pat = mf.Pattern(conn, n_nodes, dim=3, n_fields=3)          # conn: int32 cuda [nen][n_el]
    K, d = pat.assemble(mf.Form(mf.ELASTICITY, coef=1.0, nu=0.3), coords, precision=mf.F64,
                        elem_param=E, nodal_src=b)
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmf.so")

# enums of mf.h
OK, ERR_ARG, ERR_UNSUPPORTED, ERR_OVERFLOW, ERR_HIP, ERR_BAD_JACOBIAN, ERR_NONFINITE, \
    ERR_NOT_CONVERGED, ERR_OOM, ERR_BAD_MESH = range(10)
QUAD4, HEX8, HEX20, QUAD8, TET10 = 1, 2, 3, 4, 5
NODE_MAJOR, FIELD_MAJOR = 0, 1
MASS, POISSON, ELASTICITY, NS_SUPG = 0, 1, 2, 3
F64, F32 = 0, 1
SCATTER_AUTO, SCATTER_ATOMIC, SCATTER_GATHER = 0, 1, 2

_STATUS_NAMES = {
    0: "MF_OK", 1: "MF_ERR_ARG", 2: "MF_ERR_UNSUPPORTED", 3: "MF_ERR_OVERFLOW", 4: "MF_ERR_HIP",
    5: "MF_ERR_BAD_JACOBIAN", 6: "MF_ERR_NONFINITE", 7: "MF_ERR_NOT_CONVERGED", 8: "MF_ERR_OOM",
    9: "MF_ERR_BAD_MESH",
}


class MFError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class _Mesh(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_nodes", C.c_int64), ("n_elems", C.c_int64),
                ("conn", C.c_void_p)]


class _Dofs(C.Structure):
    _fields_ = [("n_fields", C.c_int32), ("coupling", C.c_void_p), ("numbering", C.c_int)]


class _Form(C.Structure):
    _fields_ = [("kind", C.c_int), ("coef", C.c_double), ("nu", C.c_double), ("rho", C.c_double),
                ("mu", C.c_double), ("tau_m", C.c_double), ("tau_c", C.c_double)]


class _Fields(C.Structure):
    _fields_ = [("elem_param", C.c_void_p), ("nodal_src", C.c_void_p), ("lin_state", C.c_void_p),
                ("dirichlet", C.c_void_p)]


class _Quad(C.Structure):
    _fields_ = [("points_per_axis", C.c_int32)]


class _CSR(C.Structure):
    _fields_ = [("n_rows", C.c_int64), ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("values", C.c_void_p)]


class _PcgOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxit", C.c_int32), ("check_every", C.c_int32), ("use_graph", C.c_int32),
                ("precond", C.c_int), ("stall_iters", C.c_int32), ("net", C.c_void_p), ("mg", C.c_void_p)]


MG_MAX_LEVELS = 8


class _MgOpts(C.Structure):
    _fields_ = [("max_levels", C.c_int32), ("coarse_rows", C.c_int32), ("pre_sweeps", C.c_int32),
                ("post_sweeps", C.c_int32), ("coarse_sweeps", C.c_int32), ("omega", C.c_double),
                ("tau_m", C.c_double * MG_MAX_LEVELS), ("tau_c", C.c_double * MG_MAX_LEVELS)]


class _PcgResult(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32), ("fallbacks", C.c_int32),
                ("restarts", C.c_int32), ("true_relres", C.c_double)]


PRECOND_NONE, PRECOND_JACOBI, PRECOND_NN, PRECOND_MG = 0, 1, 2, 3

NEWTON_MAX_HISTORY = 64

BFORM_PENALTY, BFORM_CONVECTION, BFORM_RADIATION, BFORM_FLUX, BFORM_TRACTION, BFORM_NS_INFLOW, \
    BFORM_NS_OUTFLOW, BFORM_NS_FIX = range(8)


class _TransientOpts(C.Structure):
    _fields_ = [("dt", C.c_double), ("rho_inf", C.c_double), ("n_steps", C.c_int32), ("init_rate", C.c_int32),
                ("lin_tol", C.c_double), ("lin_maxit", C.c_int32)]


class _TransientResult(C.Structure):
    _fields_ = [("steps", C.c_int32), ("lin_iterations", C.c_int32), ("max_lin_relres", C.c_double)]


class _BForm(C.Structure):
    _fields_ = [("kind", C.c_int), ("coef", C.c_double), ("value", C.c_double * 9)]


class _BSet(C.Structure):
    _fields_ = [("form", _BForm), ("n_faces", C.c_int64), ("face_elem", C.c_void_p), ("face_id", C.c_void_p),
                ("target", C.c_void_p)]


class _NewtonOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol", C.c_double), ("max_steps", C.c_int32), ("lin_tol", C.c_double),
                ("lin_maxit", C.c_int32), ("check_every", C.c_int32), ("use_graph", C.c_int32)]


class _NewtonResult(C.Structure):
    _fields_ = [("steps", C.c_int32), ("converged", C.c_int32), ("lin_iterations", C.c_int32),
                ("res_norm", C.c_double * NEWTON_MAX_HISTORY)]


class _BatchProblem(C.Structure):
    _fields_ = [("pattern", C.c_void_p), ("form", _Form), ("coords", C.c_void_p), ("fields", _Fields),
                ("K", C.c_void_p), ("d", C.c_void_p)]


_lib = None

# every symbol declared in include/mf.h (checked by the ABI test)
EXPORTS = [
    "mf_pattern", "mf_pattern_info", "mf_pattern_grid", "mf_pattern_destroy", "mf_assemble",
    "mf_assemble_ex", "mf_status_poll", "mf_last_error", "mf_version", "mf_pcg",
    "mf_batch_create", "mf_batch_tune", "mf_batch_run", "mf_batch_info", "mf_batch_destroy",
    "mf_nn_create", "mf_nn_params", "mf_nn_set_system", "mf_nn_apply", "mf_nn_train_step", "mf_nn_destroy", "mf_spmv",
    "mf_bicgstab", "mf_ns_newton", "mf_ns_newton_ex", "mf_assemble_boundary", "mf_heat_transient",
    "mf_pcg_noalloc", "mf_pcg_noalloc_max_rows", "mf_nn_checkpoint_size", "mf_nn_save", "mf_nn_load",
    "mf_batch_tiles", "mf_mg_create", "mf_mg_levels", "mf_mg_update", "mf_mg_apply", "mf_mg_destroy",
    "mf_ns_newton_mg", "mf_mg_update_ex", "mf_heat_transient_mg",
]


def load():
    """Load libmf.so (built in-tree by paper_2111_03541_amd.build); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2111_03541_amd.build`")
    try:  # torch first: the library then binds to the HIP runtime torch has loaded, not a second copy
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    P, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
    lib.mf_pattern.argtypes = [C.POINTER(_Mesh), C.c_int, i32, C.POINTER(_Dofs), P, C.POINTER(P)]
    lib.mf_pattern_info.argtypes = [P, C.POINTER(i64), C.POINTER(i64), C.POINTER(P), C.POINTER(P), C.POINTER(P)]
    lib.mf_pattern_grid.argtypes = [P, C.POINTER(i32), C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)]
    lib.mf_pattern_destroy.argtypes = [P]
    lib.mf_pattern_destroy.restype = None
    lib.mf_assemble.argtypes = [P, C.POINTER(_Form), P, C.POINTER(_Fields), C.POINTER(_Quad), C.c_int, P, P, P]
    lib.mf_assemble_ex.argtypes = [P, C.POINTER(_Form), P, C.POINTER(_Fields), C.POINTER(_Quad), C.c_int,
                                   C.c_int, P, P, P]
    lib.mf_status_poll.argtypes = [P, C.POINTER(i64)]
    lib.mf_pcg.argtypes = [C.POINTER(_CSR), P, P, C.POINTER(_PcgOpts), C.POINTER(_PcgResult), P]
    lib.mf_pcg_noalloc.argtypes = [C.POINTER(_CSR), P, P, C.POINTER(_PcgOpts), C.POINTER(_PcgResult), P]
    lib.mf_pcg_noalloc_max_rows.argtypes = []
    lib.mf_pcg_noalloc_max_rows.restype = i64
    lib.mf_nn_checkpoint_size.argtypes = [P, C.POINTER(i64)]
    lib.mf_batch_tiles.argtypes = [P, C.POINTER(i32), P, P, P]
    lib.mf_nn_save.argtypes = [P, P, i64]
    lib.mf_nn_load.argtypes = [P, P, i64]
    lib.mf_batch_create.argtypes = [C.POINTER(_BatchProblem), i32, C.c_int, C.POINTER(P)]
    lib.mf_batch_tune.argtypes = [P, C.c_char_p, P]
    lib.mf_batch_run.argtypes = [P, P]
    lib.mf_batch_info.argtypes = [P, C.POINTER(i64), C.POINTER(i32), C.POINTER(i32), C.POINTER(i32),
                                  C.POINTER(C.c_double)]
    lib.mf_batch_destroy.argtypes = [P]
    lib.mf_batch_destroy.restype = None
    lib.mf_nn_create.argtypes = [P, i32, P, C.c_uint64, C.POINTER(P)]
    lib.mf_nn_params.argtypes = [P, P, P, C.POINTER(i64)]
    lib.mf_nn_set_system.argtypes = [P, C.POINTER(_CSR), P, P]
    lib.mf_nn_apply.argtypes = [P, P, P, P]
    lib.mf_nn_train_step.argtypes = [P, P, P, C.c_double, C.POINTER(C.c_double), P, P]
    lib.mf_spmv.argtypes = [C.POINTER(_CSR), P, P, P]
    lib.mf_heat_transient.argtypes = [P, C.c_double, C.c_double, P, P, P, P, C.POINTER(_Quad),
                                      C.POINTER(_TransientOpts), P, P, C.POINTER(_TransientResult), P]
    lib.mf_heat_transient_mg.argtypes = [P, C.c_double, C.c_double, P, P, P, P, C.POINTER(_MgOpts), C.POINTER(_Quad),
                                         C.POINTER(_TransientOpts), P, P, C.POINTER(_TransientResult), P]
    lib.mf_assemble_boundary.argtypes = [P, C.POINTER(_BForm), P, i64, P, P, P, P, C.c_int, P, P, P]
    lib.mf_bicgstab.argtypes = [C.POINTER(_CSR), P, P, C.POINTER(_PcgOpts), C.POINTER(_PcgResult), P]
    lib.mf_ns_newton.argtypes = [P, C.POINTER(_Form), P, P, P, C.POINTER(_Quad), C.POINTER(_NewtonOpts),
                                 C.POINTER(_NewtonResult), P]
    lib.mf_ns_newton_ex.argtypes = [P, C.POINTER(_Form), P, P, P, C.POINTER(_BSet), C.c_int32, C.POINTER(_Quad),
                                    C.POINTER(_NewtonOpts), C.POINTER(_NewtonResult), P]
    lib.mf_nn_destroy.argtypes = [P]
    lib.mf_nn_destroy.restype = None
    lib.mf_mg_create.argtypes = [P, C.POINTER(_MgOpts), P, C.POINTER(P)]
    lib.mf_mg_levels.argtypes = [P, C.POINTER(i32), P]
    lib.mf_mg_update.argtypes = [P, C.POINTER(_Form), P, C.POINTER(_Fields), C.POINTER(_Quad), P, P]
    lib.mf_mg_apply.argtypes = [P, P, P, P]
    lib.mf_mg_destroy.argtypes = [P]
    lib.mf_mg_destroy.restype = None
    lib.mf_mg_update_ex.argtypes = [P, C.POINTER(_Form), P, C.POINTER(_Fields), C.POINTER(_BSet), C.c_int32,
                                    C.POINTER(_Quad), P, P]
    lib.mf_ns_newton_mg.argtypes = [P, C.POINTER(_Form), P, P, P, C.POINTER(_BSet), C.c_int32, C.POINTER(_MgOpts),
                                    C.POINTER(_Quad), C.POINTER(_NewtonOpts), C.POINTER(_NewtonResult), P]
    lib.mf_last_error.restype = C.c_char_p
    lib.mf_version.restype = C.c_char_p
    _lib = lib
    return lib


def check(status: int):
    if status != OK:
        raise MFError(status, load().mf_last_error().decode())


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _require(t, name, dtype, numel=None, optional=True):
    """Checks a tensor argument before its address reaches the library: on the GPU,
    contiguous, of the dtype and (when given) of the element count.  A host tensor or a
    short array would otherwise reach the kernels as a bad pointer."""
    if t is None:
        if optional:
            return
        raise ValueError(f"{name} is required")
    if not getattr(t, "is_cuda", False):
        raise ValueError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")


def form_fields(kind: int, dim: int) -> int:
    return {MASS: 1, POISSON: 1, ELASTICITY: dim, NS_SUPG: dim + 1}[kind]


class Form:
    def __init__(self, kind: int, coef=1.0, nu=0.0, rho=0.0, mu=0.0, tau_m=0.0, tau_c=0.0):
        self.kind = kind
        self.c = _Form(kind, coef, nu, rho, mu, tau_m, tau_c)


class Pattern:
    """mf_pattern handle.  conn: int32 CUDA tensor [nen][n_elems] (contiguous)."""

    def __init__(self, conn, n_nodes: int, dim: int, n_fields: int, coupling=None,
                 numbering: int = NODE_MAJOR, stream=None, elem: int = None):
        import torch
        lib = load()
        assert conn.is_cuda and conn.dtype == torch.int32 and conn.is_contiguous()
        self.dim, self.n_fields, self.numbering = dim, n_fields, numbering
        self.n_nodes, self.n_elems = int(n_nodes), int(conn.shape[1])
        self._conn = conn
        mesh = _Mesh(dim, self.n_nodes, self.n_elems, conn.data_ptr())
        cpl = None
        if coupling is not None:
            cpl = (C.c_uint8 * (n_fields * n_fields))(*[int(bool(v)) for v in
                                                        __import__("numpy").asarray(coupling).reshape(-1)])
        dofs = _Dofs(n_fields, C.cast(cpl, C.c_void_p) if cpl is not None else None, numbering)
        h = C.c_void_p()
        if elem is None:
            if dim == 3:
                elem = {20: HEX20, 10: TET10}.get(int(conn.shape[0]), HEX8)
            else:
                elem = QUAD8 if conn.shape[0] == 8 else QUAD4
        self.elem = elem
        check(lib.mf_pattern(C.byref(mesh), elem, 2 if elem in (HEX20, QUAD8, TET10) else 1, C.byref(dofs),
                             _stream(stream), C.byref(h)))
        self._h = h
        n_rows, nnz = C.c_int64(), C.c_int64()
        check(lib.mf_pattern_info(h, C.byref(n_rows), C.byref(nnz), None, None, None))
        self.n_rows, self.nnz = n_rows.value, nnz.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.mf_pattern_destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def grid(self):
        g = C.c_int32()
        nx, ny, nz = C.c_int64(), C.c_int64(), C.c_int64()
        check(load().mf_pattern_grid(self._h, C.byref(g), C.byref(nx), C.byref(ny), C.byref(nz)))
        return bool(g.value), (nx.value, ny.value, nz.value)

    def arrays(self):
        """(row_ptr, col_idx, rank) copied to host numpy arrays (sync)."""
        import numpy as np
        import torch
        lib = load()
        rp, ci, rk = C.c_void_p(), C.c_void_p(), C.c_void_p()
        check(lib.mf_pattern_info(self._h, None, None, C.byref(rp), C.byref(ci), C.byref(rk)))
        torch.cuda.synchronize()
        nen = {HEX20: 20, QUAD8: 8, TET10: 10}.get(self.elem, 1 << self.dim)
        out = []
        for ptr, n, dt in ((rp, self.n_rows + 1, np.int32), (ci, self.nnz, np.int32),
                           (rk, nen * nen * self.n_elems, np.uint8)):
            host = np.zeros(max(n, 1), dtype=dt)
            if n > 0:
                _memcpy_d2h(host.ctypes.data, ptr.value, n * host.itemsize)
            out.append(host[:n])
        out[2] = out[2].reshape(nen * nen, self.n_elems)
        return tuple(out)

    def device_arrays(self):
        """Raw device pointers (row_ptr, col_idx, rank), valid while the pattern lives."""
        rp, ci, rk = C.c_void_p(), C.c_void_p(), C.c_void_p()
        check(load().mf_pattern_info(self._h, None, None, C.byref(rp), C.byref(ci), C.byref(rk)))
        return rp.value, ci.value, rk.value

    def assemble(self, form: Form, coords, precision: int = F64, elem_param=None, nodal_src=None,
                 lin_state=None, dirichlet=None, K=None, d=None, scatter: int = SCATTER_AUTO,
                 points_per_axis: int = None, stream=None):
        """Fill K [nnz] and d [n_rows] (allocated here when not given) on the stream."""
        import torch
        lib = load()
        dt = torch.float64 if precision == F64 else torch.float32
        dev = coords.device
        _require(coords, "coords", torch.float64, self.dim * self.n_nodes, optional=False)
        if K is None:
            K = torch.empty(self.nnz, dtype=dt, device=dev)
        if d is None:
            d = torch.empty(self.n_rows, dtype=dt, device=dev)
        _require(K, "K", dt, self.nnz)
        _require(d, "d", dt, self.n_rows)
        _require(elem_param, "elem_param", dt, self.n_elems)
        nsrc = {MASS: 1, POISSON: 1, ELASTICITY: self.dim}.get(form.kind, 0)
        _require(nodal_src, "nodal_src", dt, nsrc * self.n_nodes if nsrc else None)
        _require(lin_state, "lin_state", dt, (self.dim + 1) * self.n_nodes)
        _require(dirichlet, "dirichlet", torch.uint8, self.n_rows)
        f = _Fields(_ptr(elem_param), _ptr(nodal_src), _ptr(lin_state), _ptr(dirichlet))
        q = _Quad(points_per_axis or {HEX20: 3, QUAD8: 3, TET10: 4}.get(self.elem, 2))
        check(lib.mf_assemble_ex(self._h, C.byref(form.c), _ptr(coords), C.byref(f), C.byref(q), precision,
                                 scatter, _ptr(K), _ptr(d), _stream(stream)))
        return K, d

    def assemble_boundary(self, kind: int, coords, face_elem, face_id, coef=1.0, value=(), state=None,
                          target=None, K=None, d=None, precision: int = F64, stream=None):
        """Add the face integrals of a boundary form into K and d (zeros when not given).

        face_elem int32 / face_id uint8 CUDA tensors; value: up to 9 constants (g, T_env,
        the load stress sigma^l row-major, or for the flow forms u^w, rho, mu)."""
        import torch
        lib = load()
        dt = torch.float64 if precision == F64 else torch.float32
        dev = coords.device
        _require(coords, "coords", torch.float64, self.dim * self.n_nodes, optional=False)
        if K is None:
            K = torch.zeros(self.nnz, dtype=dt, device=dev)
        if d is None:
            d = torch.zeros(self.n_rows, dtype=dt, device=dev)
        _require(K, "K", dt, self.nnz)
        _require(d, "d", dt, self.n_rows)
        _require(state, "state", dt, self.n_fields * self.n_nodes)
        _require(target, "target", dt, self.n_fields * self.n_nodes)
        _require(face_elem, "face_elem", torch.int32, optional=False)
        _require(face_id, "face_id", torch.uint8, int(face_elem.shape[0]), optional=False)
        vals = list(value) + [0.0] * (9 - len(value))
        f = _BForm(kind, coef, (C.c_double * 9)(*vals))
        check(lib.mf_assemble_boundary(self._h, C.byref(f), _ptr(coords), int(face_elem.shape[0]), _ptr(face_elem),
                                       _ptr(face_id), _ptr(state), _ptr(target), precision, _ptr(K), _ptr(d),
                                       _stream(stream)))
        return K, d

    def status(self):
        """(status, first bad element or -1) of the last assembly (sync)."""
        bad = C.c_int64()
        st = load().mf_status_poll(self._h, C.byref(bad))
        return st, bad.value


_hip = None


def _memcpy_d2h(dst: int, src: int, nbytes: int):
    """Synchronous device-to-host copy of library-owned arrays (HIP runtime, as loaded by torch)."""
    global _hip
    if _hip is None:
        _hip = C.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        _hip.hipMemcpy.restype = C.c_int
    rc = _hip.hipMemcpy(C.c_void_p(dst), C.c_void_p(src), nbytes, 2)  # hipMemcpyDeviceToHost
    if rc != 0:
        raise MFError(ERR_HIP, f"hipMemcpy failed with {rc}")


class Batch:
    """mf_batch handle: many structured problems assembled by one persistent launch.

    problems: list of dicts with keys pattern (Pattern), form (Form), coords, and optional
    elem_param, nodal_src, dirichlet; K and d are allocated here unless given."""

    def __init__(self, problems, precision: int = F32):
        import torch
        lib = load()
        dt = torch.float64 if precision == F64 else torch.float32
        self.problems = []
        arr = (_BatchProblem * len(problems))()
        for k, pr in enumerate(problems):
            pat = pr["pattern"]
            K = pr.get("K")
            d = pr.get("d")
            dev = pr["coords"].device
            if K is None:
                K = torch.empty(pat.nnz, dtype=dt, device=dev)
            if d is None:
                d = torch.empty(pat.n_rows, dtype=dt, device=dev)
            keep = dict(pr, K=K, d=d)
            self.problems.append(keep)
            arr[k].pattern = pat.handle
            arr[k].form = pr["form"].c
            arr[k].coords = pr["coords"].data_ptr()
            arr[k].fields = _Fields(_ptr(pr.get("elem_param")), _ptr(pr.get("nodal_src")), None,
                                    _ptr(pr.get("dirichlet")))
            arr[k].K = K.data_ptr()
            arr[k].d = d.data_ptr()
        h = C.c_void_p()
        check(lib.mf_batch_create(arr, len(problems), precision, C.byref(h)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.mf_batch_destroy(h)
            self._h = None

    def tune(self, cache_path=None, stream=None):
        check(load().mf_batch_tune(self._h, None if cache_path is None else cache_path.encode(), _stream(stream)))
        return self.info()

    def run(self, stream=None):
        check(load().mf_batch_run(self._h, _stream(stream)))

    def info(self):
        n, wg, order, graphed, us = C.c_int64(), C.c_int32(), C.c_int32(), C.c_int32(), C.c_double()
        check(load().mf_batch_info(self._h, C.byref(n), C.byref(wg), C.byref(order), C.byref(graphed),
                                   C.byref(us)))
        nc = C.c_int32()
        probs, chunks, cross = (C.c_int32 * 8)(), (C.c_int32 * 8)(), (C.c_int32 * 8)()
        check(load().mf_batch_tiles(self._h, C.byref(nc), probs, chunks, cross))
        names = ["poisson", "elasticity"]
        tiles = {f"{names[c // 3]}/bucket{c % 3}": {"problems": probs[c], "chunks": chunks[c],
                                                      "cross_section": f"{cross[c]}x{8 // cross[c]}"}
                 for c in range(nc.value) if probs[c] > 0}
        return {"items": n.value, "workgroups": wg.value, "order": order.value, "graphed": bool(graphed.value),
                "tuned_us": us.value, "tiles": tiles}


class Net:
    """mf_nn handle: the learned multilevel convolution preconditioner on a node grid."""

    def __init__(self, grid, channels, seed: int = 0):
        import numpy as np
        lib = load()
        g = (C.c_int32 * 3)(*[int(v) for v in grid])
        ch = (C.c_int32 * len(channels))(*[int(v) for v in channels])
        h = C.c_void_p()
        check(lib.mf_nn_create(g, len(channels), ch, seed, C.byref(h)))
        self._h = h
        self.grid, self.channels = tuple(grid), list(channels)
        n = C.c_int64()
        check(lib.mf_nn_params(h, None, None, C.byref(n)))
        self.n_params = n.value
        self._np = np
        self._bound = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.mf_nn_destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def get_params(self):
        out = self._np.zeros(self.n_params, self._np.float32)
        check(load().mf_nn_params(self._h, out.ctypes.data_as(C.c_void_p), None, None))
        return out

    def set_params(self, values):
        v = self._np.ascontiguousarray(values, dtype=self._np.float32)
        assert v.size == self.n_params
        check(load().mf_nn_params(self._h, None, v.ctypes.data_as(C.c_void_p), None))

    def set_system(self, row_ptr, col_idx, values, dirichlet=None, stream=None):
        A = _CSR(int(self._np.prod(self.grid)), _ptr_any(row_ptr), _ptr_any(col_idx), _ptr(values))
        check(load().mf_nn_set_system(self._h, C.byref(A), _ptr(dirichlet), _stream(stream)))
        self._bound = (row_ptr, col_idx, values, dirichlet)

    def apply(self, r, z=None, stream=None):
        import torch
        if z is None:
            z = torch.empty_like(r)
        check(load().mf_nn_apply(self._h, _ptr(r), _ptr(z), _stream(stream)))
        return z

    def train_step(self, r, lr, e=None, stream=None):
        loss = C.c_double()
        check(load().mf_nn_train_step(self._h, _ptr(r), _ptr(e), lr, C.byref(loss), None, _stream(stream)))
        return loss.value

    def grad(self, r, e=None, stream=None):
        loss = C.c_double()
        g = self._np.zeros(self.n_params, self._np.float32)
        check(load().mf_nn_train_step(self._h, _ptr(r), _ptr(e), 0.0, C.byref(loss), g.ctypes.data_as(C.c_void_p),
                                      _stream(stream)))
        return loss.value, g

    def save(self, path, trained_with=None):
        """Parameters to path.npy and the architecture (and, when given, how the weights
        were trained) to path.json."""
        import json
        self._np.save(path + ".npy", self.get_params())
        meta = {"grid": self.grid, "channels": self.channels, "n_params": self.n_params}
        if trained_with:
            meta["trained_with"] = trained_with
        with open(path + ".json", "w") as f:
            json.dump(meta, f)

    def load_params(self, path):
        self.set_params(self._np.load(path + ".npy"))

    def checkpoint(self):
        """The training state (mf_nn_save) as bytes."""
        lib = load()
        n = C.c_int64()
        check(lib.mf_nn_checkpoint_size(self._h, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        check(lib.mf_nn_save(self._h, buf, n.value))
        return buf.raw

    def restore(self, data: bytes):
        """Restore a training state made by checkpoint() (mf_nn_load)."""
        buf = C.create_string_buffer(data, len(data))
        check(load().mf_nn_load(self._h, buf, len(data)))

    def save_checkpoint(self, path):
        with open(path, "wb") as f:
            f.write(self.checkpoint())

    def load_checkpoint(self, path):
        with open(path, "rb") as f:
            self.restore(f.read())


def mg_opts(max_levels=0, coarse_rows=0, pre_sweeps=2, post_sweeps=2, coarse_sweeps=20, omega=0.5, tau_m=(),
            tau_c=()):
    """Options of the multigrid cycle (mf_mg_opts); tau_m[l], tau_c[l]: the flow form's
    stabilisation constants on level l (entry 0 unused, 0 = the form's own)."""
    tm = list(tau_m) + [0.0] * (MG_MAX_LEVELS - len(tau_m))
    tc = list(tau_c) + [0.0] * (MG_MAX_LEVELS - len(tau_c))
    return _MgOpts(max_levels, coarse_rows, pre_sweeps, post_sweeps, coarse_sweeps, omega,
                   (C.c_double * MG_MAX_LEVELS)(*tm[:MG_MAX_LEVELS]), (C.c_double * MG_MAX_LEVELS)(*tc[:MG_MAX_LEVELS]))


class Multigrid:
    """Geometric multigrid V-cycle on a structured-grid pattern (mf_mg_t)."""

    def __init__(self, pattern, stream=None, **opts):
        lib = load()
        self.pattern = pattern
        self.opts = mg_opts(**opts)
        h = C.c_void_p()
        check(lib.mf_mg_create(pattern.handle, C.byref(self.opts), _stream(stream), C.byref(h)))
        self.handle = h
        self._K = None

    def levels(self):
        """Element counts per axis of every level, finest first."""
        n = C.c_int32()
        dims = (C.c_int64 * (3 * MG_MAX_LEVELS))()
        check(load().mf_mg_levels(self.handle, C.byref(n), dims))
        return [tuple(dims[3 * l:3 * l + 3]) for l in range(n.value)]

    def update(self, form, coords, K, lin_state=None, dirichlet=None, points_per_axis=2, stream=None, boundary=(),
               elem_param=None):
        """Assemble the coarse levels for the level-0 operator K (kept referenced);
        boundary: face sets as for ns_newton, in K and on every level; elem_param: the
        FP64 element coefficient field K was assembled with."""
        import torch
        p = self.pattern
        _require(coords, "coords", torch.float64, p.dim * p.n_nodes, optional=False)
        _require(K, "K", torch.float64, p.nnz, optional=False)
        _require(lin_state, "lin_state", torch.float64, 4 * p.n_nodes)
        _require(dirichlet, "dirichlet", torch.uint8, p.n_rows)
        _require(elem_param, "elem_param", torch.float64, p.n_elems)
        F = _Fields(_ptr(elem_param), None, _ptr(lin_state), _ptr(dirichlet))
        q = _Quad(points_per_axis)
        sets = _bsets(boundary, p)
        check(load().mf_mg_update_ex(self.handle, C.byref(form.c), _ptr(coords), C.byref(F), sets, len(boundary),
                                     C.byref(q), _ptr(K), _stream(stream)))
        self._K = K
        self._keep = boundary

    def apply(self, r, z=None, stream=None):
        """z = V(0, r), one cycle on the stream."""
        import torch
        _require(r, "r", torch.float64, self.pattern.n_rows, optional=False)
        if z is None:
            z = torch.empty_like(r)
        _require(z, "z", torch.float64, self.pattern.n_rows, optional=False)
        check(load().mf_mg_apply(self.handle, _ptr(r), _ptr(z), _stream(stream)))
        return z

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.mf_mg_destroy(h)
            self.handle = None


def pcg(row_ptr, col_idx, values, b, x=None, tol=1e-8, maxit=20000, precond=PRECOND_JACOBI, net=None,
        check_every=8, use_graph=True, stream=None, raise_on_fail=True, stall_iters=0, mg=None):
    """Solve K x = b (FP64 CSR on the device; row_ptr/col_idx int32) by PCG from x0 = 0.

    Returns (x, result dict).  use_graph needs a non-default stream; with the default
    stream the iterations run eagerly.  stall_iters: iterations without progress that
    restart the solve from the current x (0 = the library default)."""
    import torch
    lib = load()
    n = int(b.shape[0])
    if x is None:
        x = torch.empty(n, dtype=torch.float64, device=b.device)
    A = _CSR(n, _ptr_any(row_ptr), _ptr_any(col_idx), _ptr(values))
    opts = _PcgOpts(tol, maxit, check_every, int(bool(use_graph)), precond, stall_iters,
                    None if net is None else net.handle, None if mg is None else mg.handle)
    res = _PcgResult()
    st = lib.mf_pcg(C.byref(A), _ptr(b), _ptr(x), C.byref(opts), C.byref(res), _stream(stream))
    out = {"iterations": res.iterations, "converged": bool(res.converged), "fallbacks": res.fallbacks,
           "restarts": res.restarts, "true_relres": res.true_relres, "status": st}
    if st != OK and raise_on_fail:
        raise MFError(st, lib.mf_last_error().decode())
    return x, out


def pcg_noalloc(row_ptr, col_idx, values, b, x, tol=1e-8, maxit=20000, precond=PRECOND_JACOBI, check_every=8,
                stream=None, raise_on_fail=True):
    """mf_pcg_noalloc: PCG on the library's fixed device workspace (no device allocation
    in the call; at most noalloc_max_rows() rows; Jacobi or no preconditioner).  x is the
    caller's output vector.  Returns (x, result dict)."""
    import torch
    lib = load()
    n = int(b.shape[0])
    _require(b, "b", torch.float64, optional=False)
    _require(x, "x", torch.float64, n, optional=False)
    A = _CSR(n, _ptr_any(row_ptr), _ptr_any(col_idx), _ptr(values))
    opts = _PcgOpts(tol, maxit, check_every, 0, precond, 0, None, None)
    res = _PcgResult()
    st = lib.mf_pcg_noalloc(C.byref(A), _ptr(b), _ptr(x), C.byref(opts), C.byref(res), _stream(stream))
    out = {"iterations": res.iterations, "converged": bool(res.converged), "fallbacks": res.fallbacks,
           "restarts": res.restarts, "true_relres": res.true_relres, "status": st}
    if st != OK and raise_on_fail:
        raise MFError(st, lib.mf_last_error().decode())
    return x, out


def noalloc_max_rows() -> int:
    return int(load().mf_pcg_noalloc_max_rows())


def bicgstab(row_ptr, col_idx, values, b, x=None, tol=1e-8, maxit=20000, precond=PRECOND_JACOBI,
             check_every=8, use_graph=True, stream=None, raise_on_fail=True, mg=None):
    """Solve K x = b for a non-symmetric FP64 CSR K on the device by BiCGStab from x0 = 0.

    Returns (x, result dict) like pcg."""
    import torch
    lib = load()
    n = int(b.shape[0])
    if x is None:
        x = torch.empty(n, dtype=torch.float64, device=b.device)
    A = _CSR(n, _ptr_any(row_ptr), _ptr_any(col_idx), _ptr(values))
    opts = _PcgOpts(tol, maxit, check_every, int(bool(use_graph)), precond, 0, None,
                    None if mg is None else mg.handle)
    res = _PcgResult()
    st = lib.mf_bicgstab(C.byref(A), _ptr(b), _ptr(x), C.byref(opts), C.byref(res), _stream(stream))
    out = {"iterations": res.iterations, "converged": bool(res.converged), "true_relres": res.true_relres,
           "restarts": res.restarts, "status": st}
    if st != OK and raise_on_fail:
        raise MFError(st, lib.mf_last_error().decode())
    return x, out


def _bsets(boundary, pattern):
    """Face sets (kind, face_elem int32 cuda, face_id uint8 cuda, coef, value, target or None)
    as an mf_bset array."""
    import torch
    sets = (_BSet * max(1, len(boundary)))()
    for k, (kind, fe, fi, coef, value, target) in enumerate(boundary):
        _require(fe, "face_elem", torch.int32, optional=False)
        _require(fi, "face_id", torch.uint8, int(fe.shape[0]), optional=False)
        _require(target, "target", torch.float64, pattern.n_fields * pattern.n_nodes)
        vals = list(value) + [0.0] * (9 - len(value))
        sets[k] = _BSet(_BForm(kind, coef, (C.c_double * 9)(*vals)), int(fe.shape[0]), _ptr(fe), _ptr(fi),
                        _ptr(target))
    return sets


def ns_newton(pattern, form, coords, state, dirichlet=None, rtol=1e-10, atol=0.0, max_steps=20, lin_tol=1e-10,
              lin_maxit=20000, check_every=8, use_graph=True, points_per_axis=2, stream=None, raise_on_fail=True,
              boundary=(), multigrid=None):
    """Newton iteration for the steady flow form; state [4][n_nodes] FP64 (cuda) is updated
    in place.  boundary: face sets (kind, face_elem int32 cuda, face_id uint8 cuda, coef,
    value, target or None) whose boundary forms enter every step before the Dirichlet
    elimination.  multigrid: None (Jacobi-preconditioned solves) or a dict of mg_opts
    arguments (mf_ns_newton_mg, the face sets on every level).  Returns the result dict
    (steps, converged, lin_iterations, res_norm)."""
    import torch
    lib = load()
    _require(state, "state", torch.float64, 4 * pattern.n_nodes, optional=False)
    _require(coords, "coords", torch.float64, pattern.dim * pattern.n_nodes, optional=False)
    _require(dirichlet, "dirichlet", torch.uint8, pattern.n_rows)
    opts = _NewtonOpts(rtol, atol, max_steps, lin_tol, lin_maxit, check_every, int(bool(use_graph)))
    res = _NewtonResult()
    q = _Quad(points_per_axis)
    sets = _bsets(boundary, pattern)
    if multigrid is not None:
        mo = mg_opts(**multigrid)
        st = lib.mf_ns_newton_mg(pattern.handle, C.byref(form.c), _ptr(coords), _ptr(state), _ptr(dirichlet), sets,
                                 len(boundary), C.byref(mo), C.byref(q), C.byref(opts), C.byref(res),
                                 _stream(stream))
    else:
        st = lib.mf_ns_newton_ex(pattern.handle, C.byref(form.c), _ptr(coords), _ptr(state), _ptr(dirichlet), sets,
                                 len(boundary), C.byref(q), C.byref(opts), C.byref(res), _stream(stream))
    out = {"steps": res.steps, "converged": bool(res.converged), "lin_iterations": res.lin_iterations,
           "res_norm": [res.res_norm[k] for k in range(min(res.steps + 1, NEWTON_MAX_HISTORY))], "status": st}
    if st != OK and raise_on_fail:
        raise MFError(st, lib.mf_last_error().decode())
    return out


def heat_transient(pattern, coords, T, Tdot, dt, n_steps, capacity=1.0, conductivity=1.0, elem_k=None, source=None,
                   dirichlet=None, rho_inf=0.5, init_rate=False, lin_tol=1e-12, lin_maxit=20000,
                   points_per_axis=2, stream=None, multigrid=None):
    """Generalized-alpha steps of C dT/dt - div(k grad T) = s; T and Tdot (FP64 cuda,
    [n_nodes]) are updated in place.  multigrid: None (Jacobi-PCG) or a dict of mg_opts
    arguments (mf_heat_transient_mg).  Returns the result dict."""
    import torch
    lib = load()
    _require(coords, "coords", torch.float64, pattern.dim * pattern.n_nodes, optional=False)
    _require(T, "T", torch.float64, pattern.n_nodes, optional=False)
    _require(Tdot, "Tdot", torch.float64, pattern.n_nodes, optional=False)
    _require(elem_k, "elem_k", torch.float64, pattern.n_elems)
    _require(source, "source", torch.float64, pattern.n_nodes)
    _require(dirichlet, "dirichlet", torch.uint8, pattern.n_rows)
    opts = _TransientOpts(dt, rho_inf, n_steps, int(bool(init_rate)), lin_tol, lin_maxit)
    res = _TransientResult()
    q = _Quad(points_per_axis)
    if multigrid is not None:
        mo = mg_opts(**multigrid)
        check(lib.mf_heat_transient_mg(pattern.handle, capacity, conductivity, _ptr(coords), _ptr(elem_k),
                                       _ptr(source), _ptr(dirichlet), C.byref(mo), C.byref(q), C.byref(opts), _ptr(T),
                                       _ptr(Tdot), C.byref(res), _stream(stream)))
    else:
        check(lib.mf_heat_transient(pattern.handle, capacity, conductivity, _ptr(coords), _ptr(elem_k),
                                    _ptr(source), _ptr(dirichlet), C.byref(q), C.byref(opts), _ptr(T), _ptr(Tdot),
                                    C.byref(res), _stream(stream)))
    return {"steps": res.steps, "lin_iterations": res.lin_iterations, "max_lin_relres": res.max_lin_relres}


def spmv(row_ptr, col_idx, values, x, y=None, stream=None):
    """y = K x for an FP64 CSR matrix on the device."""
    import torch
    if y is None:
        y = torch.empty_like(x)
    A = _CSR(int(x.shape[0]), _ptr_any(row_ptr), _ptr_any(col_idx), _ptr(values))
    check(load().mf_spmv(C.byref(A), _ptr(x), _ptr(y), _stream(stream)))
    return y


def _ptr_any(t):
    """A torch tensor or a raw device address (int)."""
    if t is None:
        return None
    return C.c_void_p(t if isinstance(t, int) else t.data_ptr())


def version() -> str:
    return load().mf_version().decode()
