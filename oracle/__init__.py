"""Oracle: plain FP64 CPU finite-element assembly (arXiv 2111.03541, Sec. 2 and Sec. 4).

TEST INFRASTRUCTURE ONLY.  Only `tests/`, the smoke check and the benchmark's CPU
baseline leg may import this package.  The product library never does, and the two
share no code: this wrapper drives `oracle.c`, compiled with gcc, through ctypes.

Every function here marshals numpy arrays; the arithmetic lives in `oracle.c`
(sequential FP64 C, element by element, scattered in element-id order).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MASS, POISSON, ELASTICITY, NS_SUPG = 0, 1, 2, 3
NODE_MAJOR, FIELD_MAJOR = 0, 1
ERR_BAD_JACOBIAN = 2

_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build()
    lib = C.CDLL(_LIB)
    P = C.c_void_p
    i64 = C.c_int64
    lib.or_gauss.argtypes = [C.c_int, P, P]
    lib.or_gauss.restype = C.c_int
    lib.or_basis.argtypes = [C.c_int, P, P, P]
    lib.or_basis.restype = None
    lib.or_pattern_build.argtypes = [C.c_int, i64, i64, P, C.c_int, P, C.c_int]
    lib.or_pattern_build.restype = P
    lib.or_pattern_sizes.argtypes = [P, P, P, P]
    lib.or_pattern_copy.argtypes = [P, P, P, P, P, P]
    lib.or_pattern_free.argtypes = [P]
    lib.or_assemble.argtypes = [P, C.c_int, P, P, P, P, P, P, C.c_int, P, P, P]
    lib.or_assemble.restype = C.c_int
    lib.or_residual.argtypes = [P, C.c_int, P, P, P, P, P, C.c_int, P, P]
    lib.or_residual.restype = C.c_int
    lib.or_assemble_colored.argtypes = [P, C.c_int, P, P, P, P, P, C.c_int, C.c_int, P, P, P, P]
    lib.or_assemble_colored.restype = C.c_int
    lib.or_pcg_jacobi.argtypes = [i64, P, P, P, P, C.c_double, i64, P, P]
    lib.or_pcg_jacobi.restype = i64
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def gauss(p: int):
    lib = _load()
    pts = np.zeros(p)
    wts = np.zeros(p)
    if lib.or_gauss(p, _ptr(pts), _ptr(wts)):
        raise ValueError("unsupported number of Gauss points")
    return pts, wts


def basis(dim: int, xi):
    lib = _load()
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    nen = 1 << dim
    N = np.zeros(nen)
    dN = np.zeros((nen, dim))
    lib.or_basis(dim, _ptr(xi), _ptr(N), _ptr(dN))
    return N, dN


def form_nf(kind: int, dim: int) -> int:
    return dim if kind == ELASTICITY else (dim + 1 if kind == NS_SUPG else 1)


class Pattern:
    """CSR pattern of K: row_ptr (int64), col_idx (int32), rank map, node graph."""

    def __init__(self, mesh, nf: int, coupling=None, numbering: int = NODE_MAJOR):
        lib = _load()
        self.mesh = mesh
        self.nf = nf
        self.numbering = numbering
        conn = np.ascontiguousarray(mesh.conn, dtype=np.int32)
        self._conn = conn
        cpl = None if coupling is None else np.ascontiguousarray(coupling, dtype=np.uint8).reshape(-1)
        h = lib.or_pattern_build(mesh.dim, mesh.n_nodes, mesh.n_elems, _ptr(conn), nf, _ptr(cpl),
                                 numbering)
        if not h:
            raise ValueError("oracle pattern: bad arguments")
        self._h = h
        n_rows = np.zeros(1, np.int64)
        nnz = np.zeros(1, np.int64)
        npairs = np.zeros(1, np.int64)
        lib.or_pattern_sizes(h, _ptr(n_rows), _ptr(nnz), _ptr(npairs))
        self.n_rows, self.nnz, self.n_pairs = int(n_rows[0]), int(nnz[0]), int(npairs[0])
        self.row_ptr = np.zeros(self.n_rows + 1, np.int64)
        self.col_idx = np.zeros(self.nnz, np.int32)
        nen = mesh.nen
        self.rank = np.zeros((nen * nen, mesh.n_elems), np.uint8)
        self.nbr_ptr = np.zeros(mesh.n_nodes + 1, np.int64)
        self.nbr = np.zeros(self.n_pairs, np.int32)
        lib.or_pattern_copy(h, _ptr(self.row_ptr), _ptr(self.col_idx), _ptr(self.rank),
                            _ptr(self.nbr_ptr), _ptr(self.nbr))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.or_pattern_free(h)
            self._h = None

    def to_scipy(self, values):
        import scipy.sparse as sp
        return sp.csr_matrix((values, self.col_idx, self.row_ptr), shape=(self.n_rows, self.n_rows))


def _params(coef=1.0, nu=0.0, rho=0.0, mu=0.0, tau_m=0.0, tau_c=0.0):
    return np.array([coef, nu, rho, mu, tau_m, tau_c], dtype=np.float64)


def _opt(a, dtype=np.float64):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


def assemble(pat: Pattern, kind: int, params=None, elem_param=None, nodal_src=None, state=None,
             dirichlet=None, qpa: int = 2, want_K: bool = True):
    """Return (K values [nnz] or None, d [n_rows]).  Raises on det J <= 0."""
    lib = _load()
    prm = _params(**(params or {}))
    K = np.zeros(pat.nnz) if want_K else None
    d = np.zeros(pat.n_rows)
    bad = np.zeros(1, np.int64)
    ep, ns, st = _opt(elem_param), _opt(nodal_src), _opt(state)
    dm = _opt(dirichlet, np.uint8)
    rc = lib.or_assemble(pat._h, kind, _ptr(prm), _ptr(pat.mesh.coords), _ptr(ep), _ptr(ns), _ptr(st),
                         _ptr(dm), qpa, _ptr(K), _ptr(d), _ptr(bad))
    if rc == ERR_BAD_JACOBIAN:
        raise FloatingPointError(f"det J <= 0 in element {int(bad[0])}")
    if rc:
        raise RuntimeError(f"oracle assemble failed with code {rc}")
    return K, d


def assemble_parallel(pat: Pattern, kind: int, params=None, elem_param=None, nodal_src=None, state=None,
                      qpa: int = 2, threads: int = 1, want_K: bool = True):
    """The same assembly as assemble() without constraints, element colour by element
    colour on `threads` OpenMP threads (the timed CPU baseline).  Returns (K, d, threads
    actually used)."""
    lib = _load()
    prm = _params(**(params or {}))
    K = np.zeros(pat.nnz) if want_K else None
    d = np.zeros(pat.n_rows)
    bad = np.zeros(1, np.int64)
    used = np.zeros(1, np.int32)
    ep, ns, st = _opt(elem_param), _opt(nodal_src), _opt(state)
    rc = lib.or_assemble_colored(pat._h, kind, _ptr(prm), _ptr(pat.mesh.coords), _ptr(ep), _ptr(ns), _ptr(st),
                                 qpa, int(threads), _ptr(K), _ptr(d), _ptr(bad), _ptr(used))
    if rc == ERR_BAD_JACOBIAN:
        raise FloatingPointError(f"det J <= 0 in element {int(bad[0])}")
    if rc:
        raise RuntimeError(f"oracle parallel assemble failed with code {rc}")
    return K, d, int(used[0])


def residual(pat: Pattern, kind: int, params=None, elem_param=None, nodal_src=None, state=None,
             qpa: int = 2):
    lib = _load()
    prm = _params(**(params or {}))
    R = np.zeros(pat.n_rows)
    bad = np.zeros(1, np.int64)
    ep, ns, st = _opt(elem_param), _opt(nodal_src), _opt(state)
    rc = lib.or_residual(pat._h, kind, _ptr(prm), _ptr(pat.mesh.coords), _ptr(ep), _ptr(ns), _ptr(st),
                         qpa, _ptr(R), _ptr(bad))
    if rc == ERR_BAD_JACOBIAN:
        raise FloatingPointError(f"det J <= 0 in element {int(bad[0])}")
    if rc:
        raise RuntimeError(f"oracle residual failed with code {rc}")
    return R


def pcg_jacobi(row_ptr, col_idx, values, b, tol=1e-8, maxit=10000):
    """Jacobi-PCG from x0 = 0; returns (x, iterations or -1, true relative residual)."""
    lib = _load()
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    v = np.ascontiguousarray(values, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    rel = np.zeros(1)
    it = lib.or_pcg_jacobi(b.shape[0], _ptr(rp), _ptr(ci), _ptr(v), _ptr(b), tol, maxit, _ptr(x), _ptr(rel))
    return x, int(it), float(rel[0])
