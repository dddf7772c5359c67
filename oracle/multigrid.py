"""Oracle: geometric multigrid V-cycle on nested structured grids of 8-node hexahedra.

TEST INFRASTRUCTURE ONLY.  Only `tests/`, the smoke check and the benchmark's CPU
baseline leg may import this module; the product library never does.

The paper leaves the linear solve of Sec. 2.2 D-4 open.  Multigrid is the preconditioner
used here for the Krylov solve of the Newton step (Sec. 2.1) when the Jacobi one is not
enough.  What follows is textbook geometric multigrid (Briggs, Henson and McCormick,
"A Multigrid Tutorial"; Trottenberg, Oosterlee and Schueller, "Multigrid"):

- Levels.  Level 0 is the caller's structured grid (node i + (nx+1)(j + (ny+1)k), element
  ex + nx(ey + ny ez), corner a at offsets (a&1, (a>>1)&1, (a>>2)&1)).  Level l+1 has half
  the elements per axis of level l, and its node (i, j, k) is the level-l node (2i, 2j, 2k).
- Coarse operators.  Rediscretisation: the same weak form assembled on the coarse grid.
  Its node coordinates, the linearisation state and the Dirichlet flags are the values at
  the coincident fine nodes (injection).  Boundary forms on element faces (Sec. 4.1-4.3)
  enter every level: a coarse element face is the union of four fine ones, and the fine
  face (element (ex,ey,ez), local face 2 axis + side) stands for the coarse face of
  element (ex/2, ey/2, ez/2) with the same local face when its two in-plane indices are
  even and its index along the axis is even for side 0, odd for side 1; the other fine
  faces drop out.  Nodal targets are injected.  The operator is the domain form plus the
  faces, then the Dirichlet elimination (unit row, zero column).  An element coefficient
  field (conductivity, Young's modulus) is carried to a coarse element as the arithmetic
  mean of its eight children.
- Prolongation P.  Trilinear interpolation of the coarse nodal values, the embedding of the
  coarse Q1 space in the fine one, field by field.  A fine node with an even index along an
  axis takes that axis's coarse node; one with an odd index takes the mean of the two
  coarse neighbours.  Restriction: R = P^T (full weighting).
- Smoother.  Damped Jacobi x <- x + omega D^-1 (b - A x), D = diag A, with D^-1 taken as 0
  where the diagonal is 0.
- V-cycle V(l, b).
  - On the coarsest level: `coarse_sweeps` sweeps from x = 0.
  - Otherwise:
    - start from x = 0 and apply `pre` sweeps;
    - r = b - A x;
    - b_c = R r, with the coarse level's Dirichlet rows set to 0;
    - x += P V(l+1, b_c);
    - apply `post` sweeps.

Pins are in tests/test_oracle_multigrid.py:
- P reproduces trilinear functions exactly.
- R^T = P, and full weighting has the textbook weights.
- On an undistorted grid, P^T A_fine P equals the coarse rediscretisation for mass,
  conduction and elasticity, also with a penalty boundary form on faces.  Nested
  conforming spaces with exact Gauss quadrature fix this (Galerkin identity).
- On a box, the coarsened face list is the coarse box's face list.
- As a stationary iteration, the V-cycle reduces the error of the Q1 conduction problem
  at a grid-independent rate.
"""
from __future__ import annotations

import numpy as np

from . import NODE_MAJOR, Pattern, assemble
from . import boundary as OB


class GridMesh:
    """A structured grid of 8-node hexahedra in the lexicographic numbering above."""

    def __init__(self, dims, coords):
        nx, ny, nz = (int(v) for v in dims)
        self.shape = (nx, ny, nz)
        self.coords = np.ascontiguousarray(coords, dtype=np.float64)
        ex, ey, ez = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
        ex, ey, ez = (v.ravel(order="F") for v in (ex, ey, ez))
        conn = np.empty((8, nx * ny * nz), np.int32)
        for a in range(8):
            i = ex + (a & 1)
            j = ey + ((a >> 1) & 1)
            k = ez + ((a >> 2) & 1)
            conn[a] = i + (nx + 1) * (j + (ny + 1) * k)
        self.conn = conn

    dim = 3
    nen = 8

    @property
    def n_nodes(self):
        return self.coords.shape[1]

    @property
    def n_elems(self):
        return self.conn.shape[1]


def node_ijk(dims):
    """(i, j, k) of every node of a grid with dims elements per axis, in node-id order."""
    nx, ny, nz = dims
    v = np.arange((nx + 1) * (ny + 1) * (nz + 1))
    return v % (nx + 1), (v // (nx + 1)) % (ny + 1), v // ((nx + 1) * (ny + 1))


def injection(fine_dims):
    """Fine node id of every coarse node (coarse node (i,j,k) is fine node (2i,2j,2k))."""
    nx, ny, nz = fine_dims
    cd = (nx // 2, ny // 2, nz // 2)
    i, j, k = node_ijk(cd)
    return (2 * i) + (nx + 1) * ((2 * j) + (ny + 1) * (2 * k))


def dof_index(node, field, n_nodes, nf, numbering):
    return node * nf + field if numbering == NODE_MAJOR else field * n_nodes + node


def prolongation(fine_dims, nf, numbering=NODE_MAJOR):
    """P (scipy CSR, fine rows x coarse rows): trilinear interpolation, field by field."""
    import scipy.sparse as sp
    nx, ny, nz = fine_dims
    cd = (nx // 2, ny // 2, nz // 2)
    nnf = (nx + 1) * (ny + 1) * (nz + 1)
    nnc = (cd[0] + 1) * (cd[1] + 1) * (cd[2] + 1)
    fi, fj, fk = node_ijk(fine_dims)
    rows, cols, vals = [], [], []
    # along one axis: an even index 2m takes coarse node m with weight 1; an odd index 2m+1
    # takes coarse nodes m and m+1 with weight 1/2 each
    def parents(idx):
        out = []
        for side in (0, 1):
            par = (idx + side) // 2
            w = np.where(idx % 2 == 1, 0.5, 1.0 if side == 0 else 0.0)
            out.append((par, w))
        return out
    for px, wx in parents(fi):
        for py, wy in parents(fj):
            for pz, wz in parents(fk):
                w = wx * wy * wz
                keep = w != 0.0
                node_c = px + (cd[0] + 1) * (py + (cd[1] + 1) * pz)
                rows.append(np.nonzero(keep)[0])
                cols.append(node_c[keep])
                vals.append(w[keep])
    P1 = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(nnf, nnc))
    I = sp.identity(nf, format="csr")
    P = sp.kron(P1, I, format="csr") if numbering == NODE_MAJOR else sp.kron(I, P1, format="csr")
    return P


def coarsen_faces(fine_dims, face_elem, face_id):
    """The coarse faces (element ids, local face ids) that the fine faces stand for
    (module docstring), in the order of the fine list."""
    nx, ny, nz = fine_dims
    e = np.asarray(face_elem, np.int64)
    f = np.asarray(face_id, np.int64)
    idx = np.stack([e % nx, (e // nx) % ny, e // (nx * ny)])
    axis, side = f >> 1, f & 1
    keep = np.ones(e.shape, bool)
    for a in range(3):
        normal = axis == a
        keep &= np.where(normal, (idx[a] % 2) == side, (idx[a] % 2) == 0)
    cx, cy = nx // 2, ny // 2
    ce = idx[0] // 2 + cx * (idx[1] // 2 + cy * (idx[2] // 2))
    return ce[keep].astype(np.int32), f[keep].astype(np.uint8)


def coarsen_elem(fine_dims, values):
    """Coarse element (ex,ey,ez): the mean of the fine elements (2ex+a, 2ey+b, 2ez+c)."""
    nx, ny, nz = fine_dims
    v = np.asarray(values, np.float64).reshape(nz, ny, nx)
    kids = [v[c::2, b::2, a::2] for c in (0, 1) for b in (0, 1) for a in (0, 1)]
    return (sum(kids) / 8.0).ravel()


def eliminate(A, mask):
    """Dirichlet elimination of the rows and columns flagged in mask: unit row, zero
    column."""
    import scipy.sparse as sp
    keep = sp.diags((~mask).astype(np.float64))
    return (keep @ A @ keep + sp.diags(mask.astype(np.float64))).tocsr()


def build_levels(fine_dims, coords, nf, kind, params_per_level, n_levels, state=None, dirichlet=None,
                 numbering=NODE_MAJOR, K0=None, face_sets=(), elem_param=None):
    """The level hierarchy: a list of dicts with the grid dims, the coarse mesh, the
    pattern, the operator A (scipy CSR), the Dirichlet flags and D^-1.  Level 0's operator
    is K0 when given (the caller's assembled fine matrix), else the oracle's assembly.
    params_per_level[l]: the form's scalar parameters on level l.  face_sets: boundary
    forms (kind, coef, value, face_elem, face_id, target or None) given on level 0.
    elem_param: the element coefficient field of level 0 (or None)."""
    levels = []
    dims = tuple(int(v) for v in fine_dims)
    crd = np.asarray(coords, np.float64)
    st = None if state is None else np.asarray(state, np.float64)
    msk = None if dirichlet is None else np.asarray(dirichlet, np.uint8)
    faces = [list(fs) for fs in face_sets]
    ep = None if elem_param is None else np.asarray(elem_param, np.float64)
    for l in range(n_levels):
        if l > 0:
            src = injection(dims)
            if ep is not None:
                ep = coarsen_elem(dims, ep)
            nn_f = crd.shape[1]
            for fs in faces:
                fs[3], fs[4] = coarsen_faces(dims, fs[3], fs[4])
                if fs[5] is not None:
                    fs[5] = np.asarray(fs[5])[:, src]
            dims = (dims[0] // 2, dims[1] // 2, dims[2] // 2)
            crd = crd[:, src]
            if st is not None:
                st = st[:, src]
            if msk is not None:
                f = np.arange(nf)
                msk = msk[dof_index(src[:, None], f[None, :], nn_f, nf, numbering)]
                msk = msk.ravel() if numbering == NODE_MAJOR else msk.T.ravel()
        mesh = GridMesh(dims, crd)
        pat = Pattern(mesh, nf, numbering=numbering)
        if l == 0 and K0 is not None:
            A = pat.to_scipy(np.asarray(K0, np.float64))
        elif faces:
            K, _ = assemble(pat, kind, params_per_level[l], state=st, elem_param=ep)
            A = pat.to_scipy(K)
            for bk, coef, value, fe, fi, tg in faces:
                Kb, _ = OB.assemble_boundary(pat, bk, coef, value, fe, fi, state=st, target=tg)
                A = A + Kb
            if msk is not None:
                A = eliminate(A, msk.astype(bool))
        else:
            K, _ = assemble(pat, kind, params_per_level[l], state=st, dirichlet=msk, elem_param=ep)
            A = pat.to_scipy(K)
        diag = A.diagonal()
        dinv = np.where(diag != 0.0, 1.0 / np.where(diag != 0.0, diag, 1.0), 0.0)
        levels.append(dict(dims=dims, mesh=mesh, pattern=pat, A=A.tocsr(), dinv=dinv,
                           mask=None if msk is None else msk.astype(bool),
                           P=None))
    for l in range(n_levels - 1):
        levels[l]["P"] = prolongation(levels[l]["dims"], nf, numbering)
    return levels


def jacobi(A, dinv, b, x, omega, sweeps):
    """`sweeps` damped Jacobi sweeps from x (x = None means x = 0)."""
    for s in range(sweeps):
        if x is None:
            x = omega * dinv * b
        else:
            x = x + omega * dinv * (b - A @ x)
    return np.zeros_like(b) if x is None else x


def vcycle(levels, b, omega=0.5, pre=2, post=2, coarse_sweeps=20, level=0):
    """One V-cycle V(level, b) (module docstring)."""
    lv = levels[level]
    A, dinv = lv["A"], lv["dinv"]
    if level == len(levels) - 1:
        return jacobi(A, dinv, b, None, omega, coarse_sweeps)
    x = jacobi(A, dinv, b, None, omega, pre)
    r = b - A @ x
    bc = lv["P"].T @ r
    cm = levels[level + 1]["mask"]
    if cm is not None:
        bc[cm] = 0.0
    x = x + lv["P"] @ vcycle(levels, bc, omega, pre, post, coarse_sweeps, level + 1)
    return jacobi(A, dinv, b, x, omega, post)
