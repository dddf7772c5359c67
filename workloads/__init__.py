"""Seeded synthetic inputs for finite-element assembly: meshes, coefficient fields, sources.

This module holds no finite-element arithmetic. It lays out the node and element
numbering of structured Q1 meshes, draws seeded random numbers and samples smooth
random fields. The HIP path's tests, the oracle's tests and the benchmark all take
their inputs from here, so both sides of every parity check see identical arrays.

Conventions (the paper leaves local node order and numbering open, Sec. 2.2 B-1):
  * node id      = i + (nx+1) * (j + (ny+1) * k)
  * element id   = ex + nx * (ey + ny * ez)
  * local node a = ax + 2*ay + 4*az  maps to node (ex+ax, ey+ay, ez+az)
  * arrays are structure-of-arrays: coords [dim][n_nodes] float64,
    conn [nen][n_elems] int32, nodal fields [n_fields][n_nodes].
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "Mesh", "structured_mesh", "permute_mesh", "lognormal_elem", "uniform_nodal",
    "fourier_velocity", "grf_lognormal_elem", "boundary_node_mask", "dof_mask",
    "batch_problem_sizes",
]


class Mesh:
    """A Q1 mesh in structure-of-arrays form."""

    def __init__(self, coords: np.ndarray, conn: np.ndarray, shape=None):
        self.coords = np.ascontiguousarray(coords, dtype=np.float64)
        self.conn = np.ascontiguousarray(conn, dtype=np.int32)
        self.shape = tuple(shape) if shape is not None else None

    @property
    def dim(self) -> int:
        return self.coords.shape[0]

    @property
    def n_nodes(self) -> int:
        return self.coords.shape[1]

    @property
    def n_elems(self) -> int:
        return self.conn.shape[1]

    @property
    def nen(self) -> int:
        return self.conn.shape[0]


def structured_mesh(n, jitter: float = 0.0, seed=None, lengths=None) -> Mesh:
    """Structured Q1 mesh of the box [0,L_0]x...x[0,L_{dim-1}] with n[d] elements per axis.

    jitter > 0 moves every interior node by an independent U[-jitter*h_d, +jitter*h_d]
    in each coordinate d (boundary nodes stay put, so the domain keeps its volume).
    """
    n = tuple(int(v) for v in n)
    dim = len(n)
    if dim not in (2, 3):
        raise ValueError("dim must be 2 or 3")
    L = np.ones(dim) if lengths is None else np.asarray(lengths, dtype=np.float64)
    npts = [v + 1 for v in n]
    axes = [np.linspace(0.0, L[d], npts[d]) for d in range(dim)]
    # node id = i + (nx+1)(j + (ny+1)k)  ->  meshgrid with 'ij' and Fortran-order ravel
    grids = np.meshgrid(*axes, indexing="ij")
    coords = np.stack([g.ravel(order="F") for g in grids]).astype(np.float64)
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        idx = np.stack(np.meshgrid(*[np.arange(p) for p in npts], indexing="ij"))
        idx = idx.reshape(dim, -1, order="F")
        interior = np.all((idx > 0) & (idx < np.asarray(n)[:, None]), axis=0)
        h = L / np.asarray(n)
        delta = rng.uniform(-1.0, 1.0, size=coords.shape) * (jitter * h)[:, None]
        coords = coords + delta * interior[None, :]
    # element connectivity
    eidx = np.stack(np.meshgrid(*[np.arange(v) for v in n], indexing="ij"))
    eidx = eidx.reshape(dim, -1, order="F")  # element id = ex + nx(ey + ny ez)
    nen = 1 << dim
    conn = np.empty((nen, eidx.shape[1]), dtype=np.int64)
    for a in range(nen):
        bits = [(a >> d) & 1 for d in range(dim)]
        node = np.zeros(eidx.shape[1], dtype=np.int64)
        stride = 1
        for d in range(dim):
            node += (eidx[d] + bits[d]) * stride
            stride *= npts[d]
        conn[a] = node
    return Mesh(coords, conn.astype(np.int32), shape=n)


def permute_mesh(mesh: Mesh, seed) -> tuple[Mesh, np.ndarray, np.ndarray]:
    """Relabel nodes and elements at random (topology and geometry unchanged).

    Returns (new_mesh, node_perm, elem_perm) with new node id = node_perm[old id] and
    new element e' holding old element elem_perm[e'].  The local node order inside each
    element is kept, so every element keeps its orientation.
    """
    rng = np.random.default_rng(seed)
    node_perm = rng.permutation(mesh.n_nodes)
    elem_perm = rng.permutation(mesh.n_elems)
    coords = np.empty_like(mesh.coords)
    coords[:, node_perm] = mesh.coords
    conn = node_perm[mesh.conn[:, elem_perm]].astype(np.int32)
    return Mesh(coords, conn, shape=None), node_perm, elem_perm


def lognormal_elem(n_elems: int, sigma: float, seed) -> np.ndarray:
    """Per-element coefficient exp(N(0, sigma^2))."""
    rng = np.random.default_rng(seed)
    return np.exp(rng.normal(0.0, sigma, size=n_elems)).astype(np.float64)


def uniform_nodal(n_fields: int, n_nodes: int, lo: float, hi: float, seed) -> np.ndarray:
    """Nodal field [n_fields][n_nodes] with entries U[lo, hi]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(n_fields, n_nodes)).astype(np.float64)


def fourier_velocity(coords: np.ndarray, seed, modes: int = 8, kmax: int = 3) -> np.ndarray:
    """Smooth random vector field sampled at the nodes: sum of `modes` Fourier modes.

    a(x) = sum_m A_m sin(2 pi k_m . x + phi_m), k_m integer in {-kmax..kmax}^dim minus 0,
    A_m ~ U[-1,1]^dim, phi_m ~ U[0, 2 pi); then scaled so max over nodes of |a|_2 is 1.
    """
    rng = np.random.default_rng(seed)
    dim = coords.shape[0]
    out = np.zeros_like(coords)
    for _ in range(modes):
        while True:
            k = rng.integers(-kmax, kmax + 1, size=dim)
            if np.any(k != 0):
                break
        A = rng.uniform(-1.0, 1.0, size=dim)
        phi = rng.uniform(0.0, 2.0 * np.pi)
        s = np.sin(2.0 * np.pi * (k @ coords) + phi)
        out += A[:, None] * s[None, :]
    scale = np.max(np.sqrt(np.sum(out * out, axis=0)))
    return out / scale


def grf_lognormal_elem(n, sigma: float, ell: float, seed) -> np.ndarray:
    """Lognormal per-element field exp(sigma * g) on a structured unit-box mesh, with g
    from grf_elem (unit-variance Gaussian field, covariance exp(-r^2 / (2 ell^2)))."""
    return np.exp(sigma * grf_elem(n, ell, seed)).astype(np.float64)


def grf_elem(n, ell: float, seed) -> np.ndarray:
    """Zero-mean, unit-variance Gaussian random field with covariance exp(-r^2/(2 ell^2)),
    sampled at element centroids by circulant embedding on a grid padded to twice the
    mesh in every axis.  Element order follows the structured numbering (x fastest).
    Any unit-norm linear combination of independent draws is again such a field."""
    n = tuple(int(v) for v in n)
    dim = len(n)
    rng = np.random.default_rng(seed)
    h = 1.0 / np.asarray(n, dtype=np.float64)
    m = [2 * v for v in n]
    # periodic distances on the padded grid
    dist2 = np.zeros(m)
    for d in range(dim):
        r = np.arange(m[d])
        r = np.minimum(r, m[d] - r) * h[d]
        shape = [1] * dim
        shape[d] = m[d]
        dist2 = dist2 + (r ** 2).reshape(shape)
    cov = np.exp(-dist2 / (2.0 * ell * ell))
    lam = np.real(np.fft.fftn(cov))
    lam = np.maximum(lam, 0.0)
    noise = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    field = np.fft.ifftn(np.sqrt(lam) * noise) * np.sqrt(np.prod(m))
    g = np.real(field)[tuple(slice(0, v) for v in n)]
    # element id = ex + nx(ey + ny ez): index [ex, ey, ez] raveled in Fortran order
    return g.ravel(order="F").astype(np.float64)


def upsample_nodes(c: np.ndarray) -> np.ndarray:
    """Piecewise-linear upsampling of a node field [nz, ny, nx] to [2nz-1, 2ny-1, 2nx-1]."""
    f = c
    for ax in range(3):
        n = f.shape[ax]
        shp = list(f.shape)
        shp[ax] = 2 * n - 1
        g = np.empty(shp)
        ev = [slice(None)] * 3
        ev[ax] = slice(0, None, 2)
        od = [slice(None)] * 3
        od[ax] = slice(1, None, 2)
        lo = [slice(None)] * 3
        lo[ax] = slice(0, n - 1)
        hi = [slice(None)] * 3
        hi[ax] = slice(1, n)
        g[tuple(ev)] = f
        g[tuple(od)] = 0.5 * (f[tuple(lo)] + f[tuple(hi)])
        f = g
    return f


def multiscale_nodal(n_nodes_axis: int, levels: int, seed) -> np.ndarray:
    """Random node field on an (n x n x n)-node grid with comparable energy at every scale:
    white noise drawn on the grid coarsened 0..levels-1 times, amplitude 2^l at level l,
    upsampled to the fine grid and summed.  Node id = x + n(y + n z)."""
    rng = np.random.default_rng(seed)
    sizes = [n_nodes_axis]
    for _ in range(levels - 1):
        sizes.append((sizes[-1] + 1) // 2)
    out = np.zeros((n_nodes_axis,) * 3)
    for l in range(levels - 1, -1, -1):
        w = rng.standard_normal((sizes[l],) * 3) * (2.0 ** l)
        acc = w if l == levels - 1 else w + acc_up
        acc_up = upsample_nodes(acc) if l > 0 else None
        if l == 0:
            out = acc
    return out.reshape(-1)


def boundary_node_mask(n) -> np.ndarray:
    """uint8 [n_nodes]: 1 for nodes on the boundary of a structured mesh."""
    n = tuple(int(v) for v in n)
    npts = [v + 1 for v in n]
    idx = np.stack(np.meshgrid(*[np.arange(p) for p in npts], indexing="ij"))
    idx = idx.reshape(len(n), -1, order="F")
    on = np.any((idx == 0) | (idx == np.asarray(n)[:, None]), axis=0)
    return on.astype(np.uint8)


def dof_mask(node_mask: np.ndarray, n_fields: int, field_major: bool,
             fields=None) -> np.ndarray:
    """Expand a node mask to a DOF mask for the given numbering.

    node-major dof(a, i) = n_fields * a + i;  field-major dof(a, i) = i * n_nodes + a.
    `fields` restricts the constraint to a subset of field indices (default: all).
    """
    nn = node_mask.shape[0]
    fields = range(n_fields) if fields is None else fields
    m = np.zeros((n_fields, nn), dtype=np.uint8)
    for i in fields:
        m[i] = node_mask
    if field_major:
        return m.reshape(-1).copy()
    return m.T.reshape(-1).copy()


def serendipity_mesh(n, jitter: float = 0.0, seed=None, lengths=None) -> Mesh:
    """Structured box of 20-node serendipity hexahedra, n = (nx, ny, nz) elements.

    Nodes: the (nx+1)(ny+1)(nz+1) corner lattice (lexicographic, as structured_mesh), then
    the midpoints of the x-, y- and z-directed edges, each set lexicographic.  Local
    nodes: 0..7 the corners a = ax + 2 ay + 4 az; 8..11 the x-edges at (y, z) bits
    (0,0), (1,0), (0,1), (1,1); 12..15 the y-edges at (x, z) bits; 16..19 the z-edges at
    (x, y) bits.  Jitter moves interior corners only; every edge midpoint is the midpoint
    of its two corners, so edges stay straight.  Returns a Mesh with nen = 20."""
    nx, ny, nz = (int(v) for v in n)
    base = structured_mesh((nx, ny, nz), jitter=jitter, seed=seed, lengths=lengths)
    X = base.coords
    NX, NY, NZ = nx + 1, ny + 1, nz + 1
    cid = lambda i, j, k: i + NX * (j + NY * k)
    n_c = NX * NY * NZ
    n_ex, n_ey = nx * NY * NZ, NX * ny * NZ
    ex_id = lambda i, j, k: n_c + i + nx * (j + NY * k)
    ey_id = lambda i, j, k: n_c + n_ex + i + NX * (j + ny * k)
    ez_id = lambda i, j, k: n_c + n_ex + n_ey + i + NX * (j + NY * k)
    n_ez = NX * NY * nz
    coords = np.zeros((3, n_c + n_ex + n_ey + n_ez))
    coords[:, :n_c] = X
    for k in range(NZ):
        for j in range(NY):
            for i in range(nx):
                coords[:, ex_id(i, j, k)] = 0.5 * (X[:, cid(i, j, k)] + X[:, cid(i + 1, j, k)])
    for k in range(NZ):
        for j in range(ny):
            for i in range(NX):
                coords[:, ey_id(i, j, k)] = 0.5 * (X[:, cid(i, j, k)] + X[:, cid(i, j + 1, k)])
    for k in range(nz):
        for j in range(NY):
            for i in range(NX):
                coords[:, ez_id(i, j, k)] = 0.5 * (X[:, cid(i, j, k)] + X[:, cid(i, j, k + 1)])
    conn = np.zeros((20, nx * ny * nz), dtype=np.int32)
    for ez in range(nz):
        for ey in range(ny):
            for ex in range(nx):
                e = ex + nx * (ey + ny * ez)
                for a in range(8):
                    conn[a, e] = cid(ex + (a & 1), ey + ((a >> 1) & 1), ez + (a >> 2))
                for m in range(4):
                    b0, b1 = m & 1, m >> 1
                    conn[8 + m, e] = ex_id(ex, ey + b0, ez + b1)
                    conn[12 + m, e] = ey_id(ex + b0, ey, ez + b1)
                    conn[16 + m, e] = ez_id(ex + b0, ey + b1, ez)
    return Mesh(coords, conn)


def serendipity_mesh_2d(n, jitter: float = 0.0, seed=None, lengths=None) -> Mesh:
    """Structured rectangle of 8-node serendipity quadrilaterals, n = (nx, ny) elements.

    Nodes: the (nx+1)(ny+1) corner lattice (lexicographic, as structured_mesh), then the
    midpoints of the x-directed edges, then of the y-directed edges, each set
    lexicographic.  Local nodes: 0..3 the corners a = ax + 2 ay; 4, 5 the x-edges at y
    bit 0, 1; 6, 7 the y-edges at x bit 0, 1.  Jitter moves interior corners only and
    every edge midpoint is the midpoint of its corners.  Returns a Mesh with nen = 8."""
    nx, ny = (int(v) for v in n)
    base = structured_mesh((nx, ny), jitter=jitter, seed=seed, lengths=lengths)
    X = base.coords
    NX, NY = nx + 1, ny + 1
    cid = lambda i, j: i + NX * j
    n_c, n_ex = NX * NY, nx * NY
    ex_id = lambda i, j: n_c + i + nx * j
    ey_id = lambda i, j: n_c + n_ex + i + NX * j
    coords = np.zeros((2, n_c + n_ex + NX * ny))
    coords[:, :n_c] = X
    for j in range(NY):
        for i in range(nx):
            coords[:, ex_id(i, j)] = 0.5 * (X[:, cid(i, j)] + X[:, cid(i + 1, j)])
    for j in range(ny):
        for i in range(NX):
            coords[:, ey_id(i, j)] = 0.5 * (X[:, cid(i, j)] + X[:, cid(i, j + 1)])
    conn = np.zeros((8, nx * ny), dtype=np.int32)
    for ey in range(ny):
        for ex in range(nx):
            e = ex + nx * ey
            for a in range(4):
                conn[a, e] = cid(ex + (a & 1), ey + (a >> 1))
            for b in range(2):
                conn[4 + b, e] = ex_id(ex, ey + b)
                conn[6 + b, e] = ey_id(ex + b, ey)
    return Mesh(coords, conn)


# Kuhn triangulation of a cube: for each ordering (p0, p1, p2) of the axes, the tetrahedron
# with vertices 0, e_p0, e_p0 + e_p1, (1, 1, 1) (corner bits as in structured_mesh).
_KUHN = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
TET10_EDGES = [(0, 1), (1, 2), (2, 0), (0, 3), (1, 3), (2, 3)]


def tet10_mesh(n, jitter: float = 0.0, seed=None, lengths=None) -> Mesh:
    """Quadratic tetrahedra (10 nodes) filling a structured box of n = (nx, ny, nz) cubes.

    Each cube splits into the six Kuhn tetrahedra around its main diagonal, which match
    across cube faces; vertices are ordered so that every tetrahedron is positively
    oriented.  Nodes: the corner lattice of structured_mesh (jittered the same way), then
    one midpoint per edge, numbered in order of first appearance.  Local nodes: vertices
    0..3, then the midpoints of the edges (0,1), (1,2), (2,0), (0,3), (1,3), (2,3).
    Midpoints sit at the middle of straight edges, so every element map is affine."""
    nx, ny, nz = (int(v) for v in n)
    base = structured_mesh((nx, ny, nz), jitter=jitter, seed=seed, lengths=lengths)
    X = base.coords
    NX, NY = nx + 1, ny + 1
    cid = lambda i, j, k: i + NX * (j + NY * k)
    verts = []
    for ez in range(nz):
        for ey in range(ny):
            for ex in range(nx):
                for perm in _KUHN:
                    c = [0, 0, 0]
                    tet = [cid(ex, ey, ez)]
                    for ax in perm:
                        c[ax] = 1
                        tet.append(cid(ex + c[0], ey + c[1], ez + c[2]))
                    P = X[:, tet]
                    if np.linalg.det(np.stack([P[:, m] - P[:, 0] for m in (1, 2, 3)], axis=1)) < 0.0:
                        tet[1], tet[2] = tet[2], tet[1]
                    verts.append(tet)
    edge_id = {}
    mids = []
    conn = np.zeros((10, len(verts)), dtype=np.int64)
    n_c = X.shape[1]
    for e, tet in enumerate(verts):
        conn[:4, e] = tet
        for m, (a, b) in enumerate(TET10_EDGES):
            key = (min(tet[a], tet[b]), max(tet[a], tet[b]))
            if key not in edge_id:
                edge_id[key] = n_c + len(mids)
                mids.append(0.5 * (X[:, key[0]] + X[:, key[1]]))
            conn[4 + m, e] = edge_id[key]
    coords = np.concatenate([X, np.array(mids).T], axis=1)
    return Mesh(coords, conn.astype(np.int32))


def rect_edges(n, sides=None):
    """Element edges on the sides of a structured 2D rectangle of n = (nx, ny) elements.

    sides: local edge ids 2 * axis + side (axis 0: the edges xi = -1 / +1, on x = 0 and
    x = L_x; axis 1: eta = -1 / +1, on y = 0 and y = L_y); default all four.  Returns
    (element ids int32, local edge ids uint8)."""
    nx, ny = (int(v) for v in n)
    sides = range(4) if sides is None else sides
    ex, ey = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    eid = (ex + nx * ey).astype(np.int64)
    idx = (ex, ey)
    elems, ids = [], []
    for f in sides:
        axis, side = f >> 1, f & 1
        sel = idx[axis] == ((n[axis] - 1) if side else 0)
        e = np.sort(eid[sel])
        elems.append(e)
        ids.append(np.full(e.shape, f))
    return np.concatenate(elems).astype(np.int32), np.concatenate(ids).astype(np.uint8)


def tet10_box_faces(mesh: Mesh, lengths=None):
    """Boundary faces of a tet10_mesh box: (element ids int32, local faces uint8), where
    local face k is the face opposite vertex k; a face is on the boundary when its three
    vertices lie on one side of the box [0, L]^3."""
    L = np.ones(3) if lengths is None else np.asarray(lengths, dtype=np.float64)
    X = mesh.coords
    elems, fids = [], []
    for e in range(mesh.n_elems):
        v = mesh.conn[:4, e]
        for k in range(4):
            f = [v[m] for m in range(4) if m != k]
            P = X[:, f]
            for ax in range(3):
                if np.all(np.abs(P[ax]) < 1e-12) or np.all(np.abs(P[ax] - L[ax]) < 1e-12):
                    elems.append(e)
                    fids.append(k)
                    break
    return np.array(elems, dtype=np.int32), np.array(fids, dtype=np.uint8)


def box_faces(n, sides=None):
    """Element faces on the sides of a structured 3D box mesh of n = (nx, ny, nz) elements.

    sides: local face ids 2 * axis + side (side 1: the face at the upper end of the axis);
    default all six.  Returns (element ids int32, local face ids uint8), side by side."""
    nx, ny, nz = (int(v) for v in n)
    sides = range(6) if sides is None else sides
    ex, ey, ez = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    eid = (ex + nx * (ey + ny * ez)).astype(np.int64)
    idx = (ex, ey, ez)
    elems, fids = [], []
    for f in sides:
        axis, side = f >> 1, f & 1
        sel = idx[axis] == ((n[axis] - 1) if side else 0)
        e = np.sort(eid[sel])
        elems.append(e)
        fids.append(np.full(e.shape, f))
    return np.concatenate(elems).astype(np.int32), np.concatenate(fids).astype(np.uint8)


def flow_boundary(mesh: Mesh, kind: str, field_major: bool = False, lid_speed: float = 1.0):
    """Initial state and Dirichlet rows of an enclosed 3D flow on a structured box mesh.

    kind "couette": u = (z, 0, 0) on every boundary node; "cavity": u = (lid_speed, 0, 0)
    on the nodes of the top face z = max (edges included), u = 0 on the rest of the
    boundary.  Velocity is constrained on all boundary nodes and the pressure at node 0.
    Interior values start at 0.  Returns (state [4][n_nodes] float64, DOF mask uint8).
    """
    coords = mesh.coords
    nn = mesh.n_nodes
    on = boundary_node_mask(mesh.shape)
    state = np.zeros((4, nn))
    if kind == "couette":
        state[0] = np.where(on != 0, coords[2], 0.0)
    elif kind == "cavity":
        top = np.isclose(coords[2], coords[2].max())
        state[0] = np.where(top, lid_speed, 0.0)
    else:
        raise ValueError(kind)
    mask = dof_mask(on, 4, field_major, fields=(0, 1, 2))
    mask[3 * nn if field_major else 3] = 1  # pressure of node 0
    return state, mask


def batch_problem_sizes(n_problems: int, lo: int, hi: int, base_seed: int = 6):
    """Per-problem element counts per axis, each drawn U{lo..hi} with seed base_seed + p."""
    sizes = []
    for p in range(n_problems):
        rng = np.random.default_rng(base_seed + p)
        sizes.append(tuple(int(v) for v in rng.integers(lo, hi + 1, size=3)))
    return sizes
