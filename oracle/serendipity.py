"""Oracle: quadratic elements in plain numpy: 20-node serendipity hexahedra, 8-node
serendipity quadrilaterals and 10-node tetrahedra.

TEST INFRASTRUCTURE ONLY.  Only `tests/`, the smoke check and the benchmark's CPU
baseline leg may import this module; the product library never does.

The paper's experiments use quadratic serendipity elements (Sec. 4); the element order is
one of the six inputs of the problem statement (Sec. 1).  Reference cube [-1, 1]^3,
local nodes as workloads.serendipity_mesh numbers them (corners a = ax + 2 ay + 4 az,
then the x-, y- and z-edge midpoints).  Shape functions, with s the corner signs:
  corner   N = (1/8)(1 + s_x x)(1 + s_y y)(1 + s_z z)(s_x x + s_y y + s_z z - 2)
  x-edge   N = (1/4)(1 - x^2)(1 + s_y y)(1 + s_z z)       (and cyclically for y, z)
Quadrature: 3 Gauss points per axis, +-sqrt(3/5) and 0 with weights 5/9 and 8/9.  The
8-node quadrilateral (basis8) is the same construction in 2D; the 10-node tetrahedron
(basis10) uses the collapsed 64-point rule gauss_tet; assemble20 and Pattern20 take any
of these meshes.
Forms as the Q1 oracle defines them at the zero state (Sec. 4.1, 4.2; K = dR/dU, d = -R):
  mass        K = int c N_a N_b,                        d = int c N_a f
  conduction  K = int c grad N_a . grad N_b,            d = int N_a f
  elasticity  K = int lam g_ai g_bj + mu g_aj g_bi + mu delta_ij g_a . g_b,  d = int N_a b_i
with c = coef * elem_param and lam, mu from E = coef * elem_param and nu.  The steady
flow form (Sec. 4.3, base terms with the SUPG/PSPG/LSIC terms) is the one of the Q1
oracle at a given state (u, p) per node: R and its full Newton tangent K = dR/dU, d = -R,
with Rm_i = rho u_k du_i/dx_k + dp/dx_i (the second derivatives of u left out of Rm, as
for the linear elements).  The pattern
is built by brute force: N(v) = sorted nodes sharing an element with v.  Boundary forms on
the element faces (8 nodes, 3x3 face rule): assemble_boundary20.
"""
from __future__ import annotations

import numpy as np

from . import ELASTICITY, MASS, NODE_MAJOR, NS_SUPG, POISSON

CORNER = np.array([[1.0 if (a >> d) & 1 else -1.0 for d in range(3)] for a in range(8)])
# edge nodes: (axis along the edge, signs of the two other axes in cyclic order)
EDGES = [(ax, ((m & 1) * 2 - 1.0, (m >> 1) * 2 - 1.0)) for ax in range(3) for m in range(4)]


def basis20(xi):
    """N [20], dN [20][3] at the reference point xi."""
    x = np.asarray(xi, dtype=np.float64)
    N = np.zeros(20)
    dN = np.zeros((20, 3))
    for a in range(8):
        s = CORNER[a]
        f = 1.0 + s * x
        t = s @ x - 2.0
        N[a] = 0.125 * f[0] * f[1] * f[2] * t
        for d in range(3):
            o = [k for k in range(3) if k != d]
            dN[a, d] = 0.125 * (s[d] * f[o[0]] * f[o[1]] * t + f[0] * f[1] * f[2] * s[d])
    for m, (ax, (s1, s2)) in enumerate(EDGES):
        o1, o2 = (ax + 1) % 3, (ax + 2) % 3
        # edge along ax: the other two axes carry the signs in the order (y, z), (x, z), (x, y)
        oth = sorted((o1, o2))
        sg = {oth[0]: s1, oth[1]: s2}
        g0 = 1.0 - x[ax] ** 2
        h1, h2 = 1.0 + sg[oth[0]] * x[oth[0]], 1.0 + sg[oth[1]] * x[oth[1]]
        N[8 + m] = 0.25 * g0 * h1 * h2
        dN[8 + m, ax] = 0.25 * (-2.0 * x[ax]) * h1 * h2
        dN[8 + m, oth[0]] = 0.25 * g0 * sg[oth[0]] * h2
        dN[8 + m, oth[1]] = 0.25 * g0 * h1 * sg[oth[1]]
    return N, dN


def basis8(xi):
    """N [8], dN [8][2] of the 8-node serendipity quadrilateral at the reference point xi.

    Local nodes: corners a = ax + 2 ay, then the x-edge midpoints at y = -1, +1, then the
    y-edge midpoints at x = -1, +1:
      corner  N = (1/4)(1 + s_x x)(1 + s_y y)(s_x x + s_y y - 1)
      x-edge  N = (1/2)(1 - x^2)(1 + s_y y),   y-edge  N = (1/2)(1 - y^2)(1 + s_x x)
    """
    x, y = (float(v) for v in xi)
    N = np.zeros(8)
    dN = np.zeros((8, 2))
    for a in range(4):
        sx, sy = (1.0 if a & 1 else -1.0), (1.0 if a >> 1 else -1.0)
        fx, fy, t = 1.0 + sx * x, 1.0 + sy * y, sx * x + sy * y - 1.0
        N[a] = 0.25 * fx * fy * t
        dN[a] = [0.25 * (sx * fy * t + fx * fy * sx), 0.25 * (fx * sy * t + fx * fy * sy)]
    for b in range(2):
        s = 1.0 if b else -1.0
        N[4 + b] = 0.5 * (1.0 - x * x) * (1.0 + s * y)
        dN[4 + b] = [-x * (1.0 + s * y), 0.5 * (1.0 - x * x) * s]
        N[6 + b] = 0.5 * (1.0 - y * y) * (1.0 + s * x)
        dN[6 + b] = [0.5 * (1.0 - y * y) * s, -y * (1.0 + s * x)]
    return N, dN


def basis10(xi):
    """N [10], dN [10][3] of the 10-node quadratic tetrahedron at the reference point xi
    (reference tetrahedron xi >= 0, xi_1 + xi_2 + xi_3 <= 1).  Barycentric coordinates
    l_0 = 1 - xi_1 - xi_2 - xi_3, l_k = xi_k; vertices N_i = l_i (2 l_i - 1), edge
    midpoints N_ij = 4 l_i l_j for the edges (0,1), (1,2), (2,0), (0,3), (1,3), (2,3)."""
    x = np.asarray(xi, dtype=np.float64)
    lam = np.array([1.0 - x.sum(), x[0], x[1], x[2]])
    dlam = np.array([[-1.0, -1.0, -1.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    N = np.zeros(10)
    dN = np.zeros((10, 3))
    for i in range(4):
        N[i] = lam[i] * (2.0 * lam[i] - 1.0)
        dN[i] = (4.0 * lam[i] - 1.0) * dlam[i]
    for m, (i, j) in enumerate([(0, 1), (1, 2), (2, 0), (0, 3), (1, 3), (2, 3)]):
        N[4 + m] = 4.0 * lam[i] * lam[j]
        dN[4 + m] = 4.0 * (lam[i] * dlam[j] + lam[j] * dlam[i])
    return N, dN


def gauss_tet():
    """64-point rule on the reference tetrahedron: the 4-point Gauss-Legendre rule on each
    axis of the unit cube, collapsed onto the tetrahedron by xi_1 = u, xi_2 = v (1 - u),
    xi_3 = w (1 - u)(1 - v) with Jacobian (1 - u)^2 (1 - v); exact for total degree 5."""
    g, gw = np.polynomial.legendre.leggauss(4)
    t, tw = 0.5 * (g + 1.0), 0.5 * gw
    pts, wts = [], []
    for k in range(4):
        for j in range(4):
            for i in range(4):
                u, v, w = t[i], t[j], t[k]
                pts.append([u, v * (1.0 - u), w * (1.0 - u) * (1.0 - v)])
                wts.append(tw[i] * tw[j] * tw[k] * (1.0 - u) ** 2 * (1.0 - v))
    return np.array(pts), np.array(wts)


def gauss3_2d():
    p = np.sqrt(3.0 / 5.0)
    pts, wts = np.array([-p, 0.0, p]), np.array([5.0, 8.0, 5.0]) / 9.0
    xi = np.array([[pts[i], pts[j]] for j in range(3) for i in range(3)])
    w = np.array([wts[i] * wts[j] for j in range(3) for i in range(3)])
    return xi, w


def gauss3():
    p = np.sqrt(3.0 / 5.0)
    pts, wts = np.array([-p, 0.0, p]), np.array([5.0, 8.0, 5.0]) / 9.0
    xi = np.array([[pts[i], pts[j], pts[k]] for k in range(3) for j in range(3) for i in range(3)])
    w = np.array([wts[i] * wts[j] * wts[k] for k in range(3) for j in range(3) for i in range(3)])
    return xi, w


class Pattern20:
    """CSR pattern of K on a 20-node hex mesh, brute force."""

    def __init__(self, mesh, nf: int, numbering: int = NODE_MAJOR):
        self.mesh, self.nf, self.numbering = mesh, nf, numbering
        nn = mesh.n_nodes
        nbr = [set() for _ in range(nn)]
        for e in range(mesh.n_elems):
            nodes = mesh.conn[:, e]
            for v in nodes:
                nbr[v].update(int(u) for u in nodes)
        self.nbr = [np.array(sorted(s), dtype=np.int64) for s in nbr]
        self.n_rows = nn * nf
        rows = []
        for r in range(self.n_rows):
            v, i = (r // nf, r % nf) if numbering == NODE_MAJOR else (r % nn, r // nn)
            if numbering == NODE_MAJOR:
                cols = (nf * self.nbr[v][:, None] + np.arange(nf)[None, :]).reshape(-1)
            else:
                cols = (np.arange(nf)[:, None] * nn + self.nbr[v][None, :]).reshape(-1)
            rows.append(cols)
        self.row_ptr = np.zeros(self.n_rows + 1, np.int64)
        self.row_ptr[1:] = np.cumsum([len(c) for c in rows])
        self.col_idx = np.concatenate(rows).astype(np.int32)
        self.nnz = int(self.row_ptr[-1])

    def dof(self, v, i):
        return self.nf * v + i if self.numbering == NODE_MAJOR else i * self.mesh.n_nodes + v

    def to_scipy(self, values):
        import scipy.sparse as sp
        return sp.csr_matrix((values, self.col_idx, self.row_ptr), shape=(self.n_rows, self.n_rows))


def ns_element(N, g, W, Ue, prm, Ke, De):
    """Flow form at one integration point: adds W times the tangent and -W times the
    residual of the element to Ke [nen][nf][nen][nf] and De [nen][nf].  N [nen], g [nen][dim]
    (physical gradients), Ue [nen][nf] the element state (velocity, then pressure)."""
    rho, mu, tm, tc = prm["rho"], prm["mu"], prm["tau_m"], prm["tau_c"]
    dim = g.shape[1]
    u = N @ Ue[:, :dim]                     # velocity
    gu = Ue[:, :dim].T @ g                  # gu[i][k] = du_i / dx_k
    p = N @ Ue[:, dim]
    gp = g.T @ Ue[:, dim]
    div = np.trace(gu)
    Rm = rho * gu @ u + gp                  # rho u_k du_i/dx_k + dp/dx_i
    adv = g @ u                             # u . grad N_a
    gg = g @ g.T
    I = np.eye(dim)
    # residual: momentum rows (a, i), continuity rows (a, p)
    Ru = (-rho * np.outer(adv, u) - g * p + mu * g @ gu.T + tm * rho * np.outer(adv, Rm) + tc * g * div)
    Rp = N * div + tm * g @ Rm
    De[:, :dim] -= W * Ru
    De[:, dim] -= W * Rp
    # tangent dR/dU: velocity-velocity, velocity-pressure, pressure-velocity, pressure-pressure
    Kuu = (-rho * np.einsum("il,a,b->aibl", I, adv, N)
           - rho * np.einsum("i,al,b->aibl", u, g, N)
           + mu * np.einsum("il,ab->aibl", I, gg)
           + tm * rho * np.einsum("i,al,b->aibl", Rm, g, N)
           + tm * rho * rho * np.einsum("a,b,il->aibl", adv, N, gu)
           + tm * rho * rho * np.einsum("il,a,b->aibl", I, adv, adv)
           + tc * np.einsum("ai,bl->aibl", g, g))
    Kup = -np.einsum("ai,b->aib", g, N) + tm * rho * np.einsum("a,bi->aib", adv, g)
    Kpu = (np.einsum("a,bl->abl", N, g)
           + tm * rho * (np.einsum("b,al->abl", N, g @ gu) + np.einsum("al,b->abl", g, adv)))
    Kpp = tm * gg
    Ke[:, :dim, :, :dim] += W * Kuu
    Ke[:, :dim, :, dim] += W * Kup
    Ke[:, dim, :, :dim] += W * Kpu
    Ke[:, dim, :, dim] += W * Kpp


def assemble20(pat: Pattern20, kind, params=None, elem_param=None, nodal_src=None, state=None):
    """(K values [nnz] in the pattern's order, d [n_rows]).  state [nf][n_nodes]: the point
    of linearisation of the flow form (zero when None)."""
    import scipy.sparse as sp
    prm = dict(coef=1.0, nu=0.0, rho=0.0, mu=0.0, tau_m=0.0, tau_c=0.0)
    prm.update(params or {})
    mesh, nf = pat.mesh, pat.nf
    dim, nen = mesh.dim, mesh.nen
    if nen == 10:
        xi, w = gauss_tet()
        basis = basis10
    else:
        xi, w = gauss3() if dim == 3 else gauss3_2d()
        basis = basis20 if dim == 3 else basis8
    tables = [basis(x) for x in xi]
    rows, cols, vals = [], [], []
    d = np.zeros(pat.n_rows)
    for e in range(mesh.n_elems):
        nodes = mesh.conn[:, e]
        X = mesh.coords[:, nodes].T  # [nen][dim]
        ep = 1.0 if elem_param is None else float(elem_param[e])
        src = np.zeros((nen, nf)) if nodal_src is None else np.asarray(nodal_src)[:, nodes].T
        Ue = np.zeros((nen, nf)) if state is None else np.asarray(state, np.float64)[:, nodes].T
        Ke = np.zeros((nen, nf, nen, nf))
        De = np.zeros((nen, nf))
        for (N, dN), wq in zip(tables, w):
            J = X.T @ dN  # J[m][n] = dx_m / dxi_n
            det = np.linalg.det(J)
            if not det > 0.0:
                raise FloatingPointError(f"det J <= 0 in element {e}")
            g = np.linalg.solve(J.T, dN.T).T  # [nen][dim] physical gradients
            W = wq * det
            fq = N @ src
            if kind == MASS:
                c = prm["coef"] * ep
                Ke[:, 0, :, 0] += W * c * np.outer(N, N)
                De[:, 0] += W * c * N * fq[0]
            elif kind == POISSON:
                c = prm["coef"] * ep
                Ke[:, 0, :, 0] += W * c * (g @ g.T)
                De[:, 0] += W * N * fq[0]
            elif kind == ELASTICITY:
                E, nu = prm["coef"] * ep, prm["nu"]
                lam = E * nu / ((1 + nu) * (1 - 2 * nu))
                mu = E / (2 * (1 + nu))
                gg = g @ g.T
                Ke += W * (lam * np.einsum("ai,bj->aibj", g, g) + mu * np.einsum("aj,bi->aibj", g, g)
                           + mu * np.einsum("ab,ij->aibj", gg, np.eye(dim)))
                De += W * np.outer(N, fq)
            elif kind == NS_SUPG:
                ns_element(N, g, W, Ue, prm, Ke, De)
            else:
                raise ValueError(kind)
        for a in range(nen):
            for i in range(nf):
                r = pat.dof(nodes[a], i)
                d[r] += De[a, i]
                for b in range(nen):
                    for j in range(nf):
                        rows.append(r)
                        cols.append(pat.dof(nodes[b], j))
                        vals.append(Ke[a, i, b, j])
    S = sp.coo_matrix((vals, (rows, cols)), shape=(pat.n_rows, pat.n_rows)).tocsr()
    S.sum_duplicates()
    rr = np.repeat(np.arange(pat.n_rows), np.diff(pat.row_ptr))
    K = np.asarray(S[rr, pat.col_idx]).ravel()
    return K, d


def ref_nodes20():
    """Reference coordinates [20][3] of the local nodes."""
    X = np.zeros((20, 3))
    X[:8] = CORNER
    for m, (ax, (s1, s2)) in enumerate(EDGES):
        oth = sorted(((ax + 1) % 3, (ax + 2) % 3))
        X[8 + m, oth[0]], X[8 + m, oth[1]] = s1, s2
    return X


def assemble_boundary20(pat: Pattern20, kind, coef, value, face_elem, face_id, state=None, target=None):
    """Boundary forms on faces of 20-node hexahedra: (scipy CSR [n_rows x n_rows], d).

    The forms and sign of the Q1 oracle (oracle/boundary.py; Sec. 2.2 opening, Sec. 4.1,
    4.2), R = -d_paper, K = dR/dU, d = -R:
      penalty / convection  R_(a,i) = int coef N_a (u_i - g_i)
      radiation             R_a     = int coef N_a (T^4 - T_env^4)
      traction              R_(a,i) = - int N_a t_i,  t = sigma^l n, or the nodal traction
                            `target` interpolated with the basis
    Face (axis, side) is xi_axis = -1 or +1 with its eight nodes; the face rule is 3x3
    Gauss in the two other reference coordinates, dS = |t_u x t_v|, n = (t_u x t_v)/dS
    signed by the side.
    """
    import scipy.sparse as sp
    from .boundary import CONVECTION, PENALTY, RADIATION, TRACTION
    mesh, nf = pat.mesh, pat.nf
    value = np.asarray(value, dtype=np.float64)
    p1, w1 = gauss3()[0][:3, 0], np.array([5.0, 8.0, 5.0]) / 9.0
    R0 = ref_nodes20()
    rows, cols, vals = [], [], []
    d = np.zeros(pat.n_rows)
    for e, fid in zip(np.asarray(face_elem), np.asarray(face_id)):
        e, fid = int(e), int(fid)
        axis, side = fid >> 1, fid & 1
        u, v = (axis + 1) % 3, (axis + 2) % 3
        nodes = mesh.conn[:, e]
        X = mesh.coords[:, nodes].T
        U = state[:, nodes].T if state is not None else np.zeros((20, nf))
        if target is not None:
            G = np.asarray(target)[:, nodes].T
        else:
            G = np.tile(value[:nf], (20, 1))
        Ke = np.zeros((20, nf, 20, nf))
        Re = np.zeros((20, nf))
        for jv in range(3):
            for ju in range(3):
                xi = np.zeros(3)
                xi[axis] = 1.0 if side else -1.0
                xi[u], xi[v] = p1[ju], p1[jv]
                N, dN = basis20(xi)
                J = X.T @ dN
                nr = (1.0 if side else -1.0) * np.cross(J[:, u], J[:, v])
                dS = np.linalg.norm(nr)
                n = nr / dS
                w = w1[ju] * w1[jv] * dS
                uq, gq = N @ U, N @ G
                for i in range(nf):
                    if kind in (PENALTY, CONVECTION):
                        Ke[:, i, :, i] += coef * w * np.outer(N, N)
                        Re[:, i] += coef * w * N * (uq[i] - gq[i])
                    elif kind == RADIATION:
                        Ke[:, 0, :, 0] += coef * w * 4.0 * uq[0] ** 3 * np.outer(N, N)
                        Re[:, 0] += coef * w * N * (uq[0] ** 4 - gq[0] ** 4)
                    elif kind == TRACTION:
                        t = gq if target is not None else value.reshape(3, 3) @ n
                        Re[:, i] -= w * N * t[i]
                    else:
                        raise ValueError(kind)
        on_face = R0[:, axis] == (1.0 if side else -1.0)
        for a in np.nonzero(on_face)[0]:
            for i in range(nf):
                r = pat.dof(nodes[a], i)
                d[r] -= Re[a, i]
                for b in np.nonzero(on_face)[0]:
                    for j in range(nf):
                        if Ke[a, i, b, j] != 0.0:
                            rows.append(r)
                            cols.append(pat.dof(nodes[b], j))
                            vals.append(Ke[a, i, b, j])
        # the basis of the other twelve nodes vanishes on the face
        assert np.abs(Re[~on_face]).max(initial=0.0) < 1e-13 * max(1.0, np.abs(Re).max())
    K = sp.coo_matrix((vals, (rows, cols)), shape=(pat.n_rows, pat.n_rows)).tocsr()
    return K, d


# face k of a tetrahedron: the three vertices other than k, and the local ids of the
# midpoints of the edges among them
TET_FACE_VERTS = [(1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2)]
_TET_EDGES = [(0, 1), (1, 2), (2, 0), (0, 3), (1, 3), (2, 3)]


def tet_face_nodes(k):
    """Local ids of the six nodes of face k (opposite vertex k): vertices, then edges."""
    vs = TET_FACE_VERTS[k]
    es = [4 + m for m, (i, j) in enumerate(_TET_EDGES) if i in vs and j in vs]
    return list(vs) + es


def assemble_boundary_tet10(pat: Pattern20, kind, coef, value, face_elem, face_id, state=None, target=None):
    """Boundary forms on faces of 10-node tetrahedra: (scipy CSR, d); the forms and signs of
    assemble_boundary20.  Face k (opposite vertex k) is parametrised by the reference point
    p0 + s (p1 - p0) + t (p2 - p0) over its vertices p0, p1, p2 (s, t >= 0, s + t <= 1), with
    the collapsed 4 x 4 Gauss rule of the triangle (exact to total degree 5); dS =
    |dx/ds x dx/dt|, n signed to point away from vertex k."""
    import scipy.sparse as sp
    from .boundary import CONVECTION, PENALTY, RADIATION, TRACTION
    mesh, nf = pat.mesh, pat.nf
    value = np.asarray(value, dtype=np.float64)
    g, gw = np.polynomial.legendre.leggauss(4)
    t1, w1 = 0.5 * (g + 1.0), 0.5 * gw
    tri = [(t1[i], t1[j] * (1.0 - t1[i]), w1[i] * w1[j] * (1.0 - t1[i])) for j in range(4) for i in range(4)]
    ref = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=np.float64)
    rows, cols, vals = [], [], []
    d = np.zeros(pat.n_rows)
    for e, k in zip(np.asarray(face_elem), np.asarray(face_id)):
        e, k = int(e), int(k)
        nodes = mesh.conn[:, e]
        X = mesh.coords[:, nodes].T
        U = state[:, nodes].T if state is not None else np.zeros((10, nf))
        G = np.asarray(target)[:, nodes].T if target is not None else np.tile(value[:nf], (10, 1))
        v0, v1, v2 = (ref[m] for m in TET_FACE_VERTS[k])
        Ke = np.zeros((10, nf, 10, nf))
        Re = np.zeros((10, nf))
        # outward: away from vertex k
        xk = X[k]
        for s_, t_, wq in tri:
            xi = v0 + s_ * (v1 - v0) + t_ * (v2 - v0)
            N, dN = basis10(xi)
            J = X.T @ dN
            ts, tt = J @ (v1 - v0), J @ (v2 - v0)
            nr = np.cross(ts, tt)
            if nr @ (N @ X - xk) < 0.0:
                nr = -nr
            dS = np.linalg.norm(nr)
            n = nr / dS
            w = wq * dS
            uq, gq = N @ U, N @ G
            for i in range(nf):
                if kind in (PENALTY, CONVECTION):
                    Ke[:, i, :, i] += coef * w * np.outer(N, N)
                    Re[:, i] += coef * w * N * (uq[i] - gq[i])
                elif kind == RADIATION:
                    Ke[:, 0, :, 0] += coef * w * 4.0 * uq[0] ** 3 * np.outer(N, N)
                    Re[:, 0] += coef * w * N * (uq[0] ** 4 - gq[0] ** 4)
                elif kind == TRACTION:
                    tv = gq if target is not None else value.reshape(3, 3) @ n
                    Re[:, i] -= w * N * tv[i]
                else:
                    raise ValueError(kind)
        fn = tet_face_nodes(k)
        for a in fn:
            for i in range(nf):
                r = pat.dof(nodes[a], i)
                d[r] -= Re[a, i]
                for b in fn:
                    for j in range(nf):
                        if Ke[a, i, b, j] != 0.0:
                            rows.append(r)
                            cols.append(pat.dof(nodes[b], j))
                            vals.append(Ke[a, i, b, j])
        off = [a for a in range(10) if a not in fn]
        assert np.abs(Re[off]).max(initial=0.0) < 1e-13 * max(1.0, np.abs(Re).max())
    K = sp.coo_matrix((vals, (rows, cols)), shape=(pat.n_rows, pat.n_rows)).tocsr()
    return K, d
