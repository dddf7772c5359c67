"""Oracle: boundary forms, integrated over element faces in plain numpy loops.

TEST INFRASTRUCTURE ONLY.  Only `tests/`, the smoke check and the benchmark's CPU
baseline leg may import this module; the product library never does.

Sec. 2.2 (opening of the algorithm): boundary conditions are the domain physics one
dimension lower, assembled by the same process on face data.  Forms of Sec. 4.1 (thermal:
convection, radiation, and the fix condition with its penalty and flux terms) and Sec.
4.2 (elasticity: load traction and penalty fix), with the domain forms' sign reading
R = -d_paper, K = dR/dU, exported d = -R(U):

  penalty / convection  R_(a,i) = int coef N_a (u_i - g_i)
  radiation             R_a     = int coef N_a (T^4 - T_env^4)
  flux                  R_a     = - int coef N_a n . grad T   (grad T of the face's element)
  traction              R_(a,i) = - int N_a sigma^l_ij n_j, or - int N_a t_i with a nodal
                        traction t given as the target

and the flow boundaries of Sec. 4.3 with the flow form's reading R = +d_paper (fields
u_0, u_1, u_2, p; coef = tau^b, value[0..3) = u^w unless a target gives it per node,
value[3] = rho, value[4] = mu; (A, B) is the integral of B times the variation of A):

  every flow kind (base)  R_(a,i) += int N_a (p n_i - mu u_i,j n_j)
  inflow                  R_(a,i) += int rho N_a u^w_i (u^w . n) + mu (n . grad N_a) (u^w_i - u_i)
                                     + tau^b rho N_a (u_i - u^w_i)
                          R_(a,p) += int N_a (u^w - u) . n
  outflow                 R_(a,i) += int rho N_a u_i (u . n)
  fix                     inflow with u^w = 0 (its rho u^w u^w.n term vanishes)

The test gradient in the inflow and fix terms makes every node of the face's element a
row, not only the four face nodes.

Each face of a hexahedron is xi_axis = -1 or +1 of the reference cube; the face rule is
the 2x2 Gauss rule in the two other reference coordinates, the surface element is
|dx/dxi_u x dx/dxi_v| and the outward normal is that cross product with the sign of the
side.  The basis and its reference gradients come from the oracle's C code (or_basis).

Pins (tests/test_oracle_boundary.py): face mass sums to the area and has the closed form
of a flat square face; a uniform traction integrates to t times the area; domain Laplacian
plus flux term annihilates linear fields (divergence theorem); the radiation tangent
matches central differences.  Flow: hand-integrated values of every inflow and outflow
term on one unit cube; the flow domain form (no stabilisation) plus outflow on every face
equals the mass matrix times rho div(u u) + grad p and div u for linear u, p (integration
by parts); inflow with u^w = u equals outflow; tangents match central differences; the
fix condition's pressure-velocity blocks are antisymmetric.
"""
from __future__ import annotations

import numpy as np

from . import NODE_MAJOR, basis

PENALTY, CONVECTION, RADIATION, FLUX, TRACTION, NS_INFLOW, NS_OUTFLOW, NS_FIX = range(8)
FLOW_KINDS = (NS_INFLOW, NS_OUTFLOW, NS_FIX)


def _dof(pat, node, i):
    nf = pat.nf
    return nf * node + i if pat.numbering == NODE_MAJOR else i * pat.mesh.n_nodes + node


def assemble_boundary(pat, kind, coef, value, face_elem, face_id, state=None, target=None):
    """Face contributions only: (scipy CSR matrix [n_rows x n_rows], d [n_rows])."""
    import scipy.sparse as sp
    mesh = pat.mesh
    nf = pat.nf
    coords, conn = mesh.coords, mesh.conn
    value = np.asarray(value, dtype=np.float64)
    g = 1.0 / np.sqrt(3.0)
    rows, cols, vals = [], [], []
    d = np.zeros(pat.n_rows)
    for e, fid in zip(np.asarray(face_elem), np.asarray(face_id)):
        e, fid = int(e), int(fid)
        axis, side = fid >> 1, fid & 1
        u, v = (axis + 1) % 3, (axis + 2) % 3
        nodes = conn[:, e]
        X = coords[:, nodes].T  # [8][3]
        U = state[:, nodes].T if state is not None else np.zeros((8, nf))
        G = target[:, nodes].T if target is not None else np.tile(value[:nf], (8, 1))
        Ke = np.zeros((8, nf, 8, nf))
        Re = np.zeros((8, nf))
        for qv in (-g, g):
            for qu in (-g, g):
                xi = np.zeros(3)
                xi[axis] = 1.0 if side else -1.0
                xi[u], xi[v] = qu, qv
                N, dN = basis(3, xi)
                J = X.T @ dN  # J[m][n] = dx_m / dxi_n
                nr = (1.0 if side else -1.0) * np.cross(J[:, u], J[:, v])
                dS = np.linalg.norm(nr)
                n = nr / dS
                w = dS
                uq = N @ U
                gq = N @ G
                if kind in FLOW_KINDS:
                    grad = np.linalg.solve(J.T, dN.T).T  # rows: grad N_b = J^-T grad_xi N_b
                    _flow_point(kind, coef, value, w, n, N, grad @ n, U, uq, gq, Ke, Re)
                    continue
                for a in range(8):
                    for i in range(nf):
                        if kind in (PENALTY, CONVECTION):
                            Ke[a, i, :, i] += coef * w * N[a] * N
                            Re[a, i] += coef * w * N[a] * (uq[i] - gq[i])
                        elif kind == RADIATION:
                            Ke[a, 0, :, 0] += coef * w * N[a] * 4.0 * uq[0] ** 3 * N
                            Re[a, 0] += coef * w * N[a] * (uq[0] ** 4 - gq[0] ** 4)
                        elif kind == TRACTION:
                            t = gq if target is not None else value.reshape(3, 3) @ n
                            Re[a, i] -= w * N[a] * t[i]
                        elif kind == FLUX:
                            grad = np.linalg.solve(J.T, dN.T).T  # rows: grad N_b = J^-T grad_xi N_b
                            ng = grad @ n
                            Ke[a, 0, :, 0] -= coef * w * N[a] * ng
                            Re[a, 0] -= coef * w * N[a] * (ng @ U[:, 0])
                        else:
                            raise ValueError(kind)
        for a in range(8):
            for i in range(nf):
                r = _dof(pat, nodes[a], i)
                d[r] -= Re[a, i]
                for b in range(8):
                    for j in range(nf):
                        if Ke[a, i, b, j] != 0.0:
                            rows.append(r)
                            cols.append(_dof(pat, nodes[b], j))
                            vals.append(Ke[a, i, b, j])
    K = sp.coo_matrix((vals, (rows, cols)), shape=(pat.n_rows, pat.n_rows)).tocsr()
    return K, d


def _flow_point(kind, coef, value, w, n, N, gn, U, uq, gq, Ke, Re):
    """One face point of a flow boundary form: adds to the element residual Re [8][4] and
    tangent Ke [8][4][8][4] (gn[b] = n . grad N_b)."""
    rho, mu, tau = value[3], value[4], coef
    u, p = uq[:3], uq[3]
    uw = gq[:3] if kind == NS_INFLOW else np.zeros(3)
    un = u @ n
    for a in range(8):
        for i in range(3):
            # base: p n_i - mu u_i,j n_j
            Re[a, i] += w * N[a] * (p * n[i] - mu * (gn @ U[:, i]))
            Ke[a, i, :, 3] += w * N[a] * n[i] * N
            Ke[a, i, :, i] -= w * mu * N[a] * gn
            if kind in (NS_INFLOW, NS_FIX):
                Re[a, i] += w * rho * N[a] * uw[i] * (uw @ n)
                Re[a, i] += w * mu * gn[a] * (uw[i] - u[i])
                Ke[a, i, :, i] -= w * mu * gn[a] * N
                Re[a, i] += w * tau * rho * N[a] * (u[i] - uw[i])
                Ke[a, i, :, i] += w * tau * rho * N[a] * N
            else:
                Re[a, i] += w * rho * N[a] * u[i] * un
                for k in range(3):
                    Ke[a, i, :, k] += w * rho * N[a] * N * ((un if i == k else 0.0) + u[i] * n[k])
        if kind in (NS_INFLOW, NS_FIX):
            Re[a, 3] += w * N[a] * ((uw - u) @ n)
            for k in range(3):
                Ke[a, 3, :, k] -= w * N[a] * N * n[k]


def edge_nodes_2d(nen, eid):
    """Local ids of the nodes on edge eid = 2 * axis + side of a quadrilateral: the two
    corners with bit `axis` equal to `side`, then (8-node element) the edge midpoint."""
    axis, side = eid >> 1, eid & 1
    nodes = [a for a in range(4) if ((a >> axis) & 1) == side]
    if nen == 8:
        nodes.append(6 + side if axis == 0 else 4 + side)
    return nodes


def assemble_boundary_2d(pat, kind, coef, value, edge_elem, edge_id, state=None, target=None):
    """Boundary forms on edges of 4- and 8-node quadrilaterals: (scipy CSR, d), the forms
    and signs of the 3D faces (penalty, convection, radiation, traction with sigma^l the
    leading 2x2 block of value or a nodal traction target).  Edge eid = 2 * axis + side is
    xi_axis = -1 or +1; Gauss rule with 2 (4-node) or 3 (8-node) points along it;
    ds = |dx/dt|, n the unit normal to the tangent pointing away from the element's
    centre."""
    import scipy.sparse as sp
    from .serendipity import basis8
    mesh = pat.mesh
    nf, nen = pat.nf, mesh.nen
    value = np.asarray(value, dtype=np.float64)
    npts = 3 if nen == 8 else 2
    gp, gw = np.polynomial.legendre.leggauss(npts)
    rows, cols, vals = [], [], []
    d = np.zeros(pat.n_rows)
    for e, eid in zip(np.asarray(edge_elem), np.asarray(edge_id)):
        e, eid = int(e), int(eid)
        axis, side = eid >> 1, eid & 1
        other = 1 - axis
        nodes = mesh.conn[:, e]
        X = mesh.coords[:, nodes].T
        centre = X[:4].mean(axis=0)
        U = state[:, nodes].T if state is not None else np.zeros((nen, nf))
        G = np.asarray(target)[:, nodes].T if target is not None else np.tile(value[:nf], (nen, 1))
        Ke = np.zeros((nen, nf, nen, nf))
        Re = np.zeros((nen, nf))
        for t, wq in zip(gp, gw):
            xi = np.zeros(2)
            xi[axis] = 1.0 if side else -1.0
            xi[other] = t
            N, dN = basis8(xi) if nen == 8 else basis(2, xi)
            tang = X.T @ dN[:, other]
            nr = np.array([tang[1], -tang[0]])
            if nr @ (N @ X - centre) < 0.0:
                nr = -nr
            ds = np.linalg.norm(tang)
            n = nr / np.linalg.norm(nr)
            w = wq * ds
            uq, gq = N @ U, N @ G
            for i in range(nf):
                if kind in (PENALTY, CONVECTION):
                    Ke[:, i, :, i] += coef * w * np.outer(N, N)
                    Re[:, i] += coef * w * N * (uq[i] - gq[i])
                elif kind == RADIATION:
                    Ke[:, 0, :, 0] += coef * w * 4.0 * uq[0] ** 3 * np.outer(N, N)
                    Re[:, 0] += coef * w * N * (uq[0] ** 4 - gq[0] ** 4)
                elif kind == TRACTION:
                    tv = gq if target is not None else value.reshape(3, 3)[:2, :2] @ n
                    Re[:, i] -= w * N * tv[i]
                else:
                    raise ValueError(kind)
        en = edge_nodes_2d(nen, eid)
        for a in en:
            for i in range(nf):
                r = _dof(pat, nodes[a], i)
                d[r] -= Re[a, i]
                for b in en:
                    for j in range(nf):
                        if Ke[a, i, b, j] != 0.0:
                            rows.append(r)
                            cols.append(_dof(pat, nodes[b], j))
                            vals.append(Ke[a, i, b, j])
        off = [a for a in range(nen) if a not in en]
        assert np.abs(Re[off]).max(initial=0.0) < 1e-13 * max(1.0, np.abs(Re).max())
    K = sp.coo_matrix((vals, (rows, cols)), shape=(pat.n_rows, pat.n_rows)).tocsr()
    return K, d
