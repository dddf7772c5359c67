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
  traction              R_(a,i) = - int N_a sigma^l_ij n_j

Each face of a hexahedron is xi_axis = -1 or +1 of the reference cube; the face rule is
the 2x2 Gauss rule in the two other reference coordinates, the surface element is
|dx/dxi_u x dx/dxi_v| and the outward normal is that cross product with the sign of the
side.  The basis and its reference gradients come from the oracle's C code (or_basis).

Pins (tests/test_oracle_boundary.py): face mass sums to the area and has the closed form
of a flat square face; a uniform traction integrates to t times the area; domain Laplacian
plus flux term annihilates linear fields (divergence theorem); the radiation tangent
matches central differences.
"""
from __future__ import annotations

import numpy as np

from . import NODE_MAJOR, basis

PENALTY, CONVECTION, RADIATION, FLUX, TRACTION = 0, 1, 2, 3, 4


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
                for a in range(8):
                    for i in range(nf):
                        if kind in (PENALTY, CONVECTION):
                            Ke[a, i, :, i] += coef * w * N[a] * N
                            Re[a, i] += coef * w * N[a] * (uq[i] - gq[i])
                        elif kind == RADIATION:
                            Ke[a, 0, :, 0] += coef * w * N[a] * 4.0 * uq[0] ** 3 * N
                            Re[a, 0] += coef * w * N[a] * (uq[0] ** 4 - gq[0] ** 4)
                        elif kind == TRACTION:
                            S = value.reshape(3, 3)
                            Re[a, i] -= w * N[a] * (S[i] @ n)
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
