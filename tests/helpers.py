"""Shared test utilities: tolerance metrics and the sampled-row oracle for full-size meshes."""
import numpy as np

import oracle as O
import workloads as W

TOL = {0: 1e-12, 1: 1e-5}  # FP64, FP32 (row-scaled, see rowscaled_error)


def rowscaled_error(pat, K, Kref):
    """max_ij |K_ij - Kref_ij| / max_j |Kref_ij| (entrywise relative error fails on
    entries that cancel to ~0, so each row is scaled by its largest reference entry).
    A row whose reference is all zero must match exactly (its error is then 0 or inf)."""
    rp = np.asarray(pat.row_ptr if hasattr(pat, "row_ptr") else pat, np.int64)
    n = len(rp) - 1
    if n <= 0 or rp[-1] == 0:
        return 0.0
    diff = np.abs(np.asarray(K, np.float64) - Kref)
    ref = np.abs(np.asarray(Kref, np.float64))
    nonempty = rp[1:] > rp[:-1]
    starts = rp[:-1][nonempty]
    rowdiff = np.maximum.reduceat(diff, starts)
    rowmax = np.maximum.reduceat(ref, starts)
    err = np.where(rowmax > 0, rowdiff / np.where(rowmax > 0, rowmax, 1.0), np.where(rowdiff > 0, np.inf, 0.0))
    return float(np.max(err))


def rowscaled_sparse(A, B):
    """The row-scaled error of rowscaled_error for two scipy sparse matrices of one shape."""
    D = abs((A - B).tocsr())
    R = abs(B.tocsr())
    dmax = np.asarray(D.max(axis=1).todense()).ravel()
    rmax = np.asarray(R.max(axis=1).todense()).ravel()
    err = np.where(rmax > 0, dmax / np.where(rmax > 0, rmax, 1.0), np.where(dmax > 0, np.inf, 0.0))
    return float(err.max()) if err.size else 0.0


def vec_error(d, dref):
    d = np.asarray(d, np.float64)
    m = np.max(np.abs(dref)) if dref.size else 0.0
    return float(np.max(np.abs(d - dref)) / (m if m > 0 else 1.0)) if dref.size else 0.0


def submesh_for_nodes(mesh, nodes):
    """Elements adjacent to `nodes` and a compact renumbering of their nodes.

    Returns (sub_mesh, sub_elem_ids, local_of_global) where the rows of `nodes` in the
    sub-mesh assembly are complete (every adjacent element is present)."""
    nodes = np.asarray(nodes)
    mark = np.zeros(mesh.n_nodes, bool)
    mark[nodes] = True
    elems = np.nonzero(np.any(mark[mesh.conn], axis=0))[0]
    used = np.unique(mesh.conn[:, elems])
    local = -np.ones(mesh.n_nodes, np.int64)
    local[used] = np.arange(used.size)
    sub = W.Mesh(mesh.coords[:, used], local[mesh.conn[:, elems]].astype(np.int32))
    return sub, elems, used, local


def oracle_rows(mesh, nodes, kind, nf, params, elem_param=None, nodal_src=None, state=None, qpa=2):
    """Oracle rows of K (as dense blocks over global columns) and d for the given nodes,
    node-major numbering, without Dirichlet constraints.

    Returns {node: (cols_global [ncol], Krows [nf][ncol], d [nf])}."""
    sub, elems, used, local = submesh_for_nodes(mesh, nodes)
    pat = O.Pattern(sub, nf)
    ep = None if elem_param is None else np.asarray(elem_param, np.float64)[elems]
    ns = None if nodal_src is None else np.asarray(nodal_src, np.float64)[:, used]
    st = None if state is None else np.asarray(state, np.float64)[:, used]
    K, d = O.assemble(pat, kind, params, elem_param=ep, nodal_src=ns, state=st, qpa=qpa)
    out = {}
    for v in nodes:
        lv = local[v]
        rows = []
        for i in range(nf):
            r = nf * lv + i
            sl = slice(pat.row_ptr[r], pat.row_ptr[r + 1])
            cl = pat.col_idx[sl]
            # local dof -> global dof (node-major)
            cg = nf * used[cl // nf] + cl % nf
            rows.append((cg, K[sl]))
        cols = rows[0][0]
        out[int(v)] = (cols, np.stack([r[1] for r in rows]), d[nf * lv:nf * lv + nf].copy())
    return out
