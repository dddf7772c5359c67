"""Oracle pins for the sparsity pattern (Sec. 2.2 B-1..B-4: control-point pairs, DOF map,
sparse layout), checked against brute-force dense adjacency and closed-form counts."""
import itertools

import numpy as np
import pytest

import oracle as O
import workloads as W


def brute_pattern(mesh, nf, coupling, numbering):
    """Dense adjacency from the element lists, then the CSR it implies."""
    nn = mesh.n_nodes
    A = np.zeros((nn, nn), dtype=bool)
    for e in range(mesh.n_elems):
        nodes = mesh.conn[:, e]
        for a in nodes:
            for b in nodes:
                A[a, b] = True
    n_rows = nn * nf

    def dof(v, i):
        return nf * v + i if numbering == O.NODE_MAJOR else i * nn + v

    rows = [[] for _ in range(n_rows)]
    for v in range(nn):
        for i in range(nf):
            for w in np.nonzero(A[v])[0]:
                for j in range(nf):
                    if coupling[i][j]:
                        rows[dof(v, i)].append(dof(w, j))
    row_ptr = np.zeros(n_rows + 1, np.int64)
    cols = []
    for r in range(n_rows):
        rr = sorted(rows[r])
        row_ptr[r + 1] = row_ptr[r] + len(rr)
        cols += rr
    return row_ptr, np.array(cols, np.int32)


MESHES = [
    ("q1x1", lambda: W.structured_mesh((1, 1))),
    ("q3x2", lambda: W.structured_mesh((3, 2))),
    ("h1x1x1", lambda: W.structured_mesh((1, 1, 1))),
    ("h3x2x2", lambda: W.structured_mesh((3, 2, 2))),
    ("h3x2x2perm", lambda: W.permute_mesh(W.structured_mesh((3, 2, 2)), seed=11)[0]),
]
COUPLINGS = {
    1: [[1]],
    3: [[1, 1, 1], [1, 1, 1], [1, 1, 1]],
    2: [[1, 0], [1, 1]],  # lower-triangular block coupling (asymmetric pattern)
    4: [[1, 1, 0, 1], [1, 1, 0, 1], [0, 0, 1, 1], [1, 1, 1, 1]],
}


@pytest.mark.parametrize("name,make", MESHES)
@pytest.mark.parametrize("nf", [1, 2, 3, 4])
@pytest.mark.parametrize("numbering", [O.NODE_MAJOR, O.FIELD_MAJOR])
def test_pattern_matches_brute_force(name, make, nf, numbering):
    mesh = make()
    cpl = np.array(COUPLINGS[nf], np.uint8)
    pat = O.Pattern(mesh, nf, cpl, numbering)
    rp, ci = brute_pattern(mesh, nf, cpl, numbering)
    assert np.array_equal(pat.row_ptr, rp)
    assert np.array_equal(pat.col_idx, ci)


@pytest.mark.parametrize("name,make", MESHES)
def test_rank_map_points_at_the_right_neighbour(name, make):
    mesh = make()
    pat = O.Pattern(mesh, 1)
    nen = mesh.nen
    for e in range(mesh.n_elems):
        for a, b in itertools.product(range(nen), range(nen)):
            va, vb = mesh.conn[a, e], mesh.conn[b, e]
            r = pat.rank[a * nen + b, e]
            assert pat.nbr[pat.nbr_ptr[va] + r] == vb


@pytest.mark.parametrize("n", [(4, 5), (3, 4, 2), (5, 5, 5)])
def test_nnz_closed_form(n):
    """Node pairs of a structured Q1 mesh: prod_d (3 n_d + 1); scalar nnz = pairs * sum(coupling)."""
    mesh = W.structured_mesh(n)
    pairs = int(np.prod([3 * v + 1 for v in n]))
    for nf, cpl in [(1, [[1]]), (2, [[1, 0], [1, 1]]), (3, np.ones((3, 3)))]:
        pat = O.Pattern(mesh, nf, np.array(cpl, np.uint8))
        assert pat.n_pairs == pairs
        assert pat.nnz == pairs * int(np.sum(cpl))
    # interior row length 27 (hex) / 9 (quad)
    deg = np.diff(pat.nbr_ptr)
    assert deg.max() == 3 ** len(n)


def test_symmetric_coupling_gives_symmetric_pattern():
    mesh = W.permute_mesh(W.structured_mesh((3, 3, 2)), seed=3)[0]
    pat = O.Pattern(mesh, 3)
    S = pat.to_scipy(np.ones(pat.nnz))
    assert (S != S.T).nnz == 0
