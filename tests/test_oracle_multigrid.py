"""Oracle pins for the geometric multigrid V-cycle (oracle/multigrid.py), the preconditioner
of the Newton step's Krylov solve (Sec. 2.1; the solver of Sec. 2.2 D-4 is left open by
the paper).

  * trilinear interpolation is exact on trilinear functions of the node indices, in both
    DOF numberings;
  * R = P^T has the textbook full-weighting weights (1, 1/2, 1/4, 1/8 by the number of
    axes along which a fine node is offset from the coarse one);
  * Galerkin identity: on an undistorted (here anisotropic) box, the coarse space is a
    subspace of the fine one and 2-point Gauss integrates Q1 mass, conduction and
    elasticity exactly, so P^T A_fine P is the coarse rediscretisation;
  * the V-cycle as a stationary iteration on Q1 conduction with Dirichlet walls reduces the
    error by a grid-independent factor well below 1;
  * the cycle is a linear map (fixed sweeps, zero initial guesses);
  * face coarsening: on a box the coarsened face list is the coarse box's own, and with a
    penalty (face mass) form on part of the boundary the Galerkin identity still holds;
  * the elimination leaves unit rows and zero columns;
  * a coarse element's coefficient is the mean of its eight children; with a coefficient
    constant on each coarse element the Galerkin identity still holds.
"""
import numpy as np
import pytest

import oracle as O
import oracle.multigrid as MG
import workloads as W


def test_prolongation_is_exact_on_trilinear_functions():
    rng = np.random.default_rng(0)
    fine = (4, 6, 2)
    c = rng.uniform(-1, 1, size=8)

    def f(i, j, k):
        return (c[0] + c[1] * i + c[2] * j + c[3] * k + c[4] * i * j + c[5] * j * k + c[6] * i * k
                + c[7] * i * j * k)

    fi, fj, fk = MG.node_ijk(fine)
    ci, cj, ck = MG.node_ijk((2, 3, 1))
    for numbering in (O.NODE_MAJOR, O.FIELD_MAJOR):
        nf = 2
        P = MG.prolongation(fine, nf, numbering)
        vc = np.zeros(P.shape[1])
        expect = np.zeros(P.shape[0])
        nnc, nnf = ci.size, fi.size
        for fld in range(nf):
            s = 1.0 + fld
            vc[MG.dof_index(np.arange(nnc), fld, nnc, nf, numbering)] = s * f(ci, cj, ck)
            expect[MG.dof_index(np.arange(nnf), fld, nnf, nf, numbering)] = s * f(fi / 2, fj / 2, fk / 2)
        np.testing.assert_allclose(P @ vc, expect, rtol=0, atol=1e-13)


def test_restriction_has_full_weighting_weights():
    fine = (4, 4, 4)
    R = MG.prolongation(fine, 1).T.tocsr()
    # coarse node (1,1,1): the interior one, fine node (2,2,2)
    row = 1 + 3 * (1 + 3 * 1)
    cols = R.indices[R.indptr[row]:R.indptr[row + 1]]
    vals = R.data[R.indptr[row]:R.indptr[row + 1]]
    fi, fj, fk = MG.node_ijk(fine)
    assert cols.size == 27
    for col, v in zip(cols, vals):
        off = abs(fi[col] - 2) + abs(fj[col] - 2) + abs(fk[col] - 2)
        assert max(abs(fi[col] - 2), abs(fj[col] - 2), abs(fk[col] - 2)) == 1 or off == 0
        assert v == 0.5 ** off
    assert vals.sum() == 8.0


@pytest.mark.parametrize("kind,nf,prm", [(O.POISSON, 1, dict(coef=1.7)), (O.MASS, 1, dict(coef=2.0)),
                                         (O.ELASTICITY, 3, dict(coef=1.0, nu=0.3))])
@pytest.mark.parametrize("numbering", [O.NODE_MAJOR, O.FIELD_MAJOR])
def test_galerkin_identity_on_an_undistorted_box(kind, nf, prm, numbering):
    mesh = W.structured_mesh((4, 4, 6), lengths=(1.0, 2.0, 0.5))
    levels = MG.build_levels((4, 4, 6), mesh.coords, nf, kind, [prm, prm], 2, numbering=numbering)
    Af, Ac, P = levels[0]["A"], levels[1]["A"], levels[0]["P"]
    G = (P.T @ Af @ P).toarray()
    ref = Ac.toarray()
    scale = np.abs(ref).max()
    assert np.abs(G - ref).max() <= 1e-12 * scale
    # and the coarse grid's own geometry is the fine grid's at even nodes
    assert levels[1]["dims"] == (2, 2, 3)
    np.testing.assert_array_equal(levels[1]["mesh"].coords[:, 0], mesh.coords[:, 0])


def _conduction_rate(n, cycles=8):
    mesh = W.structured_mesh((n, n, n), jitter=0.1, seed=4)
    mask = W.boundary_node_mask(mesh.shape)
    n_levels = int(np.log2(n))  # down to 2 elements per axis
    levels = MG.build_levels((n, n, n), mesh.coords, 1, O.POISSON, [dict(coef=1.0)] * n_levels, n_levels,
                             dirichlet=mask)
    A = levels[0]["A"]
    rng = np.random.default_rng(1)
    b = rng.uniform(-1, 1, A.shape[0])
    b[mask.astype(bool)] = 0.0
    import scipy.sparse.linalg as spla
    xs = spla.spsolve(A.tocsc(), b)
    x = np.zeros_like(b)
    e0 = np.linalg.norm(xs)
    for _ in range(cycles):
        x = x + MG.vcycle(levels, b - A @ x, omega=0.5, pre=2, post=2, coarse_sweeps=20)
    return (np.linalg.norm(xs - x) / e0) ** (1.0 / cycles)


def test_vcycle_converges_at_a_grid_independent_rate():
    r8 = _conduction_rate(8)
    r16 = _conduction_rate(16)
    # V(2,2) with omega = 1/2 damped Jacobi: 0.21 on both grids; a restriction scaled by
    # half (a plausible slip) gives 0.30 and 0.60
    assert r8 < 0.25 and r16 < 0.25, (r8, r16)
    assert abs(r16 - r8) < 0.05, (r8, r16)


def test_vcycle_is_linear_on_the_flow_tangent():
    n = 8
    mesh = W.structured_mesh((n, n, n), jitter=0.1, seed=3)
    st, mask = W.flow_boundary(mesh, "cavity")
    st[:3] += 0.3 * W.fourier_velocity(mesh.coords, 2) * (1 - W.boundary_node_mask(mesh.shape))[None, :]
    prm = [dict(rho=1.0, mu=0.01, tau_m=0.01 * 2 ** l, tau_c=0.02 * 2 ** l) for l in range(3)]
    levels = MG.build_levels((n, n, n), mesh.coords, 4, O.NS_SUPG, prm, 3, state=st, dirichlet=mask)
    rng = np.random.default_rng(5)
    a, b = rng.standard_normal((2, levels[0]["A"].shape[0]))
    za, zb = MG.vcycle(levels, a), MG.vcycle(levels, b)
    z = MG.vcycle(levels, 2.0 * a - 3.0 * b)
    np.testing.assert_allclose(z, 2.0 * za - 3.0 * zb, rtol=0, atol=1e-11 * np.abs(z).max())


def test_coarsened_box_faces_are_the_coarse_box_faces():
    for dims, sides in (((4, 6, 2), None), ((8, 4, 4), [0, 3, 5])):
        fe, fi = W.box_faces(dims, sides=sides)
        ce, cf = MG.coarsen_faces(dims, fe, fi)
        re_, rf = W.box_faces(tuple(v // 2 for v in dims), sides=sides)
        assert sorted(zip(ce.tolist(), cf.tolist())) == sorted(zip(re_.tolist(), rf.tolist()))
    # an interior face (side 1 of element (1, 0, 0)) stands for the coarse element 0's side 1
    ce, cf = MG.coarsen_faces((4, 2, 2), np.array([1, 0]), np.array([1, 1]))
    assert ce.tolist() == [0] and cf.tolist() == [1]


@pytest.mark.parametrize("numbering", [O.NODE_MAJOR, O.FIELD_MAJOR])
def test_galerkin_identity_with_a_penalty_boundary_form(numbering):
    import oracle.boundary as OB
    dims = (4, 6, 4)
    mesh = W.structured_mesh(dims, lengths=(2.0, 1.0, 0.5))
    fe, fi = W.box_faces(dims, sides=[0, 3, 5])
    tg = W.uniform_nodal(3, mesh.n_nodes, -1, 1, 2)
    sets = [(OB.PENALTY, 7.0, [0.0, 0.0, 0.0], fe, fi, tg)]
    prm = dict(coef=1.0, nu=0.3)
    levels = MG.build_levels(dims, mesh.coords, 3, O.ELASTICITY, [prm, prm], 2, numbering=numbering,
                             face_sets=sets)
    Af, Ac, P = levels[0]["A"], levels[1]["A"], levels[0]["P"]
    G = (P.T @ Af @ P).toarray()
    ref = Ac.toarray()
    assert np.abs(G - ref).max() <= 1e-12 * np.abs(ref).max()
    # the faces changed the operator (a penalty adds to the face rows)
    plain = MG.build_levels(dims, mesh.coords, 3, O.ELASTICITY, [prm, prm], 2, numbering=numbering)
    assert np.abs(plain[1]["A"].toarray() - ref).max() > 1.0


def test_elimination_gives_unit_rows_and_zero_columns():
    import scipy.sparse as sp
    rng = np.random.default_rng(3)
    A = sp.csr_matrix(rng.standard_normal((6, 6)))
    mask = np.array([0, 1, 0, 0, 1, 0], bool)
    E = MG.eliminate(A, mask).toarray()
    Ad = A.toarray()
    for r in range(6):
        for c in range(6):
            if mask[r] or mask[c]:
                assert E[r, c] == (1.0 if r == c else 0.0)
            else:
                assert E[r, c] == Ad[r, c]


def test_coarse_coefficient_is_the_mean_of_the_children():
    dims = (4, 2, 6)
    v = np.arange(np.prod(dims), dtype=np.float64) ** 1.5
    c = MG.coarsen_elem(dims, v)
    assert c.shape == (6,)  # coarse grid 2 x 1 x 3
    # coarse element (1, 0, 2): fine ex in {2, 3}, ey in {0, 1}, ez in {4, 5}
    kids = [ex + 4 * (ey + 2 * ez) for ex in (2, 3) for ey in (0, 1) for ez in (4, 5)]
    assert c[1 + 2 * (0 + 1 * 2)] == pytest.approx(v[kids].mean(), rel=1e-15)


def test_galerkin_identity_with_a_piecewise_constant_coefficient():
    """A conductivity constant on each coarse element is the same field on both levels, so
    the coarse rediscretisation is P^T A P again."""
    dims = (4, 4, 4)
    mesh = W.structured_mesh(dims, lengths=(1.0, 0.5, 2.0))
    coarse = W.lognormal_elem(8, 1.0, 4)
    ex, ey, ez = np.meshgrid(np.arange(4), np.arange(4), np.arange(4), indexing="ij")
    ex, ey, ez = (a.ravel(order="F") for a in (ex, ey, ez))
    k = coarse[ex // 2 + 2 * (ey // 2 + 2 * (ez // 2))]
    levels = MG.build_levels(dims, mesh.coords, 1, O.POISSON, [dict(coef=1.0)] * 2, 2, elem_param=k)
    G = (levels[0]["P"].T @ levels[0]["A"] @ levels[0]["P"]).toarray()
    ref = levels[1]["A"].toarray()
    assert np.abs(G - ref).max() <= 1e-12 * np.abs(ref).max()
