"""Oracle pins for quadrature, basis, geometry and the three weak forms.

Each check rests on something other than the oracle's own formulas: closed-form
element matrices, exact polynomial integrals, conservation identities, rigid-body
modes, the patch test, manufactured solutions and finite differences.
Weak forms: Sec. 4.1 (thermal), Sec. 4.2 (elasticity); Newton tangent: Sec. 2.1.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O
import workloads as W


# ---------------------------------------------------------------- quadrature / basis

@pytest.mark.parametrize("p", [1, 2, 3])
def test_gauss_exact_to_degree_2p_minus_1(p):
    pts, wts = O.gauss(p)
    for k in range(2 * p):
        exact = 2.0 / (k + 1) if k % 2 == 0 else 0.0
        assert abs(np.sum(wts * pts ** k) - exact) < 1e-14
    # and not exact at degree 2p
    k = 2 * p
    assert abs(np.sum(wts * pts ** k) - 2.0 / (k + 1)) > 1e-6


@pytest.mark.parametrize("dim", [2, 3])
def test_basis_partition_of_unity_and_kronecker(dim):
    rng = np.random.default_rng(0)
    for _ in range(10):
        xi = rng.uniform(-1, 1, dim)
        N, dN = O.basis(dim, xi)
        assert abs(N.sum() - 1.0) < 1e-15
        assert np.max(np.abs(dN.sum(axis=0))) < 1e-15
    for a in range(1 << dim):
        corner = np.array([1.0 if (a >> d) & 1 else -1.0 for d in range(dim)])
        N, _ = O.basis(dim, corner)
        e = np.zeros(1 << dim)
        e[a] = 1.0
        assert np.allclose(N, e, atol=0, rtol=0)
    # derivative vs central difference
    xi = np.array([0.3, -0.2, 0.7][:dim])
    N, dN = O.basis(dim, xi)
    for d in range(dim):
        h = 1e-6
        xp, xm = xi.copy(), xi.copy()
        xp[d] += h
        xm[d] -= h
        fd = (O.basis(dim, xp)[0] - O.basis(dim, xm)[0]) / (2 * h)
        assert np.max(np.abs(fd - dN[:, d])) < 1e-9


# ---------------------------------------------------------------- closed-form elements

def hamming(a, b):
    return bin(a ^ b).count("1")


@pytest.mark.parametrize("h", [1.0, 0.25])
def test_poisson_and_mass_element_closed_forms_2d(h):
    mesh = W.structured_mesh((1, 1), lengths=[h, h])
    pat = O.Pattern(mesh, 1)
    K = pat.to_scipy(O.assemble(pat, O.POISSON, params={"coef": 3.0})[0]).toarray()
    M = pat.to_scipy(O.assemble(pat, O.MASS)[0]).toarray()
    kk = [4.0, -1.0, -2.0]          # (k/6) by Hamming distance, any h
    mm = [4.0, 2.0, 1.0]            # (h^2/36)
    for a in range(4):
        for b in range(4):
            assert abs(K[a, b] - 3.0 / 6.0 * kk[hamming(a, b)]) < 1e-14
            assert abs(M[a, b] - h * h / 36.0 * mm[hamming(a, b)]) < 1e-16


@pytest.mark.parametrize("h", [1.0, 0.5])
def test_poisson_and_mass_element_closed_forms_3d(h):
    mesh = W.structured_mesh((1, 1, 1), lengths=[h, h, h])
    pat = O.Pattern(mesh, 1)
    K = pat.to_scipy(O.assemble(pat, O.POISSON)[0]).toarray()
    M = pat.to_scipy(O.assemble(pat, O.MASS)[0]).toarray()
    kk = [4.0, 0.0, -1.0, -1.0]     # (k h / 12)
    mm = [8.0, 4.0, 2.0, 1.0]       # (h^3 / 216)
    for a in range(8):
        for b in range(8):
            assert abs(K[a, b] - h / 12.0 * kk[hamming(a, b)]) < 1e-15
            assert abs(M[a, b] - h ** 3 / 216.0 * mm[hamming(a, b)]) < 1e-16


def test_bad_jacobian_reports_element():
    mesh = W.structured_mesh((2, 2, 2))
    conn = mesh.conn.copy()
    conn[[0, 1], 5] = conn[[1, 0], 5]  # mirror element 5
    bad = W.Mesh(mesh.coords, conn)
    pat = O.Pattern(bad, 1)
    with pytest.raises(FloatingPointError, match="element 5"):
        O.assemble(pat, O.POISSON)


# ---------------------------------------------------------------- conservation / invariants

@pytest.mark.parametrize("n", [(6, 5), (4, 3, 5)])
def test_mass_sums_to_volume_and_poisson_rows_sum_to_zero(n):
    mesh = W.structured_mesh(n, jitter=0.2, seed=4)
    pat = O.Pattern(mesh, 1)
    M, dm = O.assemble(pat, O.MASS, nodal_src=np.ones((1, mesh.n_nodes)))
    assert abs(M.sum() - 1.0) < 1e-13
    k = W.lognormal_elem(mesh.n_elems, 0.5, 1)
    K, d = O.assemble(pat, O.POISSON, elem_param=k, nodal_src=np.ones((1, mesh.n_nodes)))
    S = pat.to_scipy(K)
    assert np.max(np.abs(S @ np.ones(mesh.n_nodes))) < 1e-13
    assert abs(S - S.T).max() < 1e-15
    assert abs(d.sum() - 1.0) < 1e-13         # f = 1  =>  sum d = volume
    assert np.allclose(dm, d, atol=1e-16, rtol=0)  # both equal M 1


def test_poisson_d_is_mass_times_f():
    mesh = W.structured_mesh((3, 4, 2), jitter=0.15, seed=2)
    pat = O.Pattern(mesh, 1)
    f = W.uniform_nodal(1, mesh.n_nodes, 0, 1, 5)
    M, _ = O.assemble(pat, O.MASS)
    _, d = O.assemble(pat, O.POISSON, nodal_src=f)
    assert np.max(np.abs(pat.to_scipy(M) @ f[0] - d)) < 1e-15


# ---------------------------------------------------------------- elasticity

def lame(E, nu):
    # from Young's modulus and Poisson's ratio (isotropic elasticity textbook relations)
    return E * nu / ((1 + nu) * (1 - 2 * nu)), E / (2 * (1 + nu))


def test_elasticity_single_cube_uniaxial_stress():
    """u = (eps x, -nu eps y, -nu eps z) is a uniaxial stress state sigma = E eps e1 e1.
    For one cube of side h, K u at node a equals sigma . int grad N_a = sigma s_a h^2 / 4."""
    h, E, nu, eps = 0.5, 7.0, 0.3, 1e-2
    mesh = W.structured_mesh((1, 1, 1), lengths=[h, h, h])
    pat = O.Pattern(mesh, 3)
    K = pat.to_scipy(O.assemble(pat, O.ELASTICITY, params={"coef": E, "nu": nu})[0])
    x = mesh.coords
    u = np.stack([eps * x[0], -nu * eps * x[1], -nu * eps * x[2]])  # [3][8]
    f = K @ u.T.reshape(-1)
    for a in range(8):
        s = np.array([1.0 if (a >> d) & 1 else -1.0 for d in range(3)])
        expect = np.array([E * eps * s[0], 0.0, 0.0]) * h * h / 4
        assert np.max(np.abs(f[3 * a:3 * a + 3] - expect)) < 1e-13


def test_elasticity_single_cube_shear():
    """Pure shear u = (g y, 0, 0): sigma_12 = sigma_21 = mu g (mu = E / (2(1+nu)))."""
    h, E, nu, gam = 1.0, 2.0, 0.25, 1e-2
    mesh = W.structured_mesh((1, 1, 1), lengths=[h, h, h])
    pat = O.Pattern(mesh, 3)
    K = pat.to_scipy(O.assemble(pat, O.ELASTICITY, params={"coef": E, "nu": nu})[0])
    x = mesh.coords
    u = np.stack([gam * x[1], 0 * x[1], 0 * x[1]])
    f = K @ u.T.reshape(-1)
    mu = E / (2 * (1 + nu))
    for a in range(8):
        s = np.array([1.0 if (a >> d) & 1 else -1.0 for d in range(3)])
        sig = np.zeros((3, 3))
        sig[0, 1] = sig[1, 0] = mu * gam
        assert np.max(np.abs(f[3 * a:3 * a + 3] - sig @ s * h * h / 4)) < 1e-14


def rigid_modes(coords):
    x, y, z = coords
    one, zero = np.ones_like(x), np.zeros_like(x)
    modes = [
        (one, zero, zero), (zero, one, zero), (zero, zero, one),
        (-y, x, zero), (zero, -z, y), (z, zero, -x),
    ]
    return [np.stack(m).T.reshape(-1) for m in modes]  # node-major


def test_elasticity_rigid_body_modes_symmetry_and_patch():
    mesh = W.structured_mesh((4, 3, 3), jitter=0.2, seed=7)
    pat = O.Pattern(mesh, 3)
    E = W.lognormal_elem(mesh.n_elems, 0.5, 3)
    K, _ = O.assemble(pat, O.ELASTICITY, params={"coef": 1.0, "nu": 0.3}, elem_param=E)
    S = pat.to_scipy(K)
    scale = np.abs(K).max()
    assert abs(S - S.T).max() < 1e-14 * scale
    for r in rigid_modes(mesh.coords):
        assert np.max(np.abs(S @ r)) < 1e-13 * scale
    # patch test: linear displacement => interior rows balance (piecewise-constant E is
    # not allowed here: the traction jump would be a real force), so use uniform E
    K1, _ = O.assemble(pat, O.ELASTICITY, params={"coef": 1.0, "nu": 0.3})
    S1 = pat.to_scipy(K1)
    A = np.array([[0.3, -0.1, 0.2], [0.05, 0.4, -0.3], [0.1, 0.2, -0.25]])
    u = (A @ mesh.coords).T.reshape(-1)
    f = (S1 @ u).reshape(-1, 3)
    interior = W.boundary_node_mask(mesh.shape) == 0
    assert np.max(np.abs(f[interior])) < 1e-15
    # and positive semidefinite: x^T K x >= 0
    rng = np.random.default_rng(1)
    for _ in range(5):
        v = rng.standard_normal(S.shape[0])
        assert v @ (S @ v) > 0


# ---------------------------------------------------------------- manufactured solutions

def solve_dirichlet(S, d, mask):
    free = np.nonzero(mask == 0)[0]
    u = np.zeros(S.shape[0])
    Sff = S[free][:, free].tocsc()
    u[free] = spla.spsolve(Sff, d[free])
    return u


@pytest.mark.parametrize("dim,ns", [(2, [8, 16, 32]), (3, [4, 8, 16])])
def test_poisson_manufactured_solution_second_order(dim, ns):
    errs = []
    for n in ns:
        mesh = W.structured_mesh((n,) * dim)
        pat = O.Pattern(mesh, 1)
        x = mesh.coords
        uex = np.prod(np.sin(np.pi * x), axis=0)
        f = dim * np.pi ** 2 * uex
        mask = W.boundary_node_mask(mesh.shape)
        K, d = O.assemble(pat, O.POISSON, nodal_src=f[None], dirichlet=mask)
        u = np.linalg.solve(pat.to_scipy(K).toarray(), d) if pat.n_rows < 400 else \
            spla.spsolve(pat.to_scipy(K).tocsc(), d)
        errs.append(np.max(np.abs(u - uex)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.8), (errs, rates)


def test_elasticity_manufactured_solution_second_order():
    E, nu = 1.0, 0.3
    lam, mu = lame(E, nu)
    pi = np.pi
    errs = []
    for n in [4, 8, 16]:
        mesh = W.structured_mesh((n, n, n))
        pat = O.Pattern(mesh, 3)
        x, y, z = mesh.coords
        s = np.sin(pi * mesh.coords)
        c = np.cos(pi * mesh.coords)
        phi = s[0] * s[1] * s[2]
        # u_i = phi for all i;  b = -div sigma = -(lam+mu) grad(div u) - mu lap u
        hess = np.empty((3, 3, mesh.n_nodes))
        for i in range(3):
            for k in range(3):
                if i == k:
                    hess[i, k] = -pi ** 2 * phi
                else:
                    m = 3 - i - k
                    hess[i, k] = pi ** 2 * c[i] * c[k] * s[m]
        b = np.stack([-(lam + mu) * hess[i].sum(axis=0) + 3 * mu * pi ** 2 * phi for i in range(3)])
        nmask = W.boundary_node_mask(mesh.shape)
        mask = W.dof_mask(nmask, 3, field_major=False)
        K, d = O.assemble(pat, O.ELASTICITY, params={"coef": E, "nu": nu}, nodal_src=b, dirichlet=mask)
        u = spla.spsolve(pat.to_scipy(K).tocsc(), d).reshape(-1, 3)
        errs.append(np.max(np.abs(u - phi[:, None])))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.7), (errs, rates)


# ---------------------------------------------------------------- Newton tangent = dR/dU

@pytest.mark.parametrize("kind,nf,params", [
    (O.POISSON, 1, {"coef": 2.0}),
    (O.MASS, 1, {"coef": 1.5}),
    (O.ELASTICITY, 3, {"coef": 3.0, "nu": 0.28}),
])
def test_linear_forms_tangent_is_jacobian_of_residual(kind, nf, params):
    mesh = W.structured_mesh((2, 2, 1), jitter=0.2, seed=9)
    pat = O.Pattern(mesh, nf)
    ep = W.lognormal_elem(mesh.n_elems, 0.5, 2)
    src = W.uniform_nodal(3 if kind == O.ELASTICITY else 1, mesh.n_nodes, -1, 1, 3)
    K, d = O.assemble(pat, kind, params, elem_param=ep, nodal_src=src)
    S = pat.to_scipy(K).toarray()
    R0 = O.residual(pat, kind, params, elem_param=ep, nodal_src=src)
    assert np.max(np.abs(R0 + d)) < 1e-15
    rng = np.random.default_rng(0)
    U = rng.standard_normal((nf, mesh.n_nodes))
    RU = O.residual(pat, kind, params, elem_param=ep, nodal_src=src, state=U)
    # linear forms: R(U) = K U - d exactly (node-major state vector)
    assert np.max(np.abs(RU - (S @ U.T.reshape(-1) - d))) < 1e-13


# ---------------------------------------------------------------- Dirichlet elimination

def test_dirichlet_elimination_structure():
    mesh = W.structured_mesh((4, 3))
    pat = O.Pattern(mesh, 1)
    mask = W.boundary_node_mask(mesh.shape)
    f = W.uniform_nodal(1, mesh.n_nodes, 0, 1, 1)
    K0, d0 = O.assemble(pat, O.POISSON, nodal_src=f)
    K, d = O.assemble(pat, O.POISSON, nodal_src=f, dirichlet=mask)
    S, S0 = pat.to_scipy(K).toarray(), pat.to_scipy(K0).toarray()
    for r in range(pat.n_rows):
        if mask[r]:
            e = np.zeros(pat.n_rows)
            e[r] = 1.0
            assert np.array_equal(S[r], e) and np.array_equal(S[:, r], e) and d[r] == 0.0
        else:
            assert d[r] == d0[r]
            for c in range(pat.n_rows):
                assert S[r, c] == (0.0 if mask[c] else S0[r, c])


# ---------------------------------------------------------------- CG oracle

def test_pcg_jacobi_matches_direct_solve():
    n = 32
    mesh = W.structured_mesh((n, n))
    pat = O.Pattern(mesh, 1)
    f = W.uniform_nodal(1, mesh.n_nodes, 0, 1, 1)
    mask = W.boundary_node_mask(mesh.shape)
    K, d = O.assemble(pat, O.POISSON, nodal_src=f, dirichlet=mask)
    x, it, rel = O.pcg_jacobi(pat.row_ptr, pat.col_idx, K, d, tol=1e-10)
    ref = spla.spsolve(pat.to_scipy(K).tocsc(), d)
    assert it > 0 and rel <= 1e-10
    assert np.max(np.abs(x - ref)) < 1e-9 * np.max(np.abs(ref))
    # maxit reached -> -1 and the true residual of the last iterate
    _, it2, rel2 = O.pcg_jacobi(pat.row_ptr, pat.col_idx, K, d, tol=1e-10, maxit=3)
    assert it2 == -1 and rel2 > 1e-10


def test_colour_parallel_assembly_matches_sequential():
    """The all-core oracle (element colour by colour on OpenMP threads) against the
    sequential one on a jittered elasticity mesh and a flow Jacobian: same K and d up to
    the order of the at most 8 contributions per entry."""
    import os
    from helpers import rowscaled_error, vec_error
    threads = max(1, min(8, len(os.sched_getaffinity(0))))
    for kind, nf, n in ((O.ELASTICITY, 3, (9, 7, 6)), (O.NS_SUPG, 4, (5, 4, 4))):
        mesh = W.structured_mesh(n, jitter=0.15, seed=3)
        pat = O.Pattern(mesh, nf)
        if kind == O.ELASTICITY:
            kw = dict(params={"coef": 1.0, "nu": 0.3}, elem_param=W.lognormal_elem(mesh.n_elems, 0.5, 1),
                      nodal_src=W.uniform_nodal(3, mesh.n_nodes, -1, 1, 2))
        else:
            st = np.vstack([W.fourier_velocity(mesh.coords, 4), W.uniform_nodal(1, mesh.n_nodes, -0.5, 0.5, 5)])
            kw = dict(params={"rho": 1.0, "mu": 0.01, "tau_m": 0.02, "tau_c": 0.05}, state=st)
        K1, d1 = O.assemble(pat, kind, **kw)
        K2, d2, used = O.assemble_parallel(pat, kind, threads=threads, **kw)
        assert used == threads
        assert rowscaled_error(pat, K2, K1) <= 1e-13 and vec_error(d2, d1) <= 1e-13
