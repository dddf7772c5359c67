"""Oracle pins for the flow form on quadratic elements (oracle/serendipity.py, ns_element):
moments of the residual against the weak form evaluated with an independent quadrature
of the analytic fields, Poiseuille flow as an exact discrete solution, the tangent against
central differences of the residual, and the zero-state blocks against the conduction
matrix (itself pinned by the patch tests)."""
import numpy as np
import pytest

import oracle as O
import oracle.serendipity as S
import workloads as W

PRM = {"rho": 1.3, "mu": 0.7, "tau_m": 0.11, "tau_c": 0.23}


def flow_mesh(kind, n, jitter=0.0, seed=0):
    if kind == "hex20":
        return W.serendipity_mesh(n, jitter=jitter, seed=seed)
    if kind == "quad8":
        return W.serendipity_mesh_2d(n[:2], jitter=jitter, seed=seed)
    return W.tet10_mesh(n, jitter=jitter, seed=seed)


def fields(x, dim):
    """Velocity u [dim], its gradient gu[i][k] = du_i/dx_k and the pressure p at x: each a
    polynomial that every quadratic element space here holds exactly."""
    if dim == 3:
        X, Y, Z = x
        u = np.array([0.4 + 0.7 * Y - 0.3 * Z + 0.5 * X * X,
                      0.2 - 0.6 * X + 0.4 * Z + 0.3 * Y * Z,
                      -0.1 + 0.3 * X - 0.2 * Y + 0.25 * Y * Y])
        gu = np.array([[X, 0.7, -0.3],
                       [-0.6, 0.3 * Z, 0.4 + 0.3 * Y],
                       [0.3, -0.2 + 0.5 * Y, 0.0]])
        p = 0.5 - 0.8 * X + 0.3 * Y * Z
        gp = np.array([-0.8, 0.3 * Z, 0.3 * Y])
    else:
        X, Y = x
        u = np.array([0.4 + 0.7 * Y + 0.5 * X * X, 0.2 - 0.6 * X + 0.3 * X * Y])
        gu = np.array([[X, 0.7], [-0.6 + 0.3 * Y, 0.3 * X]])
        p = 0.5 - 0.8 * X + 0.3 * X * Y
        gp = np.array([-0.8 + 0.3 * Y, 0.3 * X])
    return u, gu, p, gp


def weak_form_moments(dim, prm, npts=6):
    """With the test function x_k e_i (velocity rows) or x_k, 1 (pressure rows), whose
    gradients are constants, the flow residual of Sec. 4.3 reduces to integrals of the
    fields alone.  Evaluated on the unit box with a 6-point Gauss product rule, far above
    the polynomial degrees involved.  Returns (M_u[k][i], M_p[k], S_p)."""
    rho, mu, tm, tc = prm["rho"], prm["mu"], prm["tau_m"], prm["tau_c"]
    t, w = np.polynomial.legendre.leggauss(npts)
    t, w = 0.5 * (t + 1.0), 0.5 * w
    Mu = np.zeros((dim, dim))
    Mp = np.zeros(dim)
    Sp = 0.0
    grids = np.meshgrid(*([np.arange(npts)] * dim), indexing="ij")
    for idx in zip(*(g.ravel() for g in grids)):
        x = t[list(idx)]
        wq = np.prod(w[list(idx)])
        u, gu, p, gp = fields(x, dim)
        div = np.trace(gu)
        Rm = rho * gu @ u + gp
        for k in range(dim):
            for i in range(dim):
                # grad(x_k) = e_k: convection, pressure, viscous, SUPG and LSIC terms
                Mu[k, i] += wq * (-rho * u[k] * u[i] - (k == i) * p + mu * gu[i, k]
                                  + tm * rho * u[k] * Rm[i] + tc * (k == i) * div)
            Mp[k] += wq * (x[k] * div + tm * Rm[k])
        Sp += wq * div
    return Mu, Mp, Sp


def nodal_state(mesh, f):
    dim = mesh.dim
    st = np.zeros((dim + 1, mesh.n_nodes))
    for v in range(mesh.n_nodes):
        u, _, p, _ = f(mesh.coords[:, v], dim)
        st[:dim, v], st[dim, v] = u, p
    return st


def rows_of(pat, i):
    return np.array([pat.dof(v, i) for v in range(pat.mesh.n_nodes)])


@pytest.mark.parametrize("kind,n,jitter", [("hex20", (2, 2, 1), 0.0), ("quad8", (3, 2, 1), 0.0),
                                           ("tet10", (2, 1, 1), 0.2)])
def test_flow_residual_moments_match_the_weak_form(kind, n, jitter):
    mesh = flow_mesh(kind, n, jitter, seed=2)
    dim = mesh.dim
    pat = S.Pattern20(mesh, dim + 1)
    st = nodal_state(mesh, fields)
    _, d = S.assemble20(pat, O.NS_SUPG, PRM, state=st)
    R = -d
    Mu, Mp, Sp = weak_form_moments(dim, PRM)
    X = mesh.coords
    scale = np.abs(Mu).max()
    for i in range(dim):
        Ri = R[rows_of(pat, i)]
        assert abs(Ri.sum()) < 1e-13 * scale  # constant test function: every term has grad N
        for k in range(dim):
            assert abs(X[k] @ Ri - Mu[k, i]) < 1e-12 * scale, (k, i)
    Rp = R[rows_of(pat, dim)]
    assert abs(Rp.sum() - Sp) < 1e-13 * scale
    for k in range(dim):
        assert abs(X[k] @ Rp - Mp[k]) < 1e-12 * scale, k


def poiseuille(x, dim, mu=PRM["mu"]):
    """u = (y (1 - y), 0[, 0]), p = 1 - 2 mu x: a steady solution of the incompressible
    Navier-Stokes equations (u . grad u = 0, mu lap u = grad p, div u = 0)."""
    u = np.zeros(dim)
    u[0] = x[1] * (1.0 - x[1])
    return u, None, 1.0 - 2.0 * mu * x[0], None


@pytest.mark.parametrize("kind,n,jitter", [("hex20", (3, 3, 2), 0.0), ("quad8", (4, 3, 1), 0.0),
                                           ("tet10", (2, 2, 2), 0.2)])
def test_poiseuille_flow_is_an_exact_discrete_solution(kind, n, jitter):
    # Galerkin terms with LSIC (tau_m = 0: the SUPG/PSPG residual leaves out mu lap u)
    mesh = flow_mesh(kind, n, jitter, seed=3)
    dim = mesh.dim
    pat = S.Pattern20(mesh, dim + 1)
    st = nodal_state(mesh, poiseuille)
    prm = dict(PRM, tau_m=0.0)
    _, d = S.assemble20(pat, O.NS_SUPG, prm, state=st)
    c = mesh.coords
    interior = np.all((c > 1e-12) & (c < 1 - 1e-12), axis=0)
    for i in range(dim):
        assert np.abs(d[rows_of(pat, i)][interior]).max() < 1e-13
    # the viscous rows alone do not vanish: the pressure gradient balances them
    st_nop = st.copy()
    st_nop[dim] = 0.0
    _, d_visc = S.assemble20(pat, O.NS_SUPG, prm, state=st_nop)
    assert np.abs(d_visc[rows_of(pat, 0)][interior]).max() > 1e-3
    assert np.abs(d[rows_of(pat, dim)]).max() < 1e-14  # div u = 0 in every element


@pytest.mark.parametrize("kind,n", [("hex20", (2, 1, 1)), ("quad8", (2, 2, 1)), ("tet10", (1, 1, 1))])
@pytest.mark.parametrize("numbering", [O.NODE_MAJOR, O.FIELD_MAJOR])
def test_flow_tangent_is_the_derivative_of_the_residual(kind, n, numbering):
    mesh = flow_mesh(kind, n, 0.2, seed=4)
    dim = mesh.dim
    pat = S.Pattern20(mesh, dim + 1, numbering)
    rng = np.random.default_rng(5)
    st = rng.uniform(-1.0, 1.0, (dim + 1, mesh.n_nodes))
    K, _ = S.assemble20(pat, O.NS_SUPG, PRM, state=st)
    Km = pat.to_scipy(K)
    h = 1e-6
    for _ in range(3):
        v = rng.uniform(-1.0, 1.0, st.shape)
        vr = np.zeros(pat.n_rows)
        for i in range(dim + 1):
            vr[rows_of(pat, i)] = v[i]
        dp = S.assemble20(pat, O.NS_SUPG, PRM, state=st + h * v)[1]
        dm = S.assemble20(pat, O.NS_SUPG, PRM, state=st - h * v)[1]
        fd = -(dp - dm) / (2.0 * h)  # d = -R
        Kv = Km @ vr
        assert np.abs(Kv - fd).max() < 1e-7 * np.abs(Kv).max()


@pytest.mark.parametrize("kind,n", [("hex20", (2, 1, 1)), ("quad8", (3, 2, 1)), ("tet10", (1, 1, 1))])
def test_flow_blocks_at_rest_reduce_to_conduction(kind, n):
    mesh = flow_mesh(kind, n, 0.2, seed=6)
    dim = mesh.dim
    pat = S.Pattern20(mesh, dim + 1)
    Km = pat.to_scipy(S.assemble20(pat, O.NS_SUPG, dict(PRM, tau_c=0.0))[0]).toarray()
    pat1 = S.Pattern20(mesh, 1)
    L = pat1.to_scipy(S.assemble20(pat1, O.POISSON, {"coef": 1.0})[0]).toarray()
    r = [rows_of(pat, i) for i in range(dim + 1)]
    scale = np.abs(L).max()
    # at rest: mu L on the velocity diagonal blocks, nothing between velocity components,
    # tau_m L on the pressure block, and the divergence pair B, -B^T
    for i in range(dim):
        for l in range(dim):
            want = PRM["mu"] * L if i == l else 0.0 * L
            assert np.abs(Km[np.ix_(r[i], r[l])] - want).max() < 1e-13 * scale
        assert np.abs(Km[np.ix_(r[i], r[dim])] + Km[np.ix_(r[dim], r[i])].T).max() < 1e-13 * scale
    assert np.abs(Km[np.ix_(r[dim], r[dim])] - PRM["tau_m"] * L).max() < 1e-13 * scale
