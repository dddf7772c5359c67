"""Oracle pins for the stabilised steady Navier-Stokes form (Sec. 4.3) and its Newton
tangent (Sec. 2.1, Eqs. Newton-Raphson and stiffness).

The residual is pinned term by term, by states whose integrals are known in closed form:
  * one cube element of side h: for a constant c, int c dN_a/dx_i = c s_{a,i} h^2 / 4;
  * interior nodes of a uniform grid: integration by parts moves the derivative from the
    test function onto a polynomial field; int N_a L = L(x_a) h^3 for a linear L.
The tangent is then pinned to the residual by central differences.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W


def corner_signs():
    return np.array([[1.0 if (a >> d) & 1 else -1.0 for d in range(3)] for a in range(8)])


def single_cube(h):
    mesh = W.structured_mesh((1, 1, 1), lengths=[h, h, h])
    return mesh, O.Pattern(mesh, 4)


def R_of(pat, state, **prm):
    return O.residual(pat, O.NS_SUPG, params=prm, state=state).reshape(-1, 4)  # node-major


def test_zero_state_zero_residual():
    mesh, pat = single_cube(0.3)
    R = R_of(pat, np.zeros((4, 8)), rho=1.0, mu=0.1, tau_m=0.2, tau_c=0.3)
    assert np.all(R == 0.0)


def test_pressure_term_and_continuity_term():
    h, P = 0.5, 1.7
    mesh, pat = single_cube(h)
    st = np.zeros((4, 8))
    st[3] = P
    R = R_of(pat, st, rho=1.3, mu=0.2, tau_m=0.3, tau_c=0.4)
    s = corner_signs()
    # -(u_{i,i}, p) -> -P s_ai h^2/4 ; continuity and PSPG vanish (div u = 0, grad p = 0)
    assert np.max(np.abs(R[:, :3] + P * s * h * h / 4)) < 1e-15
    assert np.max(np.abs(R[:, 3])) < 1e-15
    # linear velocity: (p, u_{i,i}) = tr(A) int N_a = tr(A) h^3 / 8
    A = np.array([[0.2, 0.1, 0.0], [0.3, -0.4, 0.2], [0.1, 0.0, 0.5]])
    st = np.zeros((4, 8))
    st[:3] = A @ mesh.coords
    R = R_of(pat, st, rho=0.0, mu=0.0, tau_m=0.0, tau_c=0.0)
    assert np.max(np.abs(R[:, 3] - np.trace(A) * h ** 3 / 8)) < 1e-15


def test_viscous_and_grad_div_terms():
    h, mu, tc = 0.5, 0.7, 0.45
    mesh, pat = single_cube(h)
    A = np.array([[0.2, 0.1, -0.3], [0.3, -0.4, 0.2], [0.1, 0.25, 0.5]])
    st = np.zeros((4, 8))
    st[:3] = A @ mesh.coords
    s = corner_signs()
    R = R_of(pat, st, rho=0.0, mu=mu, tau_m=0.0, tau_c=0.0)
    # mu (u_{i,j}, u_{i,j}) -> mu A_ij s_aj h^2/4
    assert np.max(np.abs(R[:, :3] - mu * (s @ A.T) * h * h / 4)) < 1e-15
    R2 = R_of(pat, st, rho=0.0, mu=0.0, tau_m=0.0, tau_c=tc)
    # tau_c (u_{i,i}, Rc) -> tau_c tr(A) s_ai h^2/4
    assert np.max(np.abs(R2[:, :3] - tc * np.trace(A) * s * h * h / 4)) < 1e-15


def test_convection_and_pressure_stabilisation_single_element():
    h, rho, tm = 0.5, 1.4, 0.3
    mesh, pat = single_cube(h)
    U0 = np.array([0.3, -0.5, 0.8])
    c = np.array([0.2, 0.7, -0.4])
    s = corner_signs()
    st = np.zeros((4, 8))
    st[:3] = U0[:, None]
    R = R_of(pat, st, rho=rho, mu=0.9, tau_m=tm, tau_c=0.6)
    # -rho (u_{i,j}, u_i u_j) -> -rho (U0 . s_a) U0_i h^2/4 ; Rm = 0 for constant u, p = 0
    expect = -rho * (s @ U0)[:, None] * U0[None, :] * h * h / 4
    assert np.max(np.abs(R[:, :3] - expect)) < 1e-15
    # with a linear pressure Rm = grad p = c: the tau_m parts are
    #   tau_m rho (u_{i,j}, Rm_i u_j) -> tau_m rho (U0 . s_a) c_i h^2/4
    #   tau_m (p_{,i}, Rm_i)          -> tau_m (c . s_a) h^2/4
    st[3] = c @ mesh.coords
    R1 = R_of(pat, st, rho=rho, mu=0.9, tau_m=tm, tau_c=0.6)
    R0 = R_of(pat, st, rho=rho, mu=0.9, tau_m=0.0, tau_c=0.6)
    d = R1 - R0
    assert np.max(np.abs(d[:, :3] - tm * rho * (s @ U0)[:, None] * c[None, :] * h * h / 4)) < 1e-15
    assert np.max(np.abs(d[:, 3] - tm * (s @ c) * h * h / 4)) < 1e-15


def test_convective_parts_by_integration_by_parts_on_interior_nodes():
    """u = A x with tr A = 0, p = 0, mu = tau_c = 0, uniform grid of spacing h.
    For an interior node a:  R_u = rho h^3 (A^2 x_a) - tau_m rho^2 h^3 (A^3 x_a),
                             R_p = -tau_m rho tr(A^2) h^3."""
    n = 4
    h = 1.0 / n
    rho, tm = 1.3, 0.25
    mesh = W.structured_mesh((n, n, n))
    pat = O.Pattern(mesh, 4)
    A = np.array([[0.3, 0.2, -0.1], [0.4, -0.5, 0.3], [-0.2, 0.1, 0.2]])
    st = np.zeros((4, mesh.n_nodes))
    st[:3] = A @ mesh.coords
    R = R_of(pat, st, rho=rho, mu=0.0, tau_m=tm, tau_c=0.0)
    interior = W.boundary_node_mask(mesh.shape) == 0
    x = mesh.coords[:, interior]
    A2, A3 = A @ A, A @ A @ A
    expect_u = rho * h ** 3 * (A2 @ x) - tm * rho ** 2 * h ** 3 * (A3 @ x)
    assert np.max(np.abs(R[interior, :3] - expect_u.T)) < 1e-15
    assert np.max(np.abs(R[interior, 3] + tm * rho * np.trace(A2) * h ** 3)) < 1e-15


def test_tangent_matches_central_differences():
    mesh = W.structured_mesh((2, 2, 1), jitter=0.2, seed=3)
    pat = O.Pattern(mesh, 4)
    prm = dict(rho=1.2, mu=0.05, tau_m=0.3, tau_c=0.2)
    rng = np.random.default_rng(5)
    st = rng.uniform(-1, 1, (4, mesh.n_nodes))
    K, d = O.assemble(pat, O.NS_SUPG, prm, state=st)
    S = pat.to_scipy(K).toarray()
    R0 = O.residual(pat, O.NS_SUPG, prm, state=st)
    assert np.max(np.abs(R0 + d)) < 1e-15
    eps = 1e-5
    J = np.zeros_like(S)
    for col in range(pat.n_rows):
        node, f = divmod(col, 4)
        sp, sm = st.copy(), st.copy()
        sp[f, node] += eps
        sm[f, node] -= eps
        J[:, col] = (O.residual(pat, O.NS_SUPG, prm, state=sp) -
                     O.residual(pat, O.NS_SUPG, prm, state=sm)) / (2 * eps)
    assert np.max(np.abs(J - S)) < 1e-8 * np.max(np.abs(S))
    # entries outside the element coupling are structurally present and exactly zero
    # only where the pattern says so; every Jacobian entry must sit in the pattern
    mask = pat.to_scipy(np.ones(pat.nnz)).toarray()
    assert np.max(np.abs(J * (1 - mask))) < 1e-9


def test_structure_at_zero_velocity():
    mesh = W.structured_mesh((3, 2, 2), jitter=0.15, seed=8)
    pat = O.Pattern(mesh, 4)
    pat1 = O.Pattern(mesh, 1)
    L = pat1.to_scipy(O.assemble(pat1, O.POISSON)[0]).toarray()
    mu, tm = 0.07, 0.4
    st = np.zeros((4, mesh.n_nodes))
    # a nonzero pressure leaves K_up, K_pu and K_pp alone but enters K_uu through
    # Rm = grad p in the SUPG term, so K_uu is checked at p = 0
    st[3] = W.uniform_nodal(1, mesh.n_nodes, -1, 1, 2)[0]
    K, _ = O.assemble(pat, O.NS_SUPG, dict(rho=1.0, mu=mu, tau_m=tm, tau_c=0.0), state=st)
    K0, _ = O.assemble(pat, O.NS_SUPG, dict(rho=1.0, mu=mu, tau_m=tm, tau_c=0.0),
                       state=np.zeros_like(st))
    S0 = pat.to_scipy(K0).toarray()
    S = pat.to_scipy(K).toarray()
    nn = mesh.n_nodes
    u_idx = np.array([4 * v + i for v in range(nn) for i in range(3)])
    p_idx = np.arange(nn) * 4 + 3
    Kuu = S0[np.ix_(u_idx, u_idx)]
    Kup = S[np.ix_(u_idx, p_idx)]
    Kpu = S[np.ix_(p_idx, u_idx)]
    Kpp = S[np.ix_(p_idx, p_idx)]
    assert np.max(np.abs(Kup + Kpu.T)) < 1e-15
    assert np.max(np.abs(Kuu - mu * np.kron(L, np.eye(3)))) < 1e-15
    assert np.max(np.abs(Kpp - tm * L)) < 1e-15
