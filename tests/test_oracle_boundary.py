"""Oracle pins for the boundary forms (Sec. 2.2: the physics one dimension lower; forms of
Sec. 4.1 and Sec. 4.2), computed by oracle/boundary.py."""
import numpy as np
import pytest

import oracle as O
import oracle.boundary as OB
import workloads as W


def box(n, jitter=0.0, lengths=None, seed=1):
    mesh = W.structured_mesh(n, jitter=jitter, seed=seed, lengths=lengths)
    return mesh


def test_face_mass_sums_to_area_and_matches_flat_face():
    mesh = box((3, 2, 4), jitter=0.2, lengths=[2.0, 3.0, 5.0])
    pat = O.Pattern(mesh, 1)
    fe, fi = W.box_faces((3, 2, 4))
    K, d = OB.assemble_boundary(pat, OB.PENALTY, 1.0, [0.0], fe, fi)
    area = 2 * (2 * 3 + 3 * 5 + 2 * 5)
    assert abs(K.sum() - area) < 1e-12 * area
    assert np.abs(d).max() == 0.0
    # one face of the top side: (h_x h_y / 36) [4, 2, 2, 1] between its corners
    pat3 = O.Pattern(mesh, 3)
    fe, fi = W.box_faces((3, 2, 4), sides=[5])
    K1, _ = OB.assemble_boundary(pat, OB.PENALTY, 1.0, [0.0], fe[:1], fi[:1])
    hx, hy = 2.0 / 3, 3.0 / 2
    nodes = mesh.conn[4:, fe[0]]  # top face nodes of the element
    B = K1.toarray()[np.ix_(nodes, nodes)]
    ref = hx * hy / 36 * np.array([[4, 2, 2, 1], [2, 4, 1, 2], [2, 1, 4, 2], [1, 2, 2, 4]])
    assert np.abs(B - ref).max() < 1e-15
    # vector form: the same block on each field, no coupling between fields
    K3, _ = OB.assemble_boundary(pat3, OB.PENALTY, 2.0, [0, 0, 0], *W.box_faces((3, 2, 4)))
    assert abs(K3.sum() - 3 * 2.0 * area) < 1e-12 * area
    rows, cols = K3.nonzero()
    assert np.all(rows % 3 == cols % 3)


def test_traction_integrates_to_load_times_area():
    n = (3, 3, 2)
    mesh = box(n, jitter=0.15, lengths=[1.0, 2.0, 0.5])
    pat = O.Pattern(mesh, 3)
    S = np.array([[0.3, -0.2, 0.7], [0.1, 0.5, -0.4], [0.6, 0.2, -1.1]])
    # closed surface: sum of n dS vanishes, so a uniform stress load sums to zero
    _, d = OB.assemble_boundary(pat, OB.TRACTION, 1.0, S.reshape(-1), *W.box_faces(n))
    assert np.abs(d.reshape(-1, 3).sum(axis=0)).max() < 1e-14
    # the top face alone (n = +z, area 1 x 2): the load is sigma^l e_z times the area
    _, d = OB.assemble_boundary(pat, OB.TRACTION, 1.0, S.reshape(-1), *W.box_faces(n, sides=[5]))
    assert np.abs(d.reshape(-1, 3).sum(axis=0) - S[:, 2] * 2.0).max() < 1e-14
    # the left face (n = -x, area 2 x 0.5)
    _, d = OB.assemble_boundary(pat, OB.TRACTION, 1.0, S.reshape(-1), *W.box_faces(n, sides=[0]))
    assert np.abs(d.reshape(-1, 3).sum(axis=0) + S[:, 0] * 1.0).max() < 1e-14


def test_convection_and_penalty_target_loads():
    n = (2, 3, 2)
    mesh = box(n, jitter=0.2)
    pat = O.Pattern(mesh, 1)
    _, d = OB.assemble_boundary(pat, OB.CONVECTION, 3.0, [2.5], *W.box_faces(n))
    assert abs(d.sum() - 3.0 * 2.5 * 6.0) < 1e-12
    # penalty towards g = z: the top face (z = 1) loads beta * area, the bottom nothing
    g = mesh.coords[2][None, :].copy()
    _, d = OB.assemble_boundary(pat, OB.PENALTY, 4.0, [0.0], *W.box_faces(n, sides=[5]), target=g)
    assert abs(d.sum() - 4.0) < 1e-12
    _, d = OB.assemble_boundary(pat, OB.PENALTY, 4.0, [0.0], *W.box_faces(n, sides=[4]), target=g)
    assert np.abs(d).max() < 1e-15


@pytest.mark.parametrize("numbering", [O.NODE_MAJOR, O.FIELD_MAJOR])
def test_flux_term_makes_linear_fields_exact(numbering):
    """Divergence theorem: int grad N_a . grad T = int_boundary N_a n . grad T for linear T,
    exactly under the Gauss rules on trilinear maps; so (domain + flux) T_lin = 0, and with
    the penalty towards T_lin the linear field solves the fix problem for any penalty."""
    n = (3, 2, 3)
    mesh = box(n, jitter=0.2, lengths=[1.5, 1.0, 2.0], seed=3)
    pat = O.Pattern(mesh, 1, numbering=numbering)
    k = 1.7
    Kd, _ = O.assemble(pat, O.POISSON, {"coef": k})
    Kd = pat.to_scipy(Kd)
    Kf, _ = OB.assemble_boundary(pat, OB.FLUX, k, [0.0], *W.box_faces(n))
    T = 0.3 * mesh.coords[0] - 1.2 * mesh.coords[1] + 0.7 * mesh.coords[2] + 0.4
    assert np.abs((Kd + Kf) @ T).max() < 1e-13 * np.abs(Kd @ T).max()
    # the flux residual at a state is linear: d = -K T
    _, dflux = OB.assemble_boundary(pat, OB.FLUX, k, [0.0], *W.box_faces(n), state=T[None, :])
    assert np.abs(dflux + Kf @ T).max() < 1e-14
    # fix problem: domain + flux + penalty towards T: T is the exact discrete solution
    Kp, dp = OB.assemble_boundary(pat, OB.PENALTY, 1e3, [0.0], *W.box_faces(n), target=T[None, :])
    assert np.abs((Kd + Kf + Kp) @ T - dp).max() < 1e-11 * np.abs(dp).max()


def test_radiation_tangent_by_central_differences():
    n = (2, 2, 2)
    mesh = box(n, jitter=0.2, seed=5)
    pat = O.Pattern(mesh, 1)
    fe, fi = W.box_faces(n)
    rng = np.random.default_rng(2)
    T = 1.0 + rng.random(mesh.n_nodes)
    c, Te = 0.8, 1.3
    K, d = OB.assemble_boundary(pat, OB.RADIATION, c, [Te], fe, fi, state=T[None, :])
    K = K.toarray()
    eps = 1e-5
    for j in rng.choice(mesh.n_nodes, 6, replace=False):
        e = np.zeros(mesh.n_nodes)
        e[j] = eps
        _, dp = OB.assemble_boundary(pat, OB.RADIATION, c, [Te], fe, fi, state=(T + e)[None, :])
        _, dm = OB.assemble_boundary(pat, OB.RADIATION, c, [Te], fe, fi, state=(T - e)[None, :])
        fd = -(dp - dm) / (2 * eps)  # d = -R
        assert np.abs(fd - K[:, j]).max() < 1e-8 * np.abs(K).max()
    # at T = T_env the residual vanishes
    _, d0 = OB.assemble_boundary(pat, OB.RADIATION, c, [Te], fe, fi, state=np.full((1, mesh.n_nodes), Te))
    assert np.abs(d0).max() < 1e-14


# ---------------------------------------------------------------- flow boundaries (Sec. 4.3)

def _flow(kind, pat, faces, state=None, target=None, tau=0.0, uw=(0.0, 0.0, 0.0), rho=0.0, mu=0.0):
    return OB.assemble_boundary(pat, kind, tau, [*uw, rho, mu], *faces, state=state, target=target)


def test_flow_terms_on_one_unit_cube_by_hand():
    """Face x = 1 of the unit cube: int N_a dS = 1/4 on its four nodes and
    int n . grad N_a dS = +1/4 on them, -1/4 on the four nodes behind it."""
    mesh = box((1, 1, 1))
    pat = O.Pattern(mesh, 4)
    faces = (np.array([0], np.int32), np.array([1], np.uint8))
    front = np.array([a & 1 for a in range(8)], bool)
    w0 = np.array([0.7, -0.4, 0.9])
    rho, mu, tau = 1.3, 0.25, 2.0
    # inflow at rest: rho u^w (u^w.n) + mu (n.grad N_a) u^w - tau rho u^w; p-rows (u^w.n)
    _, d = _flow(OB.NS_INFLOW, pat, faces, tau=tau, uw=w0, rho=rho, mu=mu)
    R = -d.reshape(8, 4)
    for a in range(8):
        if front[a]:
            ref = (rho * w0 * w0[0] + mu * w0 - tau * rho * w0) / 4
            assert np.abs(R[a, :3] - ref).max() < 1e-15 and abs(R[a, 3] - w0[0] / 4) < 1e-15
        else:
            assert np.abs(R[a, :3] + mu * w0 / 4).max() < 1e-15 and R[a, 3] == 0.0
    # outflow of a uniform state (u = w0, p = p0): rho u (u.n) + p n on the face nodes
    st = np.zeros((4, 8))
    st[:3] = w0[:, None]
    st[3] = -0.6
    _, d = _flow(OB.NS_OUTFLOW, pat, faces, state=st, rho=rho, mu=mu)
    R = -d.reshape(8, 4)
    ref = (rho * w0 * w0[0] + np.array([-0.6, 0.0, 0.0])) / 4
    assert np.abs(R[front, :3] - ref).max() < 1e-15
    assert np.abs(R[~front]).max() == 0.0 and np.abs(R[:, 3]).max() == 0.0
    # fix (u^w = 0) of the uniform velocity, p = 0: -mu (n.grad N_a) u + tau rho u; p-rows -u.n
    st[3] = 0.0
    _, d = _flow(OB.NS_FIX, pat, faces, state=st, tau=tau, uw=(5.0, 5.0, 5.0), rho=rho, mu=mu)
    R = -d.reshape(8, 4)
    assert np.abs(R[front, :3] - (-mu * w0 + tau * rho * w0) / 4).max() < 1e-15
    assert np.abs(R[~front, :3] - mu * w0 / 4).max() < 1e-15
    assert np.abs(R[front, 3] + w0[0] / 4).max() < 1e-15 and np.abs(R[~front, 3]).max() == 0.0


def test_flow_domain_plus_outflow_is_integration_by_parts():
    """For linear u and p on an affine box the Galerkin flow form plus the outflow form on
    every face integrates the strong form against the basis:
    R_(a,i) = int N_a (rho div(u u)_i + p_,i),  R_(a,p) = int N_a div u,
    i.e. the mass matrix times the (linear) nodal values of those fields."""
    n = (2, 3, 2)
    mesh = box(n, lengths=[1.0, 1.5, 0.8])
    pat = O.Pattern(mesh, 4)
    rng = np.random.default_rng(21)
    A, c, b = rng.normal(size=(3, 3)), rng.normal(size=3), rng.normal(size=3)
    x = mesh.coords
    u = A @ x + c[:, None]
    st = np.vstack([u, b @ x + 0.3])
    rho, mu = 1.7, 0.4
    Rd = O.residual(pat, O.NS_SUPG, {"rho": rho, "mu": mu, "tau_m": 0.0, "tau_c": 0.0}, state=st)
    _, d = _flow(OB.NS_OUTFLOW, pat, W.box_faces(n), state=st, rho=rho, mu=mu)
    Rt = (Rd - d).reshape(-1, 4)
    p1 = O.Pattern(mesh, 1)
    M = p1.to_scipy(O.assemble(p1, O.MASS, {"coef": 1.0})[0])
    f = rho * (A @ u + u * np.trace(A)) + b[:, None]
    for i in range(3):
        assert np.abs(Rt[:, i] - M @ f[i]).max() < 1e-13
    assert np.abs(Rt[:, 3] - M @ np.full(mesh.n_nodes, np.trace(A))).max() < 1e-13


def _flow_case(seed):
    n = (2, 2, 3)
    mesh = box(n, jitter=0.2, seed=seed)
    pat = O.Pattern(mesh, 4)
    rng = np.random.default_rng(seed)
    st = rng.uniform(-1, 1, (4, mesh.n_nodes))
    tg = rng.uniform(-1, 1, (4, mesh.n_nodes))
    return n, mesh, pat, st, tg


def test_inflow_with_its_own_state_is_outflow():
    n, mesh, pat, st, _ = _flow_case(3)
    faces = W.box_faces(n, sides=[0, 3, 5])
    K1, d1 = _flow(OB.NS_INFLOW, pat, faces, state=st, target=st, tau=3.0, rho=1.1, mu=0.2)
    K2, d2 = _flow(OB.NS_OUTFLOW, pat, faces, state=st, rho=1.1, mu=0.2)
    assert np.abs(d1 - d2).max() < 1e-14
    assert abs(K1 - K2).max() > 1e-3  # the tangents differ: inflow holds u^w fixed


@pytest.mark.parametrize("kind", [OB.NS_INFLOW, OB.NS_OUTFLOW, OB.NS_FIX])
def test_flow_tangent_by_central_differences(kind):
    n, mesh, pat, st, tg = _flow_case(5)
    faces = W.box_faces(n)
    args = dict(target=tg, tau=2.5, rho=1.2, mu=0.3)
    K, d0 = _flow(kind, pat, faces, state=st, **args)
    rng = np.random.default_rng(6)
    dv = rng.normal(size=st.shape)
    h = 1e-6
    _, dp = _flow(kind, pat, faces, state=st + h * dv, **args)
    _, dm = _flow(kind, pat, faces, state=st - h * dv, **args)
    dirn = dv.T.reshape(-1)  # node-major DOF order
    fd = -(dp - dm) / (2 * h)
    assert np.abs(K @ dirn - fd).max() < 1e-7 * max(1.0, np.abs(fd).max())


def test_fix_pressure_velocity_blocks_are_antisymmetric():
    n, mesh, pat, st, _ = _flow_case(7)
    K, _ = _flow(OB.NS_FIX, pat, W.box_faces(n), state=st, tau=1.0, rho=1.0, mu=0.1)
    K = K.toarray()
    dof = np.arange(pat.n_rows)
    up = np.ix_(dof % 4 < 3, dof % 4 == 3)
    pu = np.ix_(dof % 4 == 3, dof % 4 < 3)
    assert np.abs(K[up]).max() > 0.1
    assert np.abs(K[up] + K[pu].T).max() < 1e-15


# ---------------------------------------------------------------- 2D edges

@pytest.mark.parametrize("nen", [4, 8])
def test_quadrilateral_edges(nen):
    """Edges of 4- and 8-node quadrilaterals: edge mass sums to the perimeter; a uniform
    traction on a straight edge gives the consistent loads (1/2, 1/2) or (1/6, 2/3, 1/6)
    of the total; a uniform stress over the closed boundary sums to zero and over one
    side to sigma n times its length; the radiation tangent by central differences."""
    import oracle.serendipity as S
    L, n = [1.5, 0.8], (3, 2)
    mesh = (W.structured_mesh(n, jitter=0.2, seed=1, lengths=L) if nen == 4
            else W.serendipity_mesh_2d(n, jitter=0.2, seed=1, lengths=L))
    P1 = (lambda nf: O.Pattern(mesh, nf)) if nen == 4 else (lambda nf: S.Pattern20(mesh, nf))
    edges = W.rect_edges(n)
    K, _ = OB.assemble_boundary_2d(P1(1), OB.PENALTY, 1.0, [0.0], *edges)
    assert abs(K.sum() - 2 * (L[0] + L[1])) < 1e-13
    sig = np.zeros(9)
    sig[[0, 1, 3, 4]] = [0.3, -0.7, 0.4, 1.1]  # leading 2x2 block
    _, d = OB.assemble_boundary_2d(P1(2), OB.TRACTION, 1.0, sig, *edges)
    assert np.abs(d.reshape(-1, 2).sum(axis=0)).max() < 1e-14
    top = W.rect_edges(n, sides=[3])  # y = L_y, n = +y
    _, d = OB.assemble_boundary_2d(P1(2), OB.TRACTION, 1.0, sig, *top)
    assert np.abs(d.reshape(-1, 2).sum(axis=0) - np.array([sig[1], sig[4]]) * L[0]).max() < 1e-14
    # one edge: consistent loads
    e, eid = int(top[0][0]), int(top[1][0])
    _, d1 = OB.assemble_boundary_2d(P1(2), OB.TRACTION, 1.0, sig, top[0][:1], top[1][:1])
    F = d1.reshape(-1, 2)
    en = OB.edge_nodes_2d(nen, eid)
    x = mesh.coords[:, mesh.conn[en[:2], e]]
    length = np.linalg.norm(x[:, 1] - x[:, 0])
    t = np.array([sig[1], sig[4]])
    share = [0.5, 0.5] if nen == 4 else [1 / 6, 1 / 6, 2 / 3]
    for a, s in zip(en, share):
        assert np.abs(F[mesh.conn[a, e]] - s * length * t).max() < 1e-14
    T = 1.0 + np.random.default_rng(2).random((1, mesh.n_nodes))
    Kr, _ = OB.assemble_boundary_2d(P1(1), OB.RADIATION, 0.7, [1.2], *edges, state=T)
    dv = np.random.default_rng(3).normal(size=T.shape)
    h = 1e-6
    _, dp = OB.assemble_boundary_2d(P1(1), OB.RADIATION, 0.7, [1.2], *edges, state=T + h * dv)
    _, dm = OB.assemble_boundary_2d(P1(1), OB.RADIATION, 0.7, [1.2], *edges, state=T - h * dv)
    assert np.abs(Kr @ dv[0] + (dp - dm) / (2 * h)).max() < 1e-7
