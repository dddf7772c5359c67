"""Oracle pins for 20-node serendipity hexahedra (oracle/serendipity.py): basis identities,
exact volume, patch tests for linear and quadratic fields, rigid-body modes, face loads,
and the paper's cantilever against beam theory."""
import numpy as np
import pytest

import oracle as O
import oracle.serendipity as S
import workloads as W


def ref_nodes():
    X = np.zeros((20, 3))
    X[:8] = S.CORNER
    for m, (ax, (s1, s2)) in enumerate(S.EDGES):
        oth = sorted(((ax + 1) % 3, (ax + 2) % 3))
        X[8 + m, ax] = 0.0
        X[8 + m, oth[0]], X[8 + m, oth[1]] = s1, s2
    return X


def test_basis_kronecker_unity_and_gradients():
    X = ref_nodes()
    for a in range(20):
        N, _ = S.basis20(X[a])
        assert np.abs(N - np.eye(20)[a]).max() < 1e-15
    rng = np.random.default_rng(0)
    for _ in range(10):
        x = rng.uniform(-1, 1, 3)
        N, dN = S.basis20(x)
        assert abs(N.sum() - 1.0) < 1e-14 and np.abs(dN.sum(axis=0)).max() < 1e-14
        # the basis reproduces x itself: sum N_a X_a = x, sum dN_a X_a = I
        assert np.abs(N @ X - x).max() < 1e-14 and np.abs(X.T @ dN - np.eye(3)).max() < 1e-14
        for d in range(3):
            h = np.zeros(3)
            h[d] = 1e-6
            fd = (S.basis20(x + h)[0] - S.basis20(x - h)[0]) / 2e-6
            assert np.abs(fd - dN[:, d]).max() < 1e-8


def test_mesh_pattern_and_volume():
    mesh = W.serendipity_mesh((2, 3, 2), jitter=0.2, seed=3, lengths=[1.0, 1.5, 0.5])
    assert mesh.nen == 20
    # every edge midpoint is shared: node count = corners + edges
    assert mesh.n_nodes == 3 * 4 * 3 + 2 * 4 * 3 + 3 * 3 * 3 + 3 * 4 * 2
    pat = S.Pattern20(mesh, 1)
    K, d = S.assemble20(pat, O.MASS, {"coef": 1.0}, nodal_src=np.ones((1, mesh.n_nodes)))
    # straight edges keep the map trilinear, so the 3-point rule integrates det J exactly
    assert abs(K.sum() - 0.75) < 1e-14 and abs(d.sum() - 0.75) < 1e-14
    # the pattern is symmetric and each row holds its own node
    Sm = pat.to_scipy(np.ones(pat.nnz))
    assert (Sm != Sm.T).nnz == 0 and np.all(Sm.diagonal() == 1)


def test_poisson_patch_tests():
    # linear fields on a jittered mesh: interior rows of K u vanish
    n = (3, 3, 3)
    mesh = W.serendipity_mesh(n, jitter=0.2, seed=5)
    pat = S.Pattern20(mesh, 1)
    k = W.lognormal_elem(mesh.n_elems, 0.3, 6)
    K, _ = S.assemble20(pat, O.POISSON, {"coef": 1.3})
    Km = pat.to_scipy(K)
    c = mesh.coords
    interior = np.all((c > 1e-12) & (c < 1 - 1e-12), axis=0)
    u = 0.4 * c[0] - 1.1 * c[1] + 0.3 * c[2]
    assert np.abs((Km @ u)[interior]).max() < 1e-13
    assert np.abs(Km @ np.ones(mesh.n_nodes)).max() < 1e-13  # rows sum to zero
    # quadratic fields on an affine box: (K u)_a = -int N_a (lap u) for interior a
    mesh = W.serendipity_mesh(n, lengths=[1.0, 1.2, 0.9])
    pat = S.Pattern20(mesh, 1)
    K, _ = S.assemble20(pat, O.POISSON, {"coef": 1.0})
    M, _ = S.assemble20(pat, O.MASS, {"coef": 1.0})
    c = mesh.coords
    hi = np.array([1.0, 1.2, 0.9])[:, None]
    interior = np.all((c > 1e-12) & (c < hi - 1e-12), axis=0)
    u = c[0] ** 2 + c[1] * c[2] - 0.5 * c[2] ** 2  # lap u = 2 - 1 = 1
    r = pat.to_scipy(K) @ u + pat.to_scipy(M) @ np.ones(mesh.n_nodes) * 1.0
    assert np.abs(r[interior]).max() < 1e-13
    del k


def test_elasticity_rigid_body_modes():
    mesh = W.serendipity_mesh((2, 2, 3), jitter=0.2, seed=8)
    pat = S.Pattern20(mesh, 3)
    E = W.lognormal_elem(mesh.n_elems, 0.5, 9)
    K, _ = S.assemble20(pat, O.ELASTICITY, {"coef": 2.0, "nu": 0.3}, elem_param=E)
    Km = pat.to_scipy(K)
    assert abs(Km - Km.T).max() < 1e-12 * abs(Km).max()
    x, y, z = mesh.coords
    one, zero = np.ones_like(x), np.zeros_like(x)
    modes = [(one, zero, zero), (zero, one, zero), (zero, zero, one),
             (-y, x, zero), (zero, -z, y), (z, zero, -x)]
    for m in modes:
        u = np.stack(m, axis=1).reshape(-1)  # node-major
        assert np.abs(Km @ u).max() < 1e-12 * abs(Km).max()


# ---------------------------------------------------------------- faces (boundary forms)

def test_face_loads_of_the_eight_node_face():
    """A uniform traction on a flat 8-node serendipity face loads its corners with -1/12
    and its mid-side nodes with 1/3 of the total (the classic consistent loads)."""
    import oracle.boundary as OB
    mesh = W.serendipity_mesh((1, 1, 1), lengths=[2.0, 1.5, 1.0])
    pat = S.Pattern20(mesh, 3)
    sig = np.zeros((3, 3))
    sig[:, 2] = [0.4, -0.7, 1.3]  # t = sigma^l e_z on the top face
    K, d = S.assemble_boundary20(pat, OB.TRACTION, 1.0, sig.reshape(-1), [0], [5])
    F = d.reshape(-1, 3)
    area = 2.0 * 1.5
    top = np.nonzero(np.abs(mesh.coords[2] - 1.0) < 1e-12)[0]
    corner = [v for v in top if v in set(mesh.conn[:8, 0])]
    mid = [v for v in top if v not in corner]
    assert len(corner) == 4 and len(mid) == 4
    assert np.abs(F[corner] + area / 12 * sig[:, 2]).max() < 1e-14
    assert np.abs(F[mid] - area / 3 * sig[:, 2]).max() < 1e-14
    assert np.abs(np.delete(F, top, axis=0)).max() == 0.0
    # the same load as a nodal traction target
    tg = np.tile(sig[:, 2][:, None], (1, mesh.n_nodes))
    _, d2 = S.assemble_boundary20(pat, OB.TRACTION, 1.0, [], [0], [5], target=tg)
    assert np.abs(d2 - d).max() < 1e-15


def test_face_mass_and_closed_surface_load():
    import oracle.boundary as OB
    n, L = (2, 3, 2), [1.0, 1.5, 0.8]
    mesh = W.serendipity_mesh(n, jitter=0.2, seed=4, lengths=L)
    fe, fi = W.box_faces(n)
    pat = S.Pattern20(mesh, 1)
    K, _ = S.assemble_boundary20(pat, OB.PENALTY, 1.0, [0.0], fe, fi)
    area = 2 * (L[0] * L[1] + L[1] * L[2] + L[0] * L[2])
    assert abs(K.sum() - area) < 1e-12 * area
    pat3 = S.Pattern20(mesh, 3)
    sig = np.array([[0.3, -0.2, 0.7], [0.1, 0.5, -0.4], [0.6, 0.2, -1.1]])
    _, d = S.assemble_boundary20(pat3, OB.TRACTION, 1.0, sig.reshape(-1), fe, fi)
    assert np.abs(d.reshape(-1, 3).sum(axis=0)).max() < 1e-14
    fe1, fi1 = W.box_faces(n, sides=[3])  # y = L_y, n = +y, area L_x L_z
    _, d = S.assemble_boundary20(pat3, OB.TRACTION, 1.0, sig.reshape(-1), fe1, fi1)
    assert np.abs(d.reshape(-1, 3).sum(axis=0) - sig[:, 1] * L[0] * L[2]).max() < 1e-14


def test_radiation_tangent_on_quadratic_faces():
    import oracle.boundary as OB
    n = (2, 1, 2)
    mesh = W.serendipity_mesh(n, jitter=0.2, seed=6)
    pat = S.Pattern20(mesh, 1)
    fe, fi = W.box_faces(n)
    T = 1.0 + np.random.default_rng(2).random((1, mesh.n_nodes))
    K, d0 = S.assemble_boundary20(pat, OB.RADIATION, 0.7, [1.2], fe, fi, state=T)
    dv = np.random.default_rng(3).normal(size=T.shape)
    h = 1e-6
    _, dp = S.assemble_boundary20(pat, OB.RADIATION, 0.7, [1.2], fe, fi, state=T + h * dv)
    _, dm = S.assemble_boundary20(pat, OB.RADIATION, 0.7, [1.2], fe, fi, state=T - h * dv)
    assert np.abs(K @ dv[0] + (dp - dm) / (2 * h)).max() < 1e-7


def cantilever(case, mesh, P=1.0):
    """The paper's 3D cantilever (Sec. 4.2): L = 10, h = 1, E = 1, nu = 0, the face x = 0
    clamped; case 1 end load P (uniform shear traction on x = L), case 2 uniform pressure P
    on the top face y = h, case 3 pressure P (1 - x/L) on the top.  Returns the oracle's
    displacement [n_nodes][3] (direct solve)."""
    import scipy.sparse.linalg as spla
    import oracle.boundary as OB
    n = (10, 4, 4)
    pat = S.Pattern20(mesh, 3)
    Kv, _ = S.assemble20(pat, O.ELASTICITY, {"coef": 1.0, "nu": 0.0})
    K = pat.to_scipy(Kv)
    if case == 1:
        sig = np.zeros((3, 3))
        sig[1, 0] = -P  # t = sigma^l e_x = (0, -P, 0) over the unit end face
        _, d = S.assemble_boundary20(pat, OB.TRACTION, 1.0, sig.reshape(-1), *W.box_faces(n, sides=[1]))
    else:
        t = np.zeros((3, mesh.n_nodes))
        t[1] = -P * (1.0 if case == 2 else 1.0 - mesh.coords[0] / 10.0)
        _, d = S.assemble_boundary20(pat, OB.TRACTION, 1.0, [], *W.box_faces(n, sides=[3]), target=t)
    fixed = np.repeat(np.abs(mesh.coords[0]) < 1e-12, 3)
    free = ~fixed
    u = np.zeros(pat.n_rows)
    u[free] = spla.spsolve(K[free][:, free].tocsc(), d[free])
    return u.reshape(-1, 3)


def beam_deflection(case, x, P=1.0, L=10.0):
    """Euler-Bernoulli deflections of the three load cases (E = 1, I = h^4/12, h = 1)."""
    EI = 1.0 / 12.0
    if case == 1:
        return -P * x ** 2 / (6 * EI) * (3 * L - x)
    if case == 2:
        return -P * x ** 2 / (24 * EI) * (6 * L ** 2 - 4 * L * x + x ** 2)
    return -P * x ** 2 / (120 * L * EI) * (10 * L ** 3 - 10 * L ** 2 * x + 5 * L * x ** 2 - x ** 3)


@pytest.mark.parametrize("case", [1, 2, 3])
def test_cantilever_matches_beam_theory(case):
    """10 x 4 x 4 quadratic serendipity bricks against beam theory along the centre line
    y = z = h/2: within 2% of the tip deflection (shear deformation and the clamped end
    account for less than that at L/h = 10)."""
    mesh = W.serendipity_mesh((10, 4, 4), lengths=[10.0, 1.0, 1.0])
    u = cantilever(case, mesh)
    c = mesh.coords
    line = np.nonzero((np.abs(c[1] - 0.5) < 1e-12) & (np.abs(c[2] - 0.5) < 1e-12))[0]
    x = c[0, line]
    ref = beam_deflection(case, x)
    tip = np.abs(ref).max()
    assert np.abs(u[line, 1] - ref).max() < 0.02 * tip
    # symmetric about the plane z = h/2: no out-of-plane motion on the line (to rounding);
    # the end load is also antisymmetric about y = h/2, so the line does not stretch
    assert np.abs(u[line, 2]).max() < 1e-9 * tip
    if case == 1:
        assert np.abs(u[line, 0]).max() < 1e-9 * tip


# ---------------------------------------------------------------- 8-node quadrilaterals

def ref_nodes8():
    X = np.zeros((8, 2))
    for a in range(4):
        X[a] = [1.0 if a & 1 else -1.0, 1.0 if a >> 1 else -1.0]
    X[4], X[5], X[6], X[7] = [0, -1], [0, 1], [-1, 0], [1, 0]
    return X


def test_quad8_basis_kronecker_unity_and_gradients():
    X = ref_nodes8()
    for a in range(8):
        N, _ = S.basis8(X[a])
        assert np.abs(N - np.eye(8)[a]).max() < 1e-15
    rng = np.random.default_rng(1)
    for _ in range(10):
        x = rng.uniform(-1, 1, 2)
        N, dN = S.basis8(x)
        assert abs(N.sum() - 1.0) < 1e-14 and np.abs(dN.sum(axis=0)).max() < 1e-14
        assert np.abs(N @ X - x).max() < 1e-14 and np.abs(X.T @ dN - np.eye(2)).max() < 1e-14
        # the complete quadratics and x^2 y, x y^2 lie in the span: interpolation is exact
        for f in (lambda p: p[0] ** 2, lambda p: p[0] * p[1], lambda p: p[1] ** 2,
                  lambda p: p[0] ** 2 * p[1], lambda p: p[0] * p[1] ** 2):
            assert abs(N @ np.array([f(p) for p in X]) - f(x)) < 1e-14
        for d in range(2):
            h = np.zeros(2)
            h[d] = 1e-6
            fd = (S.basis8(x + h)[0] - S.basis8(x - h)[0]) / 2e-6
            assert np.abs(fd - dN[:, d]).max() < 1e-8


def test_quad8_mesh_area_and_pattern():
    mesh = W.serendipity_mesh_2d((3, 2), jitter=0.2, seed=3, lengths=[1.5, 0.8])
    assert mesh.nen == 8 and mesh.n_nodes == 4 * 3 + 3 * 3 + 4 * 2
    pat = S.Pattern20(mesh, 1)
    K, d = S.assemble20(pat, O.MASS, {"coef": 1.0}, nodal_src=np.ones((1, mesh.n_nodes)))
    assert abs(K.sum() - 1.2) < 1e-14 and abs(d.sum() - 1.2) < 1e-14
    Sm = pat.to_scipy(np.ones(pat.nnz))
    assert (Sm != Sm.T).nnz == 0 and np.all(Sm.diagonal() == 1)


def test_quad8_patch_tests():
    mesh = W.serendipity_mesh_2d((3, 4), jitter=0.2, seed=5)
    pat = S.Pattern20(mesh, 1)
    Km = pat.to_scipy(S.assemble20(pat, O.POISSON, {"coef": 1.7})[0])
    c = mesh.coords
    interior = np.all((c > 1e-12) & (c < 1 - 1e-12), axis=0)
    assert np.abs((Km @ (0.4 * c[0] - 1.1 * c[1]))[interior]).max() < 1e-13
    assert np.abs(Km @ np.ones(mesh.n_nodes)).max() < 1e-13
    # quadratic fields on an affine rectangle: (K u)_a = -int N_a lap u on interior rows
    mesh = W.serendipity_mesh_2d((3, 4), lengths=[1.0, 1.4])
    pat = S.Pattern20(mesh, 1)
    K = pat.to_scipy(S.assemble20(pat, O.POISSON, {"coef": 1.0})[0])
    M = pat.to_scipy(S.assemble20(pat, O.MASS, {"coef": 1.0})[0])
    c = mesh.coords
    hi = np.array([1.0, 1.4])[:, None]
    interior = np.all((c > 1e-12) & (c < hi - 1e-12), axis=0)
    u = 1.5 * c[0] ** 2 + c[0] * c[1] - 0.5 * c[1] ** 2  # lap u = 3 - 1 = 2
    assert np.abs((K @ u + M @ np.full(mesh.n_nodes, 2.0))[interior]).max() < 1e-13


def test_quad8_elasticity_rigid_modes():
    mesh = W.serendipity_mesh_2d((3, 2), jitter=0.2, seed=8)
    pat = S.Pattern20(mesh, 2)
    E = W.lognormal_elem(mesh.n_elems, 0.5, 9)
    Km = pat.to_scipy(S.assemble20(pat, O.ELASTICITY, {"coef": 2.0, "nu": 0.3}, elem_param=E)[0])
    assert abs(Km - Km.T).max() < 1e-12 * abs(Km).max()
    x, y = mesh.coords
    one, zero = np.ones_like(x), np.zeros_like(x)
    for m in ((one, zero), (zero, one), (-y, x)):
        assert np.abs(Km @ np.stack(m, axis=1).reshape(-1)).max() < 1e-12 * abs(Km).max()
    # uniaxial strain e_xx = 1 (plane strain): interior rows vanish, and the reaction on the
    # face x = 1 sums to (lam + 2 mu) times its length for E = 1 everywhere
    mesh = W.serendipity_mesh_2d((3, 2), jitter=0.2, seed=8)
    pat = S.Pattern20(mesh, 2)
    Km = pat.to_scipy(S.assemble20(pat, O.ELASTICITY, {"coef": 1.0, "nu": 0.3})[0])
    F = (Km @ np.stack((mesh.coords[0], np.zeros(mesh.n_nodes)), axis=1).reshape(-1)).reshape(-1, 2)
    lam, mu = 0.3 / (1.3 * 0.4), 1.0 / 2.6
    right = np.abs(mesh.coords[0] - 1.0) < 1e-12
    assert abs(F[right, 0].sum() - (lam + 2 * mu)) < 1e-12


# ---------------------------------------------------------------- 10-node tetrahedra

TET_NODES = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1],
                      [0.5, 0, 0], [0.5, 0.5, 0], [0, 0.5, 0], [0, 0, 0.5], [0.5, 0, 0.5], [0, 0.5, 0.5]])


def test_tet10_basis_and_rule():
    import math
    for a in range(10):
        N, _ = S.basis10(TET_NODES[a])
        assert np.abs(N - np.eye(10)[a]).max() < 1e-15
    rng = np.random.default_rng(3)
    for _ in range(10):
        x = rng.dirichlet(np.ones(4))[1:]
        N, dN = S.basis10(x)
        assert abs(N.sum() - 1.0) < 1e-14 and np.abs(dN.sum(axis=0)).max() < 1e-14
        assert np.abs(N @ TET_NODES - x).max() < 1e-14 and np.abs(TET_NODES.T @ dN - np.eye(3)).max() < 1e-14
        for f in (lambda p: p[0] ** 2, lambda p: p[0] * p[2], lambda p: p[1] * p[2], lambda p: p[2] ** 2):
            assert abs(N @ np.array([f(p) for p in TET_NODES]) - f(x)) < 1e-14
        for d in range(3):
            h = np.zeros(3)
            h[d] = 1e-6
            fd = (S.basis10(x + h)[0] - S.basis10(x - h)[0]) / 2e-6
            assert np.abs(fd - dN[:, d]).max() < 1e-8
    # the collapsed rule against the closed form a! b! c! / (a + b + c + 3)! up to degree 5
    xq, wq = S.gauss_tet()
    for a in range(6):
        for b in range(6 - a):
            for c in range(6 - a - b):
                exact = math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(a + b + c + 3)
                got = (wq * xq[:, 0] ** a * xq[:, 1] ** b * xq[:, 2] ** c).sum()
                assert abs(got - exact) < 1e-15, (a, b, c)


def test_tet10_mesh_volume_pattern_and_patch_tests():
    L = [1.0, 1.3, 0.7]
    mesh = W.tet10_mesh((2, 3, 2), jitter=0.2, seed=4, lengths=L)
    assert mesh.nen == 10 and mesh.n_elems == 6 * 12
    pat = S.Pattern20(mesh, 1)
    M, d = S.assemble20(pat, O.MASS, {"coef": 1.0}, nodal_src=np.ones((1, mesh.n_nodes)))
    vol = L[0] * L[1] * L[2]
    assert abs(M.sum() - vol) < 1e-14 and abs(d.sum() - vol) < 1e-14
    Sm = pat.to_scipy(np.ones(pat.nnz))
    assert (Sm != Sm.T).nnz == 0
    K = pat.to_scipy(S.assemble20(pat, O.POISSON, {"coef": 1.0})[0])
    Mm = pat.to_scipy(M)
    c = mesh.coords
    hi = np.array(L)[:, None]
    interior = np.all((c > 1e-12) & (c < hi - 1e-12), axis=0)
    assert np.abs((K @ (0.3 * c[0] - 0.8 * c[1] + 1.1 * c[2]))[interior]).max() < 1e-13
    # every element map is affine, so quadratic fields pass on the jittered mesh too
    u = c[0] ** 2 + 2.0 * c[1] * c[2] - 0.5 * c[2] ** 2 + c[0] * c[1]  # lap u = 2 - 1 = 1
    assert np.abs((K @ u + Mm @ np.ones(mesh.n_nodes))[interior]).max() < 1e-12


def test_tet10_elasticity_rigid_modes():
    mesh = W.tet10_mesh((2, 2, 1), jitter=0.2, seed=5)
    pat = S.Pattern20(mesh, 3)
    E = W.lognormal_elem(mesh.n_elems, 0.5, 6)
    Km = pat.to_scipy(S.assemble20(pat, O.ELASTICITY, {"coef": 2.0, "nu": 0.3}, elem_param=E)[0])
    assert abs(Km - Km.T).max() < 1e-12 * abs(Km).max()
    x, y, z = mesh.coords
    one, zero = np.ones_like(x), np.zeros_like(x)
    for m in ((one, zero, zero), (zero, one, zero), (zero, zero, one), (-y, x, zero), (zero, -z, y), (z, zero, -x)):
        assert np.abs(Km @ np.stack(m, axis=1).reshape(-1)).max() < 1e-12 * abs(Km).max()


def test_tet10_faces():
    """Faces of 10-node tetrahedra: a uniform traction on a flat 6-node face loads its
    vertices with nothing and each mid-side node with a third of the total; face mass
    sums to the surface area; a uniform stress over the closed surface sums to zero; the
    radiation tangent by central differences."""
    import oracle.boundary as OB
    L = [1.0, 1.3, 0.7]
    mesh = W.tet10_mesh((2, 2, 1), jitter=0.2, seed=3, lengths=L)
    fe, fi = W.tet10_box_faces(mesh, L)
    pat = S.Pattern20(mesh, 1)
    K, _ = S.assemble_boundary_tet10(pat, OB.PENALTY, 1.0, [0.0], fe, fi)
    area = 2 * (L[0] * L[1] + L[1] * L[2] + L[0] * L[2])
    assert abs(K.sum() - area) < 1e-13 * area
    pat3 = S.Pattern20(mesh, 3)
    sig = np.array([[0.3, -0.2, 0.7], [0.1, 0.5, -0.4], [0.6, 0.2, -1.1]])
    _, d = S.assemble_boundary_tet10(pat3, OB.TRACTION, 1.0, sig.reshape(-1), fe, fi)
    assert np.abs(d.reshape(-1, 3).sum(axis=0)).max() < 1e-14
    # one face: vertices 0, mid-sides 1/3 of t times its area
    e, k = int(fe[0]), int(fi[0])
    _, d1 = S.assemble_boundary_tet10(pat3, OB.TRACTION, 1.0, sig.reshape(-1), fe[:1], fi[:1])
    F = d1.reshape(-1, 3)
    fn = S.tet_face_nodes(k)
    P = mesh.coords[:, mesh.conn[fn[:3], e]]
    nr = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    c_in = mesh.coords[:, mesh.conn[:4, e]].mean(axis=1)
    if nr @ (P[:, 0] - c_in) < 0:
        nr = -nr
    a_f = 0.5 * np.linalg.norm(nr)
    t = sig @ (nr / np.linalg.norm(nr))
    for m, a in enumerate(fn):
        want = np.zeros(3) if m < 3 else a_f * t / 3.0
        assert np.abs(F[mesh.conn[a, e]] - want).max() < 1e-14
    # radiation tangent
    T = 1.0 + np.random.default_rng(2).random((1, mesh.n_nodes))
    Kr, _ = S.assemble_boundary_tet10(pat, OB.RADIATION, 0.7, [1.2], fe, fi, state=T)
    dv = np.random.default_rng(3).normal(size=T.shape)
    h = 1e-6
    _, dp = S.assemble_boundary_tet10(pat, OB.RADIATION, 0.7, [1.2], fe, fi, state=T + h * dv)
    _, dm = S.assemble_boundary_tet10(pat, OB.RADIATION, 0.7, [1.2], fe, fi, state=T - h * dv)
    assert np.abs(Kr @ dv[0] + (dp - dm) / (2 * h)).max() < 1e-7
