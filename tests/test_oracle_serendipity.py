"""Oracle pins for 20-node serendipity hexahedra (oracle/serendipity.py): basis identities,
exact volume, patch tests for linear and quadratic fields, rigid-body modes."""
import numpy as np

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
