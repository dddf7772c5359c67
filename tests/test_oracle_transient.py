"""Oracle pins for generalized-alpha time stepping of transient conduction (Sec. 2.1,
dynamic extension; domain form of Sec. 4.1), computed by oracle/transient.py."""
import numpy as np
import pytest

import oracle as O
import oracle.transient as OT
import workloads as W


def mode_problem(n=5, jitter=0.15):
    """K, M with Dirichlet boundary, and the lowest generalized eigenpair on the free rows."""
    import scipy.linalg as sl
    mesh = W.structured_mesh((n, n, n), jitter=jitter, seed=4)
    pat = O.Pattern(mesh, 1)
    k = W.lognormal_elem(mesh.n_elems, 0.3, 5)
    K, M, F = OT.operators(pat, 2.0, 1.5, elem_k=k)
    mask = W.boundary_node_mask(mesh.shape)
    free = np.flatnonzero(mask == 0)
    lam, vec = sl.eigh(K.toarray()[np.ix_(free, free)], M.toarray()[np.ix_(free, free)])
    phi = np.zeros(mesh.n_nodes)
    phi[free] = vec[:, 0]
    return K, M, F, mask, lam[0], phi


def amplification(z, rho):
    """Closed-form one-step map of the scheme for u + lambda T = 0, z = lambda dt:
    (T1, dt u1) from (T0, dt u0)."""
    c1, c2, b1 = OT.params(rho)
    den = c2 + z * c1 * b1
    # du dt = -(dt u0 (1 + z c1) + z T0) / den; T1 = T0 + dt u0 + b1 du dt
    dudt_T = -z / den
    dudt_U = -(1 + z * c1) / den
    return np.array([[1 + b1 * dudt_T, 1 + b1 * dudt_U], [dudt_T, 1 + dudt_U]])


@pytest.mark.parametrize("rho", [0.0, 0.5, 1.0])
def test_single_mode_step_matches_closed_form(rho):
    K, M, F, mask, lam, phi = mode_problem()
    F = np.zeros_like(F)
    for dt in (0.3 / lam, 3.0 / lam, 300.0 / lam):
        z = lam * dt
        G = np.zeros((2, 2))
        for col, (T0, u0) in enumerate(((phi, 0 * phi), (0 * phi, phi / dt))):
            T1, u1 = OT.heat_transient(K, M, F, T0, u0, dt, 1, rho=rho, mask=mask)
            a, b = phi @ (M @ T1), dt * (phi @ (M @ u1))  # phi is M-orthonormal
            assert np.abs(T1 - a * phi).max() < 1e-10 and np.abs(dt * u1 - b * phi).max() < 1e-10
            G[:, col] = a, b
        assert np.abs(G - amplification(z, rho)).max() < 1e-10
    # spectral radius at infinity and third-order agreement of the principal root
    ev = np.abs(np.linalg.eigvals(amplification(1e8, rho)))
    assert abs(ev.max() - rho) < 1e-3  # rho = 0: a double root, approached as z^(-1/2)
    for z in (1e-2, 2e-2):
        p = np.linalg.eigvals(amplification(z, rho))
        principal = p[np.argmin(np.abs(p - np.exp(-z)))]
        assert abs(principal - np.exp(-z)) < 0.5 * z ** 3


def test_second_order_in_time():
    K, M, F, mask, lam, phi = mode_problem(n=4)
    F = np.zeros_like(F)
    t_end = 1.0 / lam
    errs = []
    for steps in (4, 8, 16):
        dt = t_end / steps
        T, u = OT.heat_transient(K, M, F, phi, -lam * phi, dt, steps, rho=0.5, mask=mask)
        errs.append(np.abs(T - np.exp(-lam * t_end) * phi).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 4.5 and 3.7 < r2 < 4.3, errs


def test_steady_state_and_initial_rate():
    n = 5
    mesh = W.structured_mesh((n, n, n), jitter=0.1, seed=2)
    pat = O.Pattern(mesh, 1)
    s = np.ones(mesh.n_nodes)
    K, M, F, = OT.operators(pat, 1.0, 1.0, source=s)
    mask = W.boundary_node_mask(mesh.shape)
    free = mask == 0
    T0 = np.zeros(mesh.n_nodes)
    # the consistent rate: M u0 = F - K T0 on the free rows
    _, u0 = OT.heat_transient(K, M, F, T0, T0, 1.0, 0, mask=mask, init_rate=True)
    assert np.abs((M @ u0 - F)[free]).max() < 1e-12 and np.all(u0[~free] == 0)
    # L-stable (rho = 0) long steps settle on the steady solution K T = F
    T, u = OT.heat_transient(K, M, F, T0, u0, 10.0, 30, rho=0.0, mask=mask)
    import scipy.sparse.linalg as spla
    Ts = np.zeros(mesh.n_nodes)
    idx = np.flatnonzero(free)
    Ts[idx] = spla.spsolve(K[idx][:, idx].tocsc(), F[idx])
    assert np.abs(T - Ts).max() < 1e-8 * np.abs(Ts).max()
    assert np.abs(u).max() < 1e-8
