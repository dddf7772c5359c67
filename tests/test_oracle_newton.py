"""Oracle pins for the Newton iteration of the steady flow form (Sec. 2.1, the
Newton-Raphson update with the tangent stiffness; Sec. 2.2 D-4; form of Sec. 4.3).

  * Couette flow u = (z, 0, 0), p = 0 solves the discrete stabilised equations exactly on
    an undistorted grid (every term of R vanishes under 2-point Gauss: u.grad u = 0,
    grad grad u = 0, div u = 0, grad p = 0), so Newton from a zero interior must reach it;
  * with rho = 0 the problem is linear and Newton converges in one step;
  * near the solution the residual falls quadratically, which a wrong tangent would not
    give (the tangent itself is pinned by central differences in test_oracle_ns.py).
"""
import numpy as np
import pytest

import oracle as O
import oracle.newton as ON
import workloads as W


def taus(n, U=1.0, nu=0.01):
    """Per-mesh stabilisation constants from the element size h = 1/n."""
    h = 1.0 / n
    tm = ((2 * U / h) ** 2 + 9 * (4 * nu / h ** 2) ** 2) ** -0.5
    return tm, h * h / (12 * tm)


def params(n, rho=1.0, mu=0.01):
    tm, tc = taus(n)
    return dict(rho=rho, mu=mu, tau_m=tm, tau_c=tc)


def quadratic(hist, c=10.0, floor=1e-14):
    """r_{k+1}/r_0 <= c (r_k/r_0)^2 wherever r_k/r_0 < 0.1 and r_{k+1} is above the floor."""
    r0 = hist[0]
    for a, b in zip(hist[:-1], hist[1:]):
        if a / r0 < 0.1 and b / r0 > floor:
            assert b / r0 <= c * (a / r0) ** 2, (a, b, hist)


@pytest.mark.parametrize("numbering", [O.NODE_MAJOR, O.FIELD_MAJOR])
def test_couette_is_exact_and_newton_reaches_it(numbering):
    n = 5
    mesh = W.structured_mesh((n, n, n))
    pat = O.Pattern(mesh, 4, numbering=numbering)
    prm = params(n)
    st0, mask = W.flow_boundary(mesh, "couette", field_major=numbering == O.FIELD_MAJOR)
    exact = np.zeros_like(st0)
    exact[0] = mesh.coords[2]
    _, d = O.assemble(pat, O.NS_SUPG, prm, state=exact, dirichlet=mask)
    assert np.abs(d).max() < 1e-15
    st, hist, ok = ON.ns_newton(pat, prm, st0, mask, rtol=1e-13, max_steps=20)
    assert ok and len(hist) > 2
    assert np.abs(st - exact).max() < 1e-12
    quadratic(hist)


def test_stokes_converges_in_one_step():
    n = 4
    mesh = W.structured_mesh((n, n, n))
    pat = O.Pattern(mesh, 4)
    st0, mask = W.flow_boundary(mesh, "cavity")
    st, hist, ok = ON.ns_newton(pat, params(n, rho=0.0), st0, mask, rtol=1e-13, max_steps=3)
    assert ok and len(hist) == 2
    assert hist[1] <= 1e-13 * hist[0]


def test_cavity_converges_quadratically_and_keeps_boundary_values():
    n = 6
    mesh = W.structured_mesh((n, n, n))
    pat = O.Pattern(mesh, 4)
    st0, mask = W.flow_boundary(mesh, "cavity")
    st, hist, ok = ON.ns_newton(pat, params(n), st0, mask, rtol=1e-13, max_steps=20)
    assert ok and 3 <= len(hist) <= 10
    quadratic(hist)
    # constrained values are the initial ones
    node_mask = np.asarray(mask).reshape(-1, 4).T
    assert np.array_equal(st[node_mask != 0], st0[node_mask != 0])
    # the lid drags the fluid: positive u1 just below the lid, a return flow lower down
    c = mesh.coords
    mid = np.isclose(c[0], 0.5) & np.isclose(c[1], 0.5)
    z = c[2][mid]
    u = st[0][mid][np.argsort(z)]
    assert u[-2] > 0.05 and u[1:-1].min() < 0.0


def test_newton_stops_at_max_steps():
    n = 4
    mesh = W.structured_mesh((n, n, n))
    pat = O.Pattern(mesh, 4)
    st0, mask = W.flow_boundary(mesh, "cavity")
    st, hist, ok = ON.ns_newton(pat, params(n), st0, mask, rtol=1e-14, max_steps=1)
    assert not ok and len(hist) == 2
    st, hist, ok = ON.ns_newton(pat, params(n), st0, mask, rtol=1e-14, max_steps=0)
    assert not ok and len(hist) == 1 and np.array_equal(st, st0)
