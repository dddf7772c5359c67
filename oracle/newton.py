"""Oracle: Newton iteration for the steady stabilised flow form, on the oracle's assembly.

TEST INFRASTRUCTURE ONLY.  Only `tests/`, the smoke check and the benchmark's CPU
baseline leg may import this module; the product library never does.

Sec. 2.1 (the Newton-Raphson equation and the tangent stiffness that follows it): with
K^n = dR/dU at the state U^n, a sub-step solves K^n (U^{n+1} - U^n) = -R(U^n).  Sec. 2.2
D-4 solves that system with a direct or iterative solver, adds the increment to the
state (for a steady problem the time factor of the increment is 1) and returns to the
assembly of D-1.  The assembly exports d = -R, so each step here solves K dU = d.  The
linear solve is scipy's sparse LU, a library primitive.  Dirichlet rows are eliminated
by the assembly (unit row, zero column, d_r = 0), so constrained values keep the values
of the initial state.

Pins (tests/test_oracle_newton.py): Couette flow, an exact solution of the discrete
stabilised equations on an undistorted grid, is reached from a zero interior; a linear
(Stokes, rho = 0) problem converges in one step; the residual of a lid-driven cavity
falls quadratically near the solution.
"""
from __future__ import annotations

import numpy as np

from . import NODE_MAJOR, NS_SUPG, assemble


def state_increment(pat, du):
    """The DOF vector du of the pattern's numbering as a [4][n_nodes] state increment."""
    n_nodes = pat.mesh.n_nodes
    if pat.numbering == NODE_MAJOR:
        return du.reshape(n_nodes, 4).T
    return du.reshape(4, n_nodes)


def ns_newton(pat, params, state0, dirichlet=None, rtol=1e-10, atol=0.0, max_steps=20):
    """Newton from state0 ([4][n_nodes]: u1, u2, u3, p).

    Returns (state, residual norms |d|_2 before each update, converged).  Stops when
    |d|_2 <= max(rtol |d_0|_2, atol) or after max_steps updates."""
    import scipy.sparse.linalg as spla
    state = np.array(state0, dtype=np.float64, copy=True)
    hist = []
    for k in range(max_steps + 1):
        K, d = assemble(pat, NS_SUPG, params, state=state, dirichlet=dirichlet)
        r = float(np.linalg.norm(d))
        hist.append(r)
        if r <= max(rtol * hist[0], atol):
            return state, hist, True
        if k == max_steps:
            break
        du = spla.spsolve(pat.to_scipy(K).tocsc(), d)
        state += state_increment(pat, du)
    return state, hist, False
