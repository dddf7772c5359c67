"""Oracle: generalized-alpha time stepping of transient thermal conduction.

TEST INFRASTRUCTURE ONLY.  Only `tests/`, the smoke check and the benchmark's CPU
baseline leg may import this module; the product library never does.

Sec. 2.1 (dynamic extension of the Newton-Raphson update), for C dT/dt - div(k grad T)
= s (the domain form of Sec. 4.1 with its capacity term).  With u = dT/dt, the
increments of a step satisfy dT = dt (u0 + b1 du); the residual M u~ + K T~ - F is
evaluated at the relaxed values T~ = T0 + c1 dT, u~ = u0 + c2 du; its tangent with
respect to the basic variable is c1 K + c2/(b1 dt) M.  One Newton step is exact (the
problem is linear).  Parameters from the spectral radius at infinity rho (generalized
alpha for first-order systems): c2 = (3 - rho)/(2 (1 + rho)), c1 = 1/(1 + rho),
b1 = 1/2 + c2 - c1.  Dirichlet rows keep T (unit row, zero column, zero right-hand side).
The linear solves are scipy's sparse LU (a library primitive).

Pins (tests/test_oracle_transient.py): the one-step map of a single generalized
eigenmode has the scheme's closed-form amplification (spectral radius rho at large
lambda dt, exp(-lambda dt) to third order at small lambda dt); errors fall as dt^2;
the steady state is reached.
"""
from __future__ import annotations

import numpy as np

from . import MASS, POISSON, assemble


def params(rho):
    am = (3.0 - rho) / (2.0 * (1.0 + rho))
    af = 1.0 / (1.0 + rho)
    return af, am, 0.5 + am - af  # c1, c2, b1


def operators(pat, capacity, conductivity, elem_k=None, source=None):
    """(K, M, F) as scipy CSR matrices and a vector, from the oracle's assembly."""
    Kv, F = assemble(pat, POISSON, {"coef": conductivity}, elem_param=elem_k,
                     nodal_src=None if source is None else source[None, :])
    Mv, _ = assemble(pat, MASS, {"coef": capacity})
    return pat.to_scipy(Kv), pat.to_scipy(Mv), F


def eliminate(A, mask):
    """Unit rows and zero columns on the marked rows (structure kept)."""
    import scipy.sparse as sp
    if mask is None:
        return A.tocsc()
    keep = sp.diags((mask == 0).astype(np.float64))
    fix = sp.diags((mask != 0).astype(np.float64))
    return (keep @ A @ keep + fix).tocsc()


def heat_transient(K, M, F, T0, u0, dt, n_steps, rho=0.5, mask=None, init_rate=False):
    """n_steps generalized-alpha steps; returns (T, u)."""
    import scipy.sparse.linalg as spla
    c1, c2, b1 = params(rho)
    T = np.array(T0, dtype=np.float64, copy=True)
    u = np.array(u0, dtype=np.float64, copy=True)
    free = np.ones_like(T) if mask is None else (mask == 0).astype(np.float64)
    if init_rate:
        u = spla.spsolve(eliminate(M, mask), free * (F - K @ T))
    if n_steps == 0:
        return T, u
    A = spla.splu(eliminate(c1 * K + (c2 / (b1 * dt)) * M, mask))
    for _ in range(n_steps):
        rhs = free * (F - K @ T - (1.0 - c2 / b1) * (M @ u))
        dT = A.solve(rhs)
        T = T + dT
        u = u + (dT / dt - u) / b1
    return T, u
