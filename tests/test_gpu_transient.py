"""Generalized-alpha transient conduction on the GPU (mf_heat_transient) against the
oracle's stepping (oracle/transient.py) on the same inputs."""
import sys

import numpy as np
import pytest

import oracle as O
import oracle.transient as OT
import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def problem(n, seed=3):
    mesh = W.structured_mesh((n, n, n), jitter=0.15, seed=seed)
    k = W.lognormal_elem(mesh.n_elems, 0.4, seed + 1)
    s = W.uniform_nodal(1, mesh.n_nodes, 0, 1, seed + 2)[0]
    mask = W.boundary_node_mask(mesh.shape)
    rng = np.random.default_rng(seed + 3)
    T0 = np.where(mask != 0, 0.25, rng.random(mesh.n_nodes))
    return mesh, k, s, mask, T0


@pytest.mark.parametrize("rho", [0.0, 0.5, 1.0])
@pytest.mark.parametrize("init_rate", [True, False])
def test_transient_matches_oracle(mf, rho, init_rate):
    say("transient 8^3 rho", rho, "init_rate", init_rate)
    n, C, kc, dt, steps = 8, 2.0, 1.3, 0.01, 6
    mesh, k, s, mask, T0 = problem(n)
    u0 = np.zeros(mesh.n_nodes)
    pat_o = O.Pattern(mesh, 1)
    K, M, F = OT.operators(pat_o, C, kc, elem_k=k, source=s)
    T_ref, u_ref = OT.heat_transient(K, M, F, T0, u0, dt, steps, rho=rho, mask=mask, init_rate=init_rate)
    dev = torch.device("cuda:0")
    pat = mf.Pattern(torch.from_numpy(mesh.conn).to(dev), mesh.n_nodes, 3, 1)
    T = torch.from_numpy(T0.copy()).to(dev)
    U = torch.from_numpy(u0.copy()).to(dev)
    s_ = torch.cuda.Stream()
    with torch.cuda.stream(s_):
        res = mf.heat_transient(pat, torch.from_numpy(mesh.coords).to(dev), T, U, dt, steps, capacity=C,
                                conductivity=kc, elem_k=torch.from_numpy(k).to(dev),
                                source=torch.from_numpy(s).to(dev), dirichlet=torch.from_numpy(mask).to(dev),
                                rho_inf=rho, init_rate=init_rate, lin_tol=1e-13, stream=s_)
    s_.synchronize()
    say(f"  {res}")
    assert res["steps"] == steps
    Th, Uh = T.cpu().numpy(), U.cpu().numpy()
    assert np.abs(Th - T_ref).max() <= 1e-10 * np.abs(T_ref).max()
    assert np.abs(Uh - u_ref).max() <= 1e-9 * max(np.abs(u_ref).max(), 1.0)
    assert np.array_equal(Th[mask != 0], T0[mask != 0])


def test_transient_rate_only_and_errors(mf):
    say("transient rate only / argument errors")
    mesh, k, s, mask, T0 = problem(5)
    dev = torch.device("cuda:0")
    pat = mf.Pattern(torch.from_numpy(mesh.conn).to(dev), mesh.n_nodes, 3, 1)
    coords = torch.from_numpy(mesh.coords).to(dev)
    T = torch.from_numpy(T0.copy()).to(dev)
    U = torch.zeros(mesh.n_nodes, dtype=torch.float64, device=dev)
    res = mf.heat_transient(pat, coords, T, U, 0.1, 0, source=torch.from_numpy(s).to(dev),
                            dirichlet=torch.from_numpy(mask).to(dev), init_rate=True)
    assert res["steps"] == 0 and np.array_equal(T.cpu().numpy(), T0)
    K, M, F = OT.operators(O.Pattern(mesh, 1), 1.0, 1.0, source=s)
    free = mask == 0
    Uh = U.cpu().numpy()
    assert np.abs((M @ Uh - (F - K @ T0))[free]).max() < 1e-10 * np.abs(F).max()
    for bad in (dict(dt=0.0), dict(rho_inf=1.5), dict(capacity=-1.0)):
        kw = dict(dt=0.1, rho_inf=0.5, capacity=1.0) | bad
        with pytest.raises(mf.MFError):
            mf.heat_transient(pat, coords, T, U, kw["dt"], 1, capacity=kw["capacity"], rho_inf=kw["rho_inf"])
    pat3 = mf.Pattern(torch.from_numpy(mesh.conn).to(dev), mesh.n_nodes, 3, 3)
    with pytest.raises(mf.MFError):  # scalar problems only
        mf.heat_transient(pat3, coords, T, U, 0.1, 1)


@pytest.mark.parametrize("init_rate", [True, False])
def test_transient_with_multigrid_matches_oracle(mf, init_rate):
    """mf_heat_transient_mg: the steps' PCG solves preconditioned by the multigrid cycle of
    the effective matrix (5 levels, 16^3 to 1^3) reach the oracle's states as the Jacobi
    solves do, in fewer iterations."""
    say("transient 16^3 multigrid, init_rate", init_rate)
    n, C, kc, dt, steps, rho = 16, 2.0, 1.3, 0.01, 4, 0.5
    mesh, k, s, mask, T0 = problem(n, seed=5)
    u0 = np.zeros(mesh.n_nodes)
    pat_o = O.Pattern(mesh, 1)
    K, M, F = OT.operators(pat_o, C, kc, elem_k=k, source=s)
    T_ref, u_ref = OT.heat_transient(K, M, F, T0, u0, dt, steps, rho=rho, mask=mask, init_rate=init_rate)
    dev = torch.device("cuda:0")
    pat = mf.Pattern(torch.from_numpy(mesh.conn).to(dev), mesh.n_nodes, 3, 1)
    out = {}
    for name, mgo in (("jacobi", None), ("multigrid", dict(coarse_rows=1))):
        T = torch.from_numpy(T0.copy()).to(dev)
        U = torch.from_numpy(u0.copy()).to(dev)
        s_ = torch.cuda.Stream()
        with torch.cuda.stream(s_):
            res = mf.heat_transient(pat, torch.from_numpy(mesh.coords).to(dev), T, U, dt, steps, capacity=C,
                                    conductivity=kc, elem_k=torch.from_numpy(k).to(dev),
                                    source=torch.from_numpy(s).to(dev), dirichlet=torch.from_numpy(mask).to(dev),
                                    rho_inf=rho, init_rate=init_rate, lin_tol=1e-13, stream=s_, multigrid=mgo)
        s_.synchronize()
        say(f"  {name}: {res}")
        assert res["steps"] == steps
        Th, Uh = T.cpu().numpy(), U.cpu().numpy()
        assert np.abs(Th - T_ref).max() <= 1e-10 * np.abs(T_ref).max()
        assert np.abs(Uh - u_ref).max() <= 1e-9 * max(np.abs(u_ref).max(), 1.0)
        assert np.array_equal(Th[mask != 0], T0[mask != 0])
        out[name] = res["lin_iterations"]
    assert out["multigrid"] < out["jacobi"]
