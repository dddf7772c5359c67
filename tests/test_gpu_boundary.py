"""Boundary forms on the GPU (mf_assemble_boundary) against the oracle's face integrals
(oracle/boundary.py), and an end-to-end fix problem solved with the library's kernels."""
import sys

import numpy as np
import pytest

import oracle as O
import oracle.boundary as OB
import workloads as W
from helpers import rowscaled_sparse

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


N = (4, 3, 5)
S_LOAD = [0.3, -0.2, 0.7, 0.1, 0.5, -0.4, 0.6, 0.2, -1.1]

CASES = [  # (name, kind, nf, coef, value, uses state, uses target)
    ("penalty1", OB.PENALTY, 1, 50.0, [0.7], True, False),
    ("penalty1_target", OB.PENALTY, 1, 50.0, [0.0], True, True),
    ("penalty3", OB.PENALTY, 3, 20.0, [0.1, -0.2, 0.3], True, False),
    ("convection", OB.CONVECTION, 1, 3.0, [2.5], True, False),
    ("radiation", OB.RADIATION, 1, 0.8, [1.3], True, False),
    ("flux", OB.FLUX, 1, 1.7, [0.0], True, False),
    ("traction", OB.TRACTION, 3, 1.0, S_LOAD, False, False),
    ("traction_target", OB.TRACTION, 3, 1.0, [], False, True),
    # flow forms: coef = tau^b, value = (u^w, rho, mu)
    ("ns_inflow", OB.NS_INFLOW, 4, 2.5, [0.4, -0.3, 0.2, 1.2, 0.05], True, False),
    ("ns_inflow_target", OB.NS_INFLOW, 4, 2.5, [0.0, 0.0, 0.0, 1.2, 0.05], True, True),
    ("ns_outflow", OB.NS_OUTFLOW, 4, 0.0, [0.0, 0.0, 0.0, 1.2, 0.05], True, False),
    ("ns_fix", OB.NS_FIX, 4, 2.5, [0.0, 0.0, 0.0, 1.2, 0.05], True, False),
]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("numbering", [0, 1])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_boundary_form_matches_oracle(mf, case, numbering, prec):
    name, kind, nf, coef, value, use_state, use_target = case
    say("boundary", name, "numbering", numbering, "prec", prec)
    mesh = W.structured_mesh(N, jitter=0.2, seed=7, lengths=[1.0, 0.8, 1.5])
    fe, fi = W.box_faces(N)
    # a subset of the faces, unsorted, exercises arbitrary face lists
    sel = np.random.default_rng(1).permutation(fe.shape[0])[: fe.shape[0] * 2 // 3]
    fe, fi = fe[sel], fi[sel]
    rng = np.random.default_rng(3)
    state = 1.0 + rng.random((nf, mesh.n_nodes)) if use_state else None
    target = rng.standard_normal((nf, mesh.n_nodes)) if use_target else None
    fdt = np.float64 if prec == 0 else np.float32
    if prec == 1:  # the oracle takes the same float-rounded inputs
        state = None if state is None else state.astype(np.float32).astype(np.float64)
        target = None if target is None else target.astype(np.float32).astype(np.float64)
    opat = O.Pattern(mesh, nf, numbering=numbering)
    Kr, dr = OB.assemble_boundary(opat, kind, coef, value, fe, fi, state=state, target=target)
    dev = torch.device("cuda:0")
    pat = mf.Pattern(torch.from_numpy(mesh.conn).to(dev), mesh.n_nodes, 3, nf, numbering=numbering)
    tt = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a, dtype=fdt)).to(dev)
    K, d = pat.assemble_boundary(kind, torch.from_numpy(mesh.coords).to(dev), torch.from_numpy(fe).to(dev),
                                 torch.from_numpy(fi).to(dev), coef=coef, value=value, state=tt(state),
                                 target=tt(target), precision=prec)
    assert pat.status()[0] == mf.OK
    Kg = opat.to_scipy(K.double().cpu().numpy())
    dg = d.double().cpu().numpy()
    tol = 1e-12 if prec == 0 else 1e-5
    ek = rowscaled_sparse(Kg, Kr)
    say(f"  row-scaled K err {ek:.3e}")
    assert ek <= tol
    assert np.abs(dg - dr).max() <= tol * max(np.abs(dr).max(), 1e-300)


def test_fix_problem_has_the_linear_field_as_solution(mf):
    """Thermal fix condition on every face (penalty towards T_lin plus the flux term) with
    the domain Laplacian: the linear field is the exact discrete solution for any penalty;
    assembled and solved on the GPU."""
    say("fix problem end to end")
    n = (6, 5, 7)
    mesh = W.structured_mesh(n, jitter=0.2, seed=9, lengths=[1.2, 1.0, 1.4])
    T = 0.3 * mesh.coords[0] - 1.2 * mesh.coords[1] + 0.7 * mesh.coords[2] + 0.4
    dev = torch.device("cuda:0")
    pat = mf.Pattern(torch.from_numpy(mesh.conn).to(dev), mesh.n_nodes, 3, 1)
    coords = torch.from_numpy(mesh.coords).to(dev)
    fe, fi = (torch.from_numpy(a).to(dev) for a in W.box_faces(n))
    k = 1.7
    K, d = pat.assemble(mf.Form(mf.POISSON, coef=k), coords, precision=mf.F64)
    pat.assemble_boundary(mf.BFORM_FLUX, coords, fe, fi, coef=k, K=K, d=d)
    pat.assemble_boundary(mf.BFORM_PENALTY, coords, fe, fi, coef=1e3, K=K, d=d,
                          target=torch.from_numpy(T[None, :].copy()).to(dev))
    rp, ci, _ = pat.device_arrays()
    x, res = mf.bicgstab(rp, ci, K, d, tol=1e-12)
    say(f"  {res}")
    assert res["converged"]
    assert np.abs(x.cpu().numpy() - T).max() < 1e-8 * np.abs(T).max()


def test_boundary_argument_errors(mf):
    say("boundary argument errors")
    mesh = W.structured_mesh((2, 2, 2))
    dev = torch.device("cuda:0")
    pat = mf.Pattern(torch.from_numpy(mesh.conn).to(dev), mesh.n_nodes, 3, 1)
    coords = torch.from_numpy(mesh.coords).to(dev)
    fe = torch.tensor([0, 7], dtype=torch.int32, device=dev)
    # faces out of range are skipped on the device and reported by the status poll
    pat.assemble(mf.Form(mf.POISSON), coords)  # clears the status
    K, d = pat.assemble_boundary(mf.BFORM_PENALTY, coords, fe, torch.tensor([0, 6], dtype=torch.uint8, device=dev))
    assert pat.status()[0] == mf.ERR_ARG  # local face 6
    Kr, dr = pat.assemble_boundary(mf.BFORM_PENALTY, coords, fe[:1], torch.tensor([0], dtype=torch.uint8, device=dev))
    assert torch.equal(K, Kr) and torch.equal(d, dr)  # only the valid face was added
    pat.assemble(mf.Form(mf.POISSON), coords)
    assert pat.status()[0] == mf.OK
    pat.assemble_boundary(mf.BFORM_PENALTY, coords, torch.tensor([0, 8], dtype=torch.int32, device=dev),
                          torch.tensor([0, 1], dtype=torch.uint8, device=dev))
    assert pat.status()[0] == mf.ERR_ARG  # element 8 of 8
    pat.assemble(mf.Form(mf.POISSON), coords)
    with pytest.raises(mf.MFError):  # traction needs 3 fields
        pat.assemble_boundary(mf.BFORM_TRACTION, coords, fe, torch.tensor([0, 1], dtype=torch.uint8, device=dev))
    with pytest.raises(mf.MFError):  # the flow forms need 4 fields
        pat.assemble_boundary(mf.BFORM_NS_OUTFLOW, coords, fe, torch.tensor([0, 1], dtype=torch.uint8, device=dev))
    # an empty face list adds nothing
    K, d = pat.assemble_boundary(mf.BFORM_PENALTY, coords, fe[:0], torch.zeros(0, dtype=torch.uint8, device=dev))
    assert float(K.abs().max()) == 0.0 and float(d.abs().max()) == 0.0



def _pin_positions(rp, ci, r):
    """Positions in a CSR value array of row r and column r, and of their diagonal entry
    (host arrays): replacing that row and column by the identity fixes the pressure level,
    which the flow form with boundary terms on every face leaves free."""
    lo, hi = int(rp[r]), int(rp[r + 1])
    pos = np.union1d(np.nonzero(ci == r)[0], np.arange(lo, hi))
    return torch.from_numpy(pos), lo + int(np.nonzero(ci[lo:hi] == r)[0][0])


def test_cavity_newton_with_weak_boundaries(mf):
    """Lid-driven cavity whose walls (fix) and lid (inflow with a tangential u^w) are all
    weak boundary forms (Sec. 4.3): Newton steps with domain and faces assembled and the
    non-symmetric system solved on the GPU.  The residual falls quadratically and the
    result matches the oracle's Newton iteration with direct solves."""
    import scipy.sparse.linalg as spla
    say("cavity newton, weak boundaries")
    n = (6, 6, 6)
    mesh = W.structured_mesh(n, jitter=0.1, seed=12)
    rho, mu, tau_b = 1.0, 0.05, 10.0
    params = {"rho": rho, "mu": mu, "tau_m": 0.02, "tau_c": 0.05}
    sets = [(OB.NS_INFLOW, W.box_faces(n, sides=[5]), [1.0, 0.0, 0.0, rho, mu]),
            (OB.NS_FIX, W.box_faces(n, sides=[0, 1, 2, 3, 4]), [0.0, 0.0, 0.0, rho, mu])]
    steps = 5
    # oracle
    opat = O.Pattern(mesh, 4)
    sr = np.zeros((4, mesh.n_nodes))
    for _ in range(steps):
        Kr, dr = O.assemble(opat, O.NS_SUPG, params, state=sr)
        Kr = opat.to_scipy(Kr)
        for kind, faces, value in sets:
            Kb, db = OB.assemble_boundary(opat, kind, tau_b, value, *faces, state=sr)
            Kr, dr = Kr + Kb, dr + db
        Kr = Kr.tolil()
        Kr[3, :] = 0.0
        Kr[:, 3] = 0.0
        Kr[3, 3] = 1.0
        dr[3] = 0.0
        sr = sr + spla.spsolve(Kr.tocsr().tocsc(), dr).reshape(-1, 4).T
    # GPU
    dev = torch.device("cuda:0")
    pat = mf.Pattern(torch.from_numpy(mesh.conn).to(dev), mesh.n_nodes, 3, 4)
    coords = torch.from_numpy(mesh.coords).to(dev)
    rp, ci, _ = pat.device_arrays()
    pin, diag = _pin_positions(*pat.arrays()[:2], 3)
    pin = pin.to(dev)
    faces = [(kind, torch.from_numpy(fe).to(dev), torch.from_numpy(fi).to(dev), value)
             for kind, (fe, fi), value in sets]
    st = torch.zeros((4, mesh.n_nodes), dtype=torch.float64, device=dev)
    norms = []
    for _ in range(steps):
        K, d = pat.assemble(mf.Form(mf.NS_SUPG, **params), coords, precision=mf.F64, lin_state=st)
        for kind, fe, fi, value in faces:
            pat.assemble_boundary(kind, coords, fe, fi, coef=tau_b, value=value, state=st, K=K, d=d)
        assert pat.status()[0] == mf.OK
        K[pin] = 0.0
        K[diag] = 1.0
        d[3] = 0.0
        norms.append(float(d.abs().max()))
        x, res = mf.bicgstab(rp, ci, K, d, tol=1e-12)
        assert res["converged"], res
        st += x.view(-1, 4).T
    say(f"  |d| per step {norms}")
    # quadratic: |d_k+1| <= C |d_k|^2 (the oracle's run has C < 1)
    assert all(norms[k + 1] <= 2.0 * norms[k] ** 2 for k in range(1, 3)) and norms[4] < 1e-15 * norms[0]
    sg = st.cpu().numpy()
    assert np.abs(sg - sr).max() < 1e-8 * np.abs(sr).max()
    # recirculation under the lid: the axial velocity changes sign
    assert sg[0].min() < -0.1 and sg[0][np.abs(mesh.coords[2] - 1.0) < 1e-12].mean() > 0.5


# ---------------------------------------------------------------- 2D edges

EDGE_CASES = [  # (name, kind, nf, coef, value, uses state, uses target)
    ("penalty1", OB.PENALTY, 1, 40.0, [0.7], True, False),
    ("penalty2_target", OB.PENALTY, 2, 20.0, [0.0, 0.0], True, True),
    ("convection", OB.CONVECTION, 1, 3.0, [2.5], True, False),
    ("radiation", OB.RADIATION, 1, 0.8, [1.3], True, False),
    ("traction", OB.TRACTION, 2, 1.0, [0.3, -0.7, 0.0, 0.4, 1.1, 0.0, 0.0, 0.0, 0.0], False, False),
    ("traction_target", OB.TRACTION, 2, 1.0, [], False, True),
]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("numbering", [0, 1])
@pytest.mark.parametrize("nen", [4, 8])
@pytest.mark.parametrize("case", EDGE_CASES, ids=[c[0] for c in EDGE_CASES])
def test_edge_form_matches_oracle(mf, case, nen, numbering, prec):
    import oracle.serendipity as S
    name, kind, nf, coef, value, use_state, use_target = case
    say("edge", name, "nen", nen, "numbering", numbering, "prec", prec)
    n, L = (4, 3), [1.2, 0.9]
    mesh = (W.structured_mesh(n, jitter=0.2, seed=3, lengths=L) if nen == 4
            else W.serendipity_mesh_2d(n, jitter=0.2, seed=3, lengths=L))
    fe, fi = W.rect_edges(n)
    sel = np.random.default_rng(5).permutation(fe.shape[0])[: fe.shape[0] * 3 // 4]
    fe, fi = fe[sel], fi[sel]
    rng = np.random.default_rng(6)
    state = 1.0 + rng.random((nf, mesh.n_nodes)) if use_state else None
    target = rng.standard_normal((nf, mesh.n_nodes)) if use_target else None
    fdt = np.float64 if prec == 0 else np.float32
    if prec == 1:
        state = None if state is None else state.astype(np.float32).astype(np.float64)
        target = None if target is None else target.astype(np.float32).astype(np.float64)
    opat = O.Pattern(mesh, nf, numbering=numbering) if nen == 4 else S.Pattern20(mesh, nf, numbering)
    Kr, dr = OB.assemble_boundary_2d(opat, kind, coef, value, fe, fi, state=state, target=target)
    dev = torch.device("cuda:0")
    pat = mf.Pattern(torch.from_numpy(mesh.conn).to(dev), mesh.n_nodes, 2, nf, numbering=numbering)
    tt = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a, dtype=fdt)).to(dev)
    K, d = pat.assemble_boundary(kind, torch.from_numpy(mesh.coords).to(dev), torch.from_numpy(fe).to(dev),
                                 torch.from_numpy(fi).to(dev), coef=coef, value=value, state=tt(state),
                                 target=tt(target), precision=prec)
    assert pat.status()[0] == mf.OK
    Kg = opat.to_scipy(K.double().cpu().numpy())
    dg = d.double().cpu().numpy()
    tol = 1e-12 if prec == 0 else 1e-5
    ek = rowscaled_sparse(Kg, Kr)
    say(f"  row-scaled K err {ek:.3e}")
    assert ek <= tol
    assert np.abs(dg - dr).max() <= tol * max(np.abs(dr).max(), 1e-300)


def test_newton_driver_with_weak_boundaries(mf):
    """The same weakly bounded cavity through the library's Newton driver
    (mf_ns_newton_ex: face sets added every step before the elimination of the one pinned
    pressure DOF): converges and matches the oracle's converged Newton state."""
    import scipy.sparse.linalg as spla
    say("newton driver, weak boundaries")
    n = (6, 6, 6)
    mesh = W.structured_mesh(n, jitter=0.1, seed=12)
    rho, mu, tau_b = 1.0, 0.05, 10.0
    params = {"rho": rho, "mu": mu, "tau_m": 0.02, "tau_c": 0.05}
    sets = [(OB.NS_INFLOW, W.box_faces(n, sides=[5]), [1.0, 0.0, 0.0, rho, mu]),
            (OB.NS_FIX, W.box_faces(n, sides=[0, 1, 2, 3, 4]), [0.0, 0.0, 0.0, rho, mu])]
    opat = O.Pattern(mesh, 4)
    sr = np.zeros((4, mesh.n_nodes))
    for _ in range(6):
        Kr, dr = O.assemble(opat, O.NS_SUPG, params, state=sr)
        Kr = opat.to_scipy(Kr)
        for kind, faces, value in sets:
            Kb, db = OB.assemble_boundary(opat, kind, tau_b, value, *faces, state=sr)
            Kr, dr = Kr + Kb, dr + db
        Kr = Kr.tolil()
        Kr[3, :] = 0.0
        Kr[:, 3] = 0.0
        Kr[3, 3] = 1.0
        dr[3] = 0.0
        sr = sr + spla.spsolve(Kr.tocsr().tocsc(), dr).reshape(-1, 4).T
    dev = torch.device("cuda:0")
    pat = mf.Pattern(torch.from_numpy(mesh.conn).to(dev), mesh.n_nodes, 3, 4)
    coords = torch.from_numpy(mesh.coords).to(dev)
    mask = np.zeros(pat.n_rows, np.uint8)
    mask[3] = 1  # the pressure of node 0
    st = torch.zeros((4, mesh.n_nodes), dtype=torch.float64, device=dev)
    bnd = [(kind, torch.from_numpy(fe).to(dev), torch.from_numpy(fi).to(dev), tau_b, value, None)
           for kind, (fe, fi), value in sets]
    res = mf.ns_newton(pat, mf.Form(mf.NS_SUPG, **params), coords, st, dirichlet=torch.from_numpy(mask).to(dev),
                       rtol=1e-12, lin_tol=1e-12, boundary=bnd)
    say(f"  {res}")
    assert res["converged"] and res["steps"] <= 8
    sg = st.cpu().numpy()
    assert np.abs(sg - sr).max() < 1e-8 * np.abs(sr).max()
    with pytest.raises(mf.MFError):  # a face set whose form does not fit the pattern
        mf.ns_newton(pat, mf.Form(mf.NS_SUPG, **params), coords, st, boundary=[
            (mf.BFORM_TRACTION, bnd[0][1], bnd[0][2], 1.0, [0.0] * 9, None)])


def test_weak_boundary_newton_is_reproducible(mf):
    """The weakly bounded cavity solved twice through mf_ns_newton_ex: the face sets are
    scattered colour bucket by colour bucket, so both runs take the same linear iteration
    counts and end in bitwise-equal states."""
    say("newton driver, weak boundaries, two runs")
    n = (10, 10, 10)
    mesh = W.structured_mesh(n)
    rho, mu, tau_b = 1.0, 0.01, 10.0
    params = {"rho": rho, "mu": mu, "tau_m": 0.02, "tau_c": 0.05}
    sets = [(OB.NS_INFLOW, W.box_faces(n, sides=[5]), [1.0, 0.0, 0.0, rho, mu]),
            (OB.NS_FIX, W.box_faces(n, sides=[0, 1, 2, 3, 4]), [0.0, 0.0, 0.0, rho, mu])]
    dev = torch.device("cuda:0")
    pat = mf.Pattern(torch.from_numpy(mesh.conn).to(dev), mesh.n_nodes, 3, 4)
    coords = torch.from_numpy(mesh.coords).to(dev)
    mask = np.zeros(pat.n_rows, np.uint8)
    mask[3] = 1
    bnd = [(kind, torch.from_numpy(fe).to(dev), torch.from_numpy(fi).to(dev), tau_b, value, None)
           for kind, (fe, fi), value in sets]
    runs = []
    for _ in range(2):
        st = torch.zeros((4, mesh.n_nodes), dtype=torch.float64, device=dev)
        res = mf.ns_newton(pat, mf.Form(mf.NS_SUPG, **params), coords, st,
                           dirichlet=torch.from_numpy(mask).to(dev), rtol=1e-10, lin_tol=1e-10, boundary=bnd)
        say(f"  {res}")
        assert res["converged"]
        runs.append((res, st.cpu().numpy()))
    (r1, s1), (r2, s2) = runs
    assert r1["lin_iterations"] == r2["lin_iterations"] and r1["steps"] == r2["steps"]
    assert np.array_equal(s1, s2)


def test_boundary_form_is_bitwise_reproducible(mf):
    """Penalty faces on a jittered box with every face listed, and a few listed twice:
    two calls give bitwise-equal K and d, and a face listed twice counts twice."""
    say("boundary reproducible")
    n = (7, 6, 5)
    mesh = W.structured_mesh(n, jitter=0.2, seed=3)
    fe, fi = W.box_faces(n)
    dup = np.arange(0, fe.shape[0], 7)
    fe2, fi2 = np.concatenate([fe, fe[dup]]), np.concatenate([fi, fi[dup]])
    dev = torch.device("cuda:0")
    pat = mf.Pattern(torch.from_numpy(mesh.conn).to(dev), mesh.n_nodes, 3, 3)
    coords = torch.from_numpy(mesh.coords).to(dev)
    rng = np.random.default_rng(2)
    target = torch.from_numpy(rng.standard_normal((3, mesh.n_nodes))).to(dev)
    outs = []
    for _ in range(2):
        K, d = pat.assemble_boundary(OB.PENALTY, coords, torch.from_numpy(fe2).to(dev), torch.from_numpy(fi2).to(dev),
                                     coef=1e3, value=[0.0] * 9, target=target)
        assert pat.status()[0] == mf.OK
        outs.append((K.cpu().numpy(), d.cpu().numpy()))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    opat = O.Pattern(mesh, 3)
    Kr, dr = OB.assemble_boundary(opat, OB.PENALTY, 1e3, [0.0] * 9, fe2, fi2, target=target.cpu().numpy())
    assert rowscaled_sparse(opat.to_scipy(outs[0][0]), Kr) <= 1e-12
