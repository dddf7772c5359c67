"""20-node serendipity hexahedra on the GPU against the numpy oracle (oracle/serendipity.py):
pattern bit-exact, K and d within tolerance, and an end-to-end solve."""
import sys

import numpy as np
import pytest

import oracle as O
import oracle.serendipity as S
import workloads as W
from helpers import rowscaled_sparse

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def gpu_pattern(mf, mesh, nf, numbering=0):
    dev = torch.device("cuda:0")
    return mf.Pattern(torch.from_numpy(mesh.conn).to(dev), mesh.n_nodes, 3, nf, numbering=numbering)


@pytest.mark.parametrize("numbering", [0, 1])
@pytest.mark.parametrize("nf", [1, 3])
def test_pattern_bit_exact(mf, nf, numbering):
    say("hex20 pattern nf", nf, "numbering", numbering)
    mesh = W.serendipity_mesh((3, 2, 3), jitter=0.2, seed=1)
    pat = gpu_pattern(mf, mesh, nf, numbering)
    ref = S.Pattern20(mesh, nf, numbering)
    rp, ci, rk = pat.arrays()
    assert pat.grid()[0] is False
    assert np.array_equal(rp.astype(np.int64), ref.row_ptr) and np.array_equal(ci, ref.col_idx)
    # rank[a*20+b][e] is the position of node b in the sorted neighbours of node a
    for e in (0, mesh.n_elems - 1):
        for a in (0, 7, 8, 19):
            va = mesh.conn[a, e]
            nb = ref.nbr[va]
            for b in range(20):
                assert nb[rk[a * 20 + b, e]] == mesh.conn[b, e]


CASES = [  # (name, kind, nf, params, elem_param, source)
    ("mass", O.MASS, 1, {"coef": 1.7}, False, True),
    ("poisson", O.POISSON, 1, {"coef": 1.3}, True, True),
    ("elasticity", O.ELASTICITY, 3, {"coef": 2.0, "nu": 0.3}, True, True),
]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("numbering", [0, 1])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_assembly_matches_oracle(mf, case, numbering, prec):
    name, kind, nf, prm, use_ep, use_src = case
    say("hex20", name, "numbering", numbering, "prec", prec)
    mesh = W.serendipity_mesh((3, 2, 3), jitter=0.2, seed=2, lengths=[1.0, 0.7, 1.2])
    ep = W.lognormal_elem(mesh.n_elems, 0.4, 3) if use_ep else None
    src = W.uniform_nodal(nf, mesh.n_nodes, -1, 1, 4) if use_src else None
    fdt = np.float64 if prec == 0 else np.float32
    if prec == 1:  # the oracle takes the same float-rounded inputs
        ep = None if ep is None else ep.astype(np.float32).astype(np.float64)
        src = None if src is None else src.astype(np.float32).astype(np.float64)
    ref = S.Pattern20(mesh, nf, numbering)
    Kr, dr = S.assemble20(ref, kind, prm, elem_param=ep, nodal_src=src)
    dev = torch.device("cuda:0")
    pat = gpu_pattern(mf, mesh, nf, numbering)
    tt = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a, dtype=fdt)).to(dev)
    form = mf.Form(kind, coef=prm["coef"], nu=prm.get("nu", 0.0))
    K, d = pat.assemble(form, torch.from_numpy(mesh.coords).to(dev), precision=prec, elem_param=tt(ep),
                        nodal_src=tt(src))
    assert pat.status()[0] == mf.OK
    Kg, dg = K.double().cpu().numpy(), d.double().cpu().numpy()
    tol = 1e-12 if prec == 0 else 1e-5
    # row-scaled error, as for the order-1 forms
    Sr, Sg = ref.to_scipy(Kr), ref.to_scipy(Kg)
    rowmax = np.maximum(abs(Sr).max(axis=1).toarray().ravel(), 1e-300)
    err = abs(Sg - Sr).max(axis=1).toarray().ravel() / rowmax
    assert err.max() <= tol, err.max()
    assert np.abs(dg - dr).max() <= tol * max(np.abs(dr).max(), 1e-300)


def test_quadratic_solution_is_exact(mf):
    """u = x^2 + y z - z^2 / 2 has lap u = 1 and lies in the serendipity space; on an
    affine box with u on the boundary and f = -1, the discrete solution is u itself."""
    say("hex20 quadratic solve")
    n = (4, 3, 5)
    L = [1.0, 0.8, 1.3]
    mesh = W.serendipity_mesh(n, lengths=L)
    c = mesh.coords
    u = c[0] ** 2 + c[1] * c[2] - 0.5 * c[2] ** 2
    hi = np.array(L)[:, None]
    mask = np.any((np.abs(c) < 1e-12) | (np.abs(c - hi) < 1e-12), axis=0).astype(np.uint8)
    dev = torch.device("cuda:0")
    pat = gpu_pattern(mf, mesh, 1)
    K, d = pat.assemble(mf.Form(mf.POISSON, coef=1.0), torch.from_numpy(c).to(dev),
                        nodal_src=torch.full((1, mesh.n_nodes), -1.0, dtype=torch.float64, device=dev))
    # lift the boundary values: solve K w = d - K u_b on the free rows, then u = w + u_b
    ub = np.where(mask != 0, u, 0.0)
    Kub = mf.spmv(*pat.device_arrays()[:2], K, torch.from_numpy(ub).to(dev)).cpu().numpy()
    rhs = np.where(mask != 0, 0.0, d.cpu().numpy() - Kub)
    K2, _ = pat.assemble(mf.Form(mf.POISSON, coef=1.0), torch.from_numpy(c).to(dev),
                         dirichlet=torch.from_numpy(mask).to(dev))
    rp, ci, _ = pat.device_arrays()
    w, res = mf.pcg(rp, ci, K2, torch.from_numpy(rhs).to(dev), tol=1e-13)
    say(f"  {res}")
    assert np.abs(w.cpu().numpy() + ub - u).max() < 1e-9 * np.abs(u).max()


def test_hex20_argument_errors(mf):
    say("hex20 argument errors")
    mesh = W.serendipity_mesh((1, 1, 1))
    dev = torch.device("cuda:0")
    pat = gpu_pattern(mf, mesh, 1)
    coords = torch.from_numpy(mesh.coords).to(dev)
    with pytest.raises(mf.MFError):  # the quadratic element takes 3 points per axis
        pat.assemble(mf.Form(mf.POISSON), coords, points_per_axis=2)
    pat4 = gpu_pattern(mf, mesh, 4)
    st = torch.zeros((3, mesh.n_nodes), dtype=torch.float64, device=dev)
    with pytest.raises(ValueError):  # the flow state holds dim + 1 fields
        pat4.assemble(mf.Form(mf.NS_SUPG, rho=1.0, mu=0.01), coords, lin_state=st)
    with pytest.raises(mf.MFError):  # unknown element type
        mf.Pattern(torch.from_numpy(mesh.conn).to(dev), mesh.n_nodes, 3, 1, elem=7)


# ---------------------------------------------------------------- faces (boundary forms)

import oracle.boundary as OB  # noqa: E402

FACE_CASES = [  # (name, kind, nf, coef, value, uses state, uses target)
    ("penalty1", OB.PENALTY, 1, 40.0, [0.7], True, False),
    ("penalty3_target", OB.PENALTY, 3, 20.0, [0.0, 0.0, 0.0], True, True),
    ("convection", OB.CONVECTION, 1, 3.0, [2.5], True, False),
    ("radiation", OB.RADIATION, 1, 0.8, [1.3], True, False),
    ("traction", OB.TRACTION, 3, 1.0, [0.3, -0.2, 0.7, 0.1, 0.5, -0.4, 0.6, 0.2, -1.1], False, False),
    ("traction_target", OB.TRACTION, 3, 1.0, [], False, True),
]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("numbering", [0, 1])
@pytest.mark.parametrize("case", FACE_CASES, ids=[c[0] for c in FACE_CASES])
def test_boundary_form_matches_oracle(mf, case, numbering, prec):
    name, kind, nf, coef, value, use_state, use_target = case
    say("hex20 boundary", name, "numbering", numbering, "prec", prec)
    n = (3, 2, 2)
    mesh = W.serendipity_mesh(n, jitter=0.2, seed=5, lengths=[1.0, 0.8, 1.3])
    fe, fi = W.box_faces(n)
    sel = np.random.default_rng(2).permutation(fe.shape[0])[: fe.shape[0] * 3 // 4]
    fe, fi = fe[sel], fi[sel]
    rng = np.random.default_rng(4)
    state = 1.0 + rng.random((nf, mesh.n_nodes)) if use_state else None
    target = rng.standard_normal((nf, mesh.n_nodes)) if use_target else None
    fdt = np.float64 if prec == 0 else np.float32
    if prec == 1:
        state = None if state is None else state.astype(np.float32).astype(np.float64)
        target = None if target is None else target.astype(np.float32).astype(np.float64)
    ref = S.Pattern20(mesh, nf, numbering)
    Kr, dr = S.assemble_boundary20(ref, kind, coef, value, fe, fi, state=state, target=target)
    dev = torch.device("cuda:0")
    pat = gpu_pattern(mf, mesh, nf, numbering)
    tt = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a, dtype=fdt)).to(dev)
    K, d = pat.assemble_boundary(kind, torch.from_numpy(mesh.coords).to(dev), torch.from_numpy(fe).to(dev),
                                 torch.from_numpy(fi).to(dev), coef=coef, value=value, state=tt(state),
                                 target=tt(target), precision=prec)
    assert pat.status()[0] == mf.OK
    Kg = ref.to_scipy(K.double().cpu().numpy())
    dg = d.double().cpu().numpy()
    tol = 1e-12 if prec == 0 else 1e-5
    ek = rowscaled_sparse(Kg, Kr)
    say(f"  row-scaled K err {ek:.3e}")
    assert ek <= tol
    assert np.abs(dg - dr).max() <= tol * max(np.abs(dr).max(), 1e-300)


@pytest.mark.parametrize("case", [1, 2, 3])
def test_cantilever_on_the_gpu(mf, case):
    """The paper's 3D cantilever (10 x 4 x 4 quadratic bricks, E = 1, nu = 0, x = 0
    clamped): elasticity and the load assembled on the GPU, solved by Jacobi-PCG; the
    centre-line deflection against the oracle's direct solve and beam theory."""
    sys.path.insert(0, __file__.rsplit("/", 1)[0])
    from test_oracle_serendipity import beam_deflection, cantilever
    say("hex20 cantilever case", case)
    n = (10, 4, 4)
    mesh = W.serendipity_mesh(n, lengths=[10.0, 1.0, 1.0])
    ur = cantilever(case, mesh)
    dev = torch.device("cuda:0")
    pat = gpu_pattern(mf, mesh, 3)
    coords = torch.from_numpy(mesh.coords).to(dev)
    clamp = np.repeat(np.abs(mesh.coords[0]) < 1e-12, 3).astype(np.uint8)
    K, d = pat.assemble(mf.Form(mf.ELASTICITY, coef=1.0, nu=0.0), coords,
                        dirichlet=torch.from_numpy(clamp).to(dev))
    if case == 1:
        sig = [0.0, 0.0, 0.0, -1.0, 0.0, 0.0, 0.0, 0.0, 0.0]  # t = (0, -1, 0) on x = L
        fe, fi = W.box_faces(n, sides=[1])
        tg = None
    else:
        sig = []
        fe, fi = W.box_faces(n, sides=[3])  # the top face y = h
        t = np.zeros((3, mesh.n_nodes))
        t[1] = -(1.0 if case == 2 else 1.0 - mesh.coords[0] / 10.0)
        tg = torch.from_numpy(t).to(dev)
    pat.assemble_boundary(mf.BFORM_TRACTION, coords, torch.from_numpy(fe).to(dev), torch.from_numpy(fi).to(dev),
                          value=sig, target=tg, K=K, d=d)
    assert pat.status()[0] == mf.OK
    d[torch.from_numpy(clamp.astype(bool)).to(dev)] = 0.0  # the load on clamped DOFs is a reaction
    rp, ci, _ = pat.device_arrays()
    # Jacobi-scaled K has cond ~7e6: the attainable relative residual is about 1e-9
    x, res = mf.pcg(rp, ci, K, d, tol=1e-9, maxit=20000)
    say(f"  {res}")
    assert res["converged"]
    u = x.cpu().numpy().reshape(-1, 3)
    c = mesh.coords
    line = np.nonzero((np.abs(c[1] - 0.5) < 1e-12) & (np.abs(c[2] - 0.5) < 1e-12))[0]
    ref = beam_deflection(case, c[0, line])
    tip = np.abs(ref).max()
    assert np.abs(u - ur).max() < 1e-6 * np.abs(ur).max()
    assert np.abs(u[line, 1] - ref).max() < 0.02 * tip


def test_nonfinite_element_parameter_sets_status(mf):
    """A NaN Young's modulus on one 20-node brick is reported as MF_ERR_NONFINITE with
    that element's id."""
    say("hex20 non-finite E")
    mesh = W.serendipity_mesh((3, 2, 2), jitter=0.1, seed=3)
    E = W.lognormal_elem(mesh.n_elems, 0.3, 1)
    E[5] = np.nan
    dev = torch.device("cuda:0")
    pat = gpu_pattern(mf, mesh, 3, 0)
    pat.assemble(mf.Form(mf.ELASTICITY, coef=1.0, nu=0.3), torch.from_numpy(mesh.coords).to(dev),
                 elem_param=torch.from_numpy(E).to(dev))
    assert pat.status() == (mf.ERR_NONFINITE, 5)
