"""8-node serendipity quadrilaterals on the GPU against the numpy oracle
(oracle/serendipity.py): pattern bit-exact, K and d within tolerance, and a solve that is
exact for a quadratic field."""
import sys

import numpy as np
import pytest

import oracle as O
import oracle.serendipity as S
import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def gpu_pattern(mf, mesh, nf, numbering=0):
    return mf.Pattern(torch.from_numpy(mesh.conn).to(torch.device("cuda:0")), mesh.n_nodes, 2, nf,
                      numbering=numbering)


@pytest.mark.parametrize("numbering", [0, 1])
@pytest.mark.parametrize("nf", [1, 2])
def test_pattern_bit_exact(mf, nf, numbering):
    say("quad8 pattern nf", nf, "numbering", numbering)
    mesh = W.serendipity_mesh_2d((4, 3), jitter=0.2, seed=1)
    pat = gpu_pattern(mf, mesh, nf, numbering)
    assert pat.elem == mf.QUAD8
    ref = S.Pattern20(mesh, nf, numbering)
    rp, ci, rk = pat.arrays()
    assert pat.grid()[0] is False
    assert np.array_equal(rp.astype(np.int64), ref.row_ptr) and np.array_equal(ci, ref.col_idx)
    for e in (0, mesh.n_elems - 1):
        for a in (0, 3, 4, 7):
            nb = ref.nbr[mesh.conn[a, e]]
            for b in range(8):
                assert nb[rk[a * 8 + b, e]] == mesh.conn[b, e]


CASES = [  # (name, kind, nf, params, elem_param, source)
    ("mass", O.MASS, 1, {"coef": 1.7}, False, True),
    ("poisson", O.POISSON, 1, {"coef": 1.3}, True, True),
    ("elasticity", O.ELASTICITY, 2, {"coef": 2.0, "nu": 0.3}, True, True),
]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("numbering", [0, 1])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_assembly_matches_oracle(mf, case, numbering, prec):
    name, kind, nf, prm, use_ep, use_src = case
    say("quad8", name, "numbering", numbering, "prec", prec)
    mesh = W.serendipity_mesh_2d((5, 3), jitter=0.2, seed=2, lengths=[1.0, 0.7])
    ep = W.lognormal_elem(mesh.n_elems, 0.4, 3) if use_ep else None
    src = W.uniform_nodal(nf, mesh.n_nodes, -1, 1, 4) if use_src else None
    fdt = np.float64 if prec == 0 else np.float32
    if prec == 1:
        ep = None if ep is None else ep.astype(np.float32).astype(np.float64)
        src = None if src is None else src.astype(np.float32).astype(np.float64)
    ref = S.Pattern20(mesh, nf, numbering)
    Kr, dr = S.assemble20(ref, kind, prm, elem_param=ep, nodal_src=src)
    dev = torch.device("cuda:0")
    pat = gpu_pattern(mf, mesh, nf, numbering)
    tt = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a, dtype=fdt)).to(dev)
    K, d = pat.assemble(mf.Form(kind, coef=prm["coef"], nu=prm.get("nu", 0.0)), torch.from_numpy(mesh.coords).to(dev),
                        precision=prec, elem_param=tt(ep), nodal_src=tt(src))
    assert pat.status()[0] == mf.OK
    Kg, dg = K.double().cpu().numpy(), d.double().cpu().numpy()
    tol = 1e-12 if prec == 0 else 1e-5
    Sr, Sg = ref.to_scipy(Kr), ref.to_scipy(Kg)
    rowmax = np.maximum(abs(Sr).max(axis=1).toarray().ravel(), 1e-300)
    err = abs(Sg - Sr).max(axis=1).toarray().ravel() / rowmax
    assert err.max() <= tol, err.max()
    assert np.abs(dg - dr).max() <= tol * max(np.abs(dr).max(), 1e-300)


def test_quadratic_solution_is_exact(mf):
    """u = 1.5 x^2 + x y - y^2 / 2 has lap u = 2 and lies in the element space; on an
    affine rectangle with u on the boundary and f = -2 the discrete solution is u."""
    say("quad8 quadratic solve")
    L = [1.0, 1.4]
    mesh = W.serendipity_mesh_2d((6, 5), lengths=L)
    c = mesh.coords
    u = 1.5 * c[0] ** 2 + c[0] * c[1] - 0.5 * c[1] ** 2
    hi = np.array(L)[:, None]
    mask = np.any((np.abs(c) < 1e-12) | (np.abs(c - hi) < 1e-12), axis=0).astype(np.uint8)
    dev = torch.device("cuda:0")
    pat = gpu_pattern(mf, mesh, 1)
    coords = torch.from_numpy(c).to(dev)
    K, d = pat.assemble(mf.Form(mf.POISSON, coef=1.0), coords,
                        nodal_src=torch.full((1, mesh.n_nodes), -2.0, dtype=torch.float64, device=dev))
    ub = np.where(mask != 0, u, 0.0)
    rp, ci, _ = pat.device_arrays()
    Kub = mf.spmv(rp, ci, K, torch.from_numpy(ub).to(dev)).cpu().numpy()
    rhs = np.where(mask != 0, 0.0, d.cpu().numpy() - Kub)
    K2, _ = pat.assemble(mf.Form(mf.POISSON, coef=1.0), coords, dirichlet=torch.from_numpy(mask).to(dev))
    w, res = mf.pcg(rp, ci, K2, torch.from_numpy(rhs).to(dev), tol=1e-13)
    say(f"  {res}")
    assert np.abs(w.cpu().numpy() + ub - u).max() < 1e-10 * np.abs(u).max()


def test_quad8_argument_errors(mf):
    say("quad8 argument errors")
    mesh = W.serendipity_mesh_2d((2, 1))
    dev = torch.device("cuda:0")
    pat = gpu_pattern(mf, mesh, 1)
    coords = torch.from_numpy(mesh.coords).to(dev)
    with pytest.raises(mf.MFError):  # three points per axis
        pat.assemble(mf.Form(mf.POISSON), coords, points_per_axis=2)
    with pytest.raises(mf.MFError):  # the flow form needs dim + 1 = 3 fields, not 1
        pat.assemble(mf.Form(mf.NS_SUPG, rho=1.0, mu=0.01), coords,
                     lin_state=torch.zeros((3, mesh.n_nodes), dtype=torch.float64, device=dev))
    with pytest.raises(mf.MFError):  # the flux form needs 8-node hexahedra
        pat.assemble_boundary(mf.BFORM_FLUX, coords, torch.zeros(1, dtype=torch.int32, device=dev),
                              torch.zeros(1, dtype=torch.uint8, device=dev))
