"""Boundary forms on the GPU (mf_assemble_boundary) against the oracle's face integrals
(oracle/boundary.py), and an end-to-end fix problem solved with the library's kernels."""
import sys

import numpy as np
import pytest

import oracle as O
import oracle.boundary as OB
import workloads as W

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
    kscale = max(abs(Kr).max(), 1e-300)
    assert abs(Kg - Kr).max() <= tol * kscale if kscale > 1e-300 else abs(Kg).max() == 0.0
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
    # an empty face list adds nothing
    K, d = pat.assemble_boundary(mf.BFORM_PENALTY, coords, fe[:0], torch.zeros(0, dtype=torch.uint8, device=dev))
    assert float(K.abs().max()) == 0.0 and float(d.abs().max()) == 0.0
