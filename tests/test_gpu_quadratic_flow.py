"""The flow form (Sec. 4.3) on quadratic elements on the GPU against the numpy oracle
(oracle/serendipity.py): 20-node hexahedra, 8-node quadrilaterals and 10-node tetrahedra,
both numberings, FP64 and FP32, at a random state; a non-finite state is reported."""
import sys

import numpy as np
import pytest

import oracle as O
import oracle.serendipity as S
import workloads as W
from helpers import TOL, rowscaled_sparse, vec_error

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

PRM = {"rho": 1.3, "mu": 0.07, "tau_m": 0.02, "tau_c": 0.15}
MESHES = {
    "hex20": lambda: W.serendipity_mesh((3, 2, 3), jitter=0.2, seed=7, lengths=[1.0, 0.7, 1.2]),
    "quad8": lambda: W.serendipity_mesh_2d((5, 4), jitter=0.2, seed=7, lengths=[1.2, 0.9]),
    "tet10": lambda: W.tet10_mesh((2, 3, 2), jitter=0.2, seed=7),
}


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def form(mf):
    return mf.Form(mf.NS_SUPG, rho=PRM["rho"], mu=PRM["mu"], tau_m=PRM["tau_m"], tau_c=PRM["tau_c"])


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("numbering", [0, 1])
@pytest.mark.parametrize("kind", list(MESHES))
def test_flow_form_matches_oracle(mf, kind, numbering, prec):
    say("quadratic flow", kind, "numbering", numbering, "prec", prec)
    mesh = MESHES[kind]()
    dim, nf = mesh.dim, mesh.dim + 1
    state = np.random.default_rng(8).uniform(-1.0, 1.0, (nf, mesh.n_nodes))
    fdt = np.float64 if prec == 0 else np.float32
    state = state.astype(fdt).astype(np.float64)  # the oracle takes the rounded state
    ref = S.Pattern20(mesh, nf, numbering)
    Kr, dr = S.assemble20(ref, O.NS_SUPG, PRM, state=state)
    dev = torch.device("cuda:0")
    pat = mf.Pattern(torch.from_numpy(mesh.conn).to(dev), mesh.n_nodes, dim, nf, numbering=numbering)
    K, d = pat.assemble(form(mf), torch.from_numpy(mesh.coords).to(dev), precision=prec,
                        lin_state=torch.from_numpy(state.astype(fdt)).to(dev))
    assert pat.status()[0] == mf.OK
    ek = rowscaled_sparse(ref.to_scipy(K.double().cpu().numpy()), ref.to_scipy(Kr))
    ed = vec_error(d.double().cpu().numpy(), dr)
    say(f"  row-scaled K err {ek:.3e}  d err {ed:.3e}")
    assert ek <= TOL[prec] and ed <= TOL[prec]


@pytest.mark.parametrize("kind", list(MESHES))
def test_flow_form_nonfinite_state_is_reported(mf, kind):
    say("quadratic flow non-finite state", kind)
    mesh = MESHES[kind]()
    dim, nf = mesh.dim, mesh.dim + 1
    state = np.zeros((nf, mesh.n_nodes))
    e = mesh.n_elems // 2
    state[dim, mesh.conn[0, e]] = np.inf
    bad = set(np.nonzero(np.any(mesh.conn == mesh.conn[0, e], axis=0))[0].tolist())
    dev = torch.device("cuda:0")
    pat = mf.Pattern(torch.from_numpy(mesh.conn).to(dev), mesh.n_nodes, dim, nf)
    pat.assemble(form(mf), torch.from_numpy(mesh.coords).to(dev), lin_state=torch.from_numpy(state).to(dev))
    code, elem = pat.status()
    assert code == mf.ERR_NONFINITE and elem == min(bad)
