"""mf_pcg_noalloc (PCG on the library's fixed device workspace) against mf_pcg through
the C ABI: two solves in a row, the second on a smaller system, each to the same bar as
the PCG parity tests (both reach the 1e-8 true residual, iteration counts within 2%,
solutions within 1e-7 of each other); and the limits it documents."""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def poisson_system(n, seed):
    mesh = W.structured_mesh(n)
    k = W.grf_lognormal_elem(n, 1.5, 0.1, seed)
    f = W.uniform_nodal(1, mesh.n_nodes, 0, 1, seed + 1)
    mask = W.boundary_node_mask(mesh.shape)
    pat = O.Pattern(mesh, 1)
    K, d = O.assemble(pat, O.POISSON, {"coef": 1.0}, elem_param=k, nodal_src=f, dirichlet=mask)
    return pat, K, d


def test_noalloc_pcg_matches_pcg_on_two_calls(mf):
    for n, seed in (((24, 24, 24), 41), ((12, 10, 14), 43)):
        say("pcg_noalloc vs pcg", n)
        pat, K, d = poisson_system(n, seed)
        rp = torch.from_numpy(pat.row_ptr.astype(np.int32)).cuda()
        ci = torch.from_numpy(pat.col_idx).cuda()
        v = torch.from_numpy(K).cuda()
        b = torch.from_numpy(d).cuda()
        x_ref, r_ref = mf.pcg(rp, ci, v, b, tol=1e-8, check_every=1)
        x = torch.full_like(b, np.nan)  # the call overwrites its output entirely
        x, res = mf.pcg_noalloc(rp, ci, v, b, x, tol=1e-8, check_every=1)
        torch.cuda.synchronize()
        say(f"  noalloc {res}; pcg {r_ref}")
        assert res["converged"] and res["true_relres"] <= 1e-8
        assert abs(res["iterations"] - r_ref["iterations"]) <= max(2, 0.02 * r_ref["iterations"])
        xh, xr = x.cpu().numpy(), x_ref.cpu().numpy()
        S = pat.to_scipy(K)
        assert np.linalg.norm(d - S @ xh) / np.linalg.norm(d) <= 1e-8
        assert np.max(np.abs(xh - xr)) <= 1e-7 * np.max(np.abs(xr))


def test_noalloc_pcg_limits(mf):
    say("pcg_noalloc limits")
    nmax = mf.noalloc_max_rows()
    assert nmax == 1 << 20
    # one row more than the workspace holds: rejected before any device work
    n = nmax + 1
    rp = torch.zeros(n + 1, dtype=torch.int32, device="cuda")
    ci = torch.zeros(1, dtype=torch.int32, device="cuda")
    v = torch.zeros(1, dtype=torch.float64, device="cuda")
    b = torch.ones(n, dtype=torch.float64, device="cuda")
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    _, res = mf.pcg_noalloc(rp, ci, v, b, x, raise_on_fail=False)
    assert res["status"] == mf.ERR_ARG
    assert b"workspace" in mf.load().mf_last_error()
    pat, K, d = poisson_system((6, 6, 6), 5)
    rp = torch.from_numpy(pat.row_ptr.astype(np.int32)).cuda()
    ci = torch.from_numpy(pat.col_idx).cuda()
    v = torch.from_numpy(K).cuda()
    b = torch.from_numpy(d).cuda()
    x = torch.zeros_like(b)
    _, res = mf.pcg_noalloc(rp, ci, v, b, x, precond=mf.PRECOND_NN, raise_on_fail=False)
    assert res["status"] == mf.ERR_UNSUPPORTED
    # plain CG on the workspace still converges
    _, res = mf.pcg_noalloc(rp, ci, v, b, x, precond=mf.PRECOND_NONE, check_every=1)
    assert res["converged"] and res["true_relres"] <= 1e-8
