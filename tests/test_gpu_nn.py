"""Learned preconditioner kernels (BF16 inference and training) against the numpy oracle,
and flexible PCG with the network through mf_pcg."""
import sys

import numpy as np
import pytest

import oracle as O
import oracle.nn_ref as NR
import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def bf16(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    u = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def system(n, seed):
    mesh = W.structured_mesh((n, n, n))
    rng = np.random.default_rng(seed)
    k = W.grf_lognormal_elem((n, n, n), float(rng.uniform(1, 2)), 0.1, seed + 1)
    f = W.uniform_nodal(1, mesh.n_nodes, 0, 1, seed + 2)
    mask = W.boundary_node_mask(mesh.shape)
    pat = O.Pattern(mesh, 1)
    K, d = O.assemble(pat, O.POISSON, {"coef": 1.0}, elem_param=k, nodal_src=f, dirichlet=mask)
    return pat, K, d, mask


def bind(mf, net, pat, K, mask):
    rp = torch.from_numpy(pat.row_ptr.astype(np.int32)).cuda()
    ci = torch.from_numpy(pat.col_idx).cuda()
    v = torch.from_numpy(K).cuda()
    m = torch.from_numpy(mask).cuda()
    net.set_system(rp, ci, v, m)
    return rp, ci, v, m


CH = [1, 4, 8, 8]

# Element-wise bars for the BF16 kernels against the FP64 oracle run on the same
# BF16-rounded weights.  Activations are stored in BF16 (unit roundoff 2^-9 = 1.95e-3)
# and accumulated in FP32; an output passes through at most six roundings on its way
# from the input (input scaling, three convolutions, the level sum and the final
# scaling), so no entry may be off by more than 6 x 2^-9 of the largest output.
FWD_TOL = 6 * 2.0 ** -9
# Gradients: every parameter block (one level's convolution) is compared on its own,
# scaled by its largest reference entry.  Each weight gradient is a sum over grid
# points of products of two BF16-rounded activation fields, each a forward or backward
# chain of at most six roundings: 12 x 2^-9 per block.
GRAD_TOL = 12 * 2.0 ** -9


def elementwise_error(z, ref):
    return float(np.max(np.abs(z - ref)) / np.max(np.abs(ref)))


def blockwise_errors(g, gr, channels):
    """max |g - g_ref| / max |g_ref| for each convolution's weight block."""
    errs, o = [], 0
    for a, b, t in NR.param_layout(channels):
        n = a * b * t
        errs.append(elementwise_error(g[o:o + n], gr[o:o + n]))
        o += n
    assert o == g.size == gr.size
    return errs


def test_forward_matches_oracle(mf):
    say("nn forward 17^3")
    pat, K, d, mask = system(16, 7)
    net = mf.Net((17, 17, 17), CH, seed=3)
    theta = NR.init_params(CH, 11).astype(np.float32)
    net.set_params(theta)
    bind(mf, net, pat, K, mask)
    rng = np.random.default_rng(5)
    r = np.where(mask != 0, 0.0, rng.standard_normal(pat.n_rows))
    z = net.apply(torch.from_numpy(r).cuda()).cpu().numpy()
    ref = NR.Net((17, 17, 17), CH).forward(bf16(theta), r, pat.to_scipy(K).diagonal(), mask)
    err = elementwise_error(z, ref)
    say(f"  forward max error / max |z_ref| {err:.2e} (norm {np.linalg.norm(z - ref) / np.linalg.norm(ref):.2e})")
    assert err <= FWD_TOL
    assert np.all(z[mask != 0] == 0.0)
    # linear in r: a power-of-two factor commutes with every BF16 rounding, so exactly
    z2 = net.apply(torch.from_numpy(-4.0 * r).cuda()).cpu().numpy()
    assert np.linalg.norm(z2 + 4.0 * z) <= 1e-6 * np.linalg.norm(z)


def test_forward_large_tiles_matches_oracle(mf):
    """Inference at a size whose first coarse level (37^3 nodes) runs the 8^3-tile fused
    kernel, with ragged tiles on every level; against the oracle."""
    say("nn forward 73^3")
    ch = [1, 4, 8]
    pat, K, d, mask = system(72, 21)
    net = mf.Net((73, 73, 73), ch, seed=3)
    theta = NR.init_params(ch, 13).astype(np.float32)
    net.set_params(theta)
    bind(mf, net, pat, K, mask)
    rng = np.random.default_rng(8)
    r = np.where(mask != 0, 0.0, rng.standard_normal(pat.n_rows))
    z = net.apply(torch.from_numpy(r).cuda()).cpu().numpy()
    ref = NR.Net((73, 73, 73), ch).forward(bf16(theta), r, pat.to_scipy(K).diagonal(), mask)
    err = elementwise_error(z, ref)
    say(f"  forward max error / max |z_ref| {err:.2e} (norm {np.linalg.norm(z - ref) / np.linalg.norm(ref):.2e})")
    assert err <= FWD_TOL
    assert np.all(z[mask != 0] == 0.0)


def test_gradient_matches_oracle(mf):
    say("nn gradient 17^3")
    pat, K, d, mask = system(16, 9)
    net = mf.Net((17, 17, 17), CH, seed=3)
    theta = NR.init_params(CH, 12).astype(np.float32)
    net.set_params(theta)
    bind(mf, net, pat, K, mask)
    rng = np.random.default_rng(6)
    r = np.where(mask != 0, 0.0, rng.standard_normal(pat.n_rows))
    loss, g = net.grad(torch.from_numpy(r).cuda())
    Lr, gr = NR.Net((17, 17, 17), CH).loss_and_grad(bf16(theta), r, pat.to_scipy(K).diagonal(),
                                                     pat.to_scipy(K), mask)
    errs = blockwise_errors(g, gr, CH)
    say(f"  loss {loss:.6f} vs {Lr:.6f}; per-block grad errors " + " ".join(f"{e:.2e}" for e in errs))
    assert abs(loss - Lr) <= FWD_TOL * Lr
    assert max(errs) <= GRAD_TOL
    # parameters are untouched by a gradient query
    assert np.array_equal(net.get_params(), theta)


def test_energy_gradient_matches_oracle(mf):
    say("nn energy gradient 17^3")
    pat, K, d, mask = system(16, 13)
    net = mf.Net((17, 17, 17), CH, seed=3)
    theta = NR.init_params(CH, 14).astype(np.float32)
    net.set_params(theta)
    bind(mf, net, pat, K, mask)
    rng = np.random.default_rng(7)
    S = pat.to_scipy(K)
    e = np.where(mask != 0, 0.0, rng.standard_normal(pat.n_rows))
    Lr, r, gr = NR.energy_loss_and_grad(NR.Net((17, 17, 17), CH), bf16(theta), e, S.diagonal(), S, mask)
    loss, g = net.grad(torch.from_numpy(r).cuda(), e=torch.from_numpy(e).cuda())
    errs = blockwise_errors(g, gr, CH)
    say(f"  loss {loss:.6f} vs {Lr:.6f}; per-block grad errors " + " ".join(f"{e:.2e}" for e in errs))
    assert abs(loss - Lr) <= FWD_TOL * Lr
    assert max(errs) <= GRAD_TOL


def test_training_reduces_loss_and_pcg_converges(mf):
    say("nn train + pcg 16^3")
    pat, K, d, mask = system(16, 21)
    net = mf.Net((17, 17, 17), CH, seed=4)
    rp, ci, v, m = bind(mf, net, pat, K, mask)
    rng = np.random.default_rng(8)
    S = pat.to_scipy(K)
    es = [W.multiscale_nodal(17, len(CH), 40 + k) * (mask == 0) for k in range(8)]
    rs = [torch.from_numpy(S @ e).cuda() for e in es]
    es = [torch.from_numpy(e).cuda() for e in es]
    first = [net.grad(r, e=e)[0] for r, e in zip(rs, es)]
    for it in range(150):
        net.train_step(rs[it % len(rs)], 3e-3, e=es[it % len(es)])
    last = [net.grad(r, e=e)[0] for r, e in zip(rs, es)]
    say(f"  loss {np.mean(first):.4f} -> {np.mean(last):.4f}")
    assert np.mean(last) < 0.7 * np.mean(first)
    b = torch.from_numpy(d).cuda()
    x, res = mf.pcg(rp, ci, v, b, tol=1e-8, precond=mf.PRECOND_NN, net=net, check_every=1)
    _, it_j, _ = O.pcg_jacobi(pat.row_ptr, pat.col_idx, K, d, tol=1e-8)
    say(f"  nn-pcg {res}, jacobi {it_j}")
    assert res["converged"] and res["true_relres"] <= 1e-8
    xh = x.cpu().numpy()
    assert np.linalg.norm(d - S @ xh) / np.linalg.norm(d) <= 1e-8


def test_shipped_weights_beat_jacobi_on_held_out_96(mf):
    """The shipped 96^3 network on systems whose conductivity fields were never seen in
    training (fresh Gaussian-field draws): both solvers reach true relative residual 1e-8
    and the learned preconditioner needs at most half of Jacobi's iterations."""
    import json
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    wpath = os.path.join(root, "paper_2111_03541_amd", "weights", "poisson96")
    assert os.path.exists(wpath + ".npy"), "trained weights missing from the package"
    meta = json.load(open(wpath + ".json"))
    net = mf.Net(tuple(meta["grid"]), meta["channels"], seed=0)
    net.load_params(wpath)
    dev = torch.device("cuda:0")
    n = 96
    mesh = W.structured_mesh((n, n, n))
    pat = mf.Pattern(torch.from_numpy(mesh.conn).to(dev), mesh.n_nodes, 3, 1)
    coords = torch.from_numpy(mesh.coords).to(dev)
    mask = torch.from_numpy(W.boundary_node_mask(mesh.shape)).to(dev)
    rp, ci, _ = pat.device_arrays()
    for seed in (20000, 20001):
        rng = np.random.default_rng(seed)
        sigma = float(rng.uniform(1.0, 2.0))
        say("held-out 96^3 seed", seed, "sigma", round(sigma, 3))
        k = torch.from_numpy(W.grf_lognormal_elem((n, n, n), sigma, 0.1, seed + 1)).to(dev)
        f = torch.from_numpy(W.uniform_nodal(1, mesh.n_nodes, 0, 1, seed + 2)).to(dev)
        K, d = pat.assemble(mf.Form(mf.POISSON, coef=1.0), coords, precision=mf.F64, elem_param=k,
                            nodal_src=f, dirichlet=mask)
        net.set_system(rp, ci, K, mask)
        its = {}
        for name, pc in (("jacobi", mf.PRECOND_JACOBI), ("learned", mf.PRECOND_NN)):
            _, res = mf.pcg(rp, ci, K, d, tol=1e-8, maxit=20000, precond=pc,
                            net=net if pc == mf.PRECOND_NN else None)
            assert res["converged"] and res["true_relres"] <= 1e-8, (name, res)
            its[name] = res["iterations"]
        say("iterations", its)
        assert its["learned"] <= 0.5 * its["jacobi"], its


@pytest.mark.parametrize("bad", ["nan", "zero"])
def test_broken_network_falls_back_to_jacobi(mf, bad):
    """A network whose output is useless (non-finite weights, or all-zero weights so that
    z.r = 0) must not break the solve: each such application takes the Jacobi direction,
    the solve counts it as a fallback and still reaches the 1e-8 true residual in
    Jacobi's iteration count."""
    say("nn fallback", bad)
    pat, K, d, mask = system(16, 31)
    net = mf.Net((17, 17, 17), CH, seed=4)
    rp, ci, v, m = bind(mf, net, pat, K, mask)
    theta = np.zeros(net.n_params, np.float32)
    if bad == "nan":
        theta[:] = 0.01
        theta[5] = np.nan
    net.set_params(theta)
    b = torch.from_numpy(d).cuda()
    x, res = mf.pcg(rp, ci, v, b, tol=1e-8, precond=mf.PRECOND_NN, net=net, check_every=1)
    _, it_j, _ = O.pcg_jacobi(pat.row_ptr, pat.col_idx, K, d, tol=1e-8)
    say(f"  {res}, jacobi {it_j}")
    assert res["converged"] and res["true_relres"] <= 1e-8
    # every application fell back: the initial one and one per iteration
    assert res["fallbacks"] == res["iterations"] + 1
    assert abs(res["iterations"] - it_j) <= max(2, 0.02 * it_j)
    S = pat.to_scipy(K)
    assert np.linalg.norm(d - S @ x.cpu().numpy()) / np.linalg.norm(d) <= 1e-8


def test_checkpoint_resumes_training_exactly(mf, tmp_path):
    """Train 10 steps, checkpoint (parameters, Adam moments, step, seed), train 10 more;
    a fresh network restored from the checkpoint and trained on the same 10 systems ends
    with bitwise the same parameters.  A checkpoint of another architecture is refused."""
    say("nn checkpoint")
    pat, K, d, mask = system(16, 41)
    S = pat.to_scipy(K)
    es = [W.multiscale_nodal(17, len(CH), 60 + k) * (mask == 0) for k in range(4)]
    rs = [torch.from_numpy(S @ e).cuda() for e in es]
    es = [torch.from_numpy(e).cuda() for e in es]
    net = mf.Net((17, 17, 17), CH, seed=9)
    bind(mf, net, pat, K, mask)
    for it in range(10):
        net.train_step(rs[it % 4], 3e-3, e=es[it % 4])
    path = str(tmp_path / "net.ckp")
    net.save_checkpoint(path)
    for it in range(10, 20):
        net.train_step(rs[it % 4], 3e-3, e=es[it % 4])
    a = net.get_params()
    net2 = mf.Net((17, 17, 17), CH, seed=123)
    bind(mf, net2, pat, K, mask)
    assert not np.array_equal(net2.get_params(), a)
    net2.load_checkpoint(path)
    for it in range(10, 20):
        net2.train_step(rs[it % 4], 3e-3, e=es[it % 4])
    b = net2.get_params()
    assert np.array_equal(a, b)
    net3 = mf.Net((17, 17, 17), [1, 4, 8], seed=1)
    with pytest.raises(mf.MFError):
        net3.load_checkpoint(path)
