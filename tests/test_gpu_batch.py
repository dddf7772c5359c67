"""Batched persistent launch (mf_batch_*) against the oracle and the single-problem path."""
import os
import sys
import tempfile

import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import TOL, rowscaled_error, vec_error

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def make_problems(mf, sizes, prec, seed0=100):
    dt = torch.float64 if prec == mf.F64 else torch.float32
    out, host = [], []
    for p, n in enumerate(sizes):
        mesh = W.structured_mesh(n, jitter=0.2, seed=seed0 + p)
        elastic = p % 2 == 1
        nf = 3 if elastic else 1
        ep = W.lognormal_elem(mesh.n_elems, 0.5, seed0 + 1000 + p)
        src = W.uniform_nodal(nf, mesh.n_nodes, -1 if elastic else 0, 1, seed0 + 2000 + p)
        mask = None
        if p % 3 == 0:
            mask = W.dof_mask(W.boundary_node_mask(mesh.shape), nf, field_major=False)
        pat = mf.Pattern(torch.from_numpy(mesh.conn).cuda(), mesh.n_nodes, 3, nf)
        form = mf.Form(mf.ELASTICITY, coef=1.0, nu=0.3) if elastic else mf.Form(mf.POISSON, coef=1.0)
        out.append({"pattern": pat, "form": form, "coords": torch.from_numpy(mesh.coords).cuda(),
                    "elem_param": torch.from_numpy(ep).to(dt).cuda(),
                    "nodal_src": torch.from_numpy(src).to(dt).cuda(),
                    "dirichlet": None if mask is None else torch.from_numpy(mask).cuda()})
        host.append((mesh, elastic, ep, src, mask))
    return out, host


def rounded(a, prec):
    return a if prec == 0 else np.asarray(a, np.float32).astype(np.float64)


@pytest.mark.parametrize("prec", [0, 1], ids=["f64", "f32"])
def test_batch_matches_oracle(mf, prec):
    sizes = [(3, 2, 2), (5, 4, 3), (2, 7, 3), (9, 3, 4), (1, 1, 1), (6, 6, 5), (4, 9, 2), (3, 3, 8)]
    say("batch", prec, sizes)
    probs, host = make_problems(mf, sizes, prec)
    batch = mf.Batch(probs, precision=prec)
    stream = torch.cuda.Stream()
    batch.run(stream)
    stream.synchronize()
    for pr, (mesh, elastic, ep, src, mask) in zip(batch.problems, host):
        st, bad = pr["pattern"].status()
        assert st == mf.OK
        kind = O.ELASTICITY if elastic else O.POISSON
        params = {"coef": 1.0, "nu": 0.3} if elastic else {"coef": 1.0}
        ref = O.Pattern(mesh, 3 if elastic else 1)
        Kr, dr = O.assemble(ref, kind, params, elem_param=rounded(ep, prec), nodal_src=rounded(src, prec),
                            dirichlet=mask)
        K = pr["K"].double().cpu().numpy()
        d = pr["d"].double().cpu().numpy()
        assert rowscaled_error(ref, K, Kr) <= TOL[prec]
        assert vec_error(d, dr) <= TOL[prec]


def test_batch_graph_replays_and_tuner_cache(mf):
    sizes = [tuple(int(v) for v in s) for s in W.batch_problem_sizes(12, 2, 7, base_seed=40)]
    say("batch replay", sizes)
    probs, _ = make_problems(mf, sizes, 1, seed0=300)
    batch = mf.Batch(probs, precision=mf.F32)
    stream = torch.cuda.Stream()
    with tempfile.TemporaryDirectory() as tmp:
        cache = os.path.join(tmp, "tune.txt")
        info = batch.tune(cache, stream)
        assert info["tuned_us"] > 0 and os.path.exists(cache)
        batch2 = mf.Batch(probs, precision=mf.F32)
        info2 = batch2.tune(cache, stream)  # cache hit: same choice, no timing
        assert info2["order"] == info["order"] and info2["workgroups"] == info["workgroups"]
        assert info2["tuned_us"] == pytest.approx(info["tuned_us"], rel=1e-6)
    batch.run(stream)
    stream.synchronize()
    first = [(p["K"].clone(), p["d"].clone()) for p in batch.problems]
    assert batch.info()["graphed"]
    for rep in range(3):
        # eager work between replays: wipe the outputs
        for p in batch.problems:
            p["K"].fill_(123.0)
            p["d"].zero_()
        torch.cuda.synchronize()
        batch.run(stream)
        stream.synchronize()
        for (K0, d0), p in zip(first, batch.problems):
            assert torch.allclose(p["K"], K0, rtol=1e-5, atol=1e-6 * float(K0.abs().max()))
            assert torch.allclose(p["d"], d0, rtol=1e-5, atol=1e-6 * float(d0.abs().max() + 1e-30))


def test_batch_256_problems_sampled_against_oracle(mf):
    """The full batched workload: 256 problems with n_x, n_y, n_z ~ U{8..48} (seed 6+p),
    +-20% jitter, even p Poisson (lognormal k, f ~ U[0,1]), odd p elasticity (lognormal
    E, nu 0.3, b ~ U[-1,1]), FP32, one persistent launch.  Whole systems of six problems
    (the largest of each form, the first two, two drawn at random) against the oracle."""
    sizes = W.batch_problem_sizes(256, 8, 48, base_seed=6)
    say("batch 256, sizes drawn")
    probs, host = [], []
    for p, n in enumerate(sizes):
        mesh = W.structured_mesh(n, jitter=0.2, seed=6 + p)
        elastic = p % 2 == 1
        nf = 3 if elastic else 1
        ep = W.lognormal_elem(mesh.n_elems, 0.5, 10_000 + p)
        src = W.uniform_nodal(nf, mesh.n_nodes, -1.0 if elastic else 0.0, 1.0, 20_000 + p)
        pat = mf.Pattern(torch.from_numpy(mesh.conn).cuda(), mesh.n_nodes, 3, nf)
        form = mf.Form(mf.ELASTICITY, coef=1.0, nu=0.3) if elastic else mf.Form(mf.POISSON, coef=1.0)
        probs.append({"pattern": pat, "form": form, "coords": torch.from_numpy(mesh.coords).cuda(),
                      "elem_param": torch.from_numpy(ep).float().cuda(),
                      "nodal_src": torch.from_numpy(src).float().cuda()})
        host.append((mesh, elastic, ep, src))
    batch = mf.Batch(probs, precision=mf.F32)
    stream = torch.cuda.Stream()
    info = batch.tune(None, stream)  # the tuned tile shapes are the ones checked
    say("  tuned", info)
    batch.run(stream)
    stream.synchronize()
    el = [p for p in range(256) if p % 2 == 1]
    po = [p for p in range(256) if p % 2 == 0]
    big_e = max(el, key=lambda p: host[p][0].n_elems)
    big_p = max(po, key=lambda p: host[p][0].n_elems)
    rng = np.random.default_rng(0)
    pick = sorted({0, 1, big_e, big_p, *rng.choice(256, 2, replace=False).tolist()})
    for p in pick:
        mesh, elastic, ep, src = host[p]
        say("  problem", p, sizes[p], "elasticity" if elastic else "poisson")
        pr = batch.problems[p]
        assert pr["pattern"].status()[0] == mf.OK
        kind = O.ELASTICITY if elastic else O.POISSON
        params = {"coef": 1.0, "nu": 0.3} if elastic else {"coef": 1.0}
        ref = O.Pattern(mesh, 3 if elastic else 1)
        Kr, dr = O.assemble(ref, kind, params, elem_param=rounded(ep, 1), nodal_src=rounded(src, 1))
        K = pr["K"].double().cpu().numpy()
        d = pr["d"].double().cpu().numpy()
        assert rowscaled_error(ref, K, Kr) <= TOL[1]
        assert vec_error(d, dr) <= TOL[1]


@pytest.mark.parametrize("chunks,xw", [(2, 4), (3, 4), (4, 4), (1, 2), (3, 2)])
def test_batch_tile_shapes_match_oracle(mf, chunks, xw):
    """Every class's columns with an xw x (8 / xw) node cross-section, cut into `chunks`
    tiles along z (set through the tuner's cache file, which the tuner then reads back):
    whole systems against the oracle."""
    sizes = [(3, 2, 7), (5, 4, 9), (2, 3, 22), (4, 3, 25), (3, 3, 40), (2, 2, 37), (1, 1, 5), (6, 2, 3)]
    say("batch tiles", chunks, xw, sizes)
    probs, host = make_problems(mf, sizes, 1, seed0=500)
    stream = torch.cuda.Stream()
    with tempfile.TemporaryDirectory() as tmp:
        cache = os.path.join(tmp, "tune.txt")
        mf.Batch(probs, precision=mf.F32).tune(cache, stream)
        key, order, mult, us, *_ = open(cache).read().split()
        with open(cache, "w") as f:
            f.write(" ".join([key, order, mult, us] + [str(chunks)] * 6 + [str(xw)] * 6) + "\n")
        batch = mf.Batch(probs, precision=mf.F32)
        info = batch.tune(cache, stream)
    shape = f"{xw}x{8 // xw}"
    assert all(t["chunks"] == chunks and t["cross_section"] == shape for t in info["tiles"].values()), info
    batch.run(stream)
    stream.synchronize()
    for pr, (mesh, elastic, ep, src, mask) in zip(batch.problems, host):
        assert pr["pattern"].status()[0] == mf.OK
        kind = O.ELASTICITY if elastic else O.POISSON
        params = {"coef": 1.0, "nu": 0.3} if elastic else {"coef": 1.0}
        ref = O.Pattern(mesh, 3 if elastic else 1)
        Kr, dr = O.assemble(ref, kind, params, elem_param=rounded(ep, 1), nodal_src=rounded(src, 1),
                            dirichlet=mask)
        assert rowscaled_error(ref, pr["K"].double().cpu().numpy(), Kr) <= TOL[1]
        assert vec_error(pr["d"].double().cpu().numpy(), dr) <= TOL[1]
