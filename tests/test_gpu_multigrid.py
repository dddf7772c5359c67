"""The geometric multigrid preconditioner (mf_mg_*) and the Newton driver that uses it
(mf_ns_newton_mg) on the GPU, against the oracle's V-cycle (oracle/multigrid.py), which
assembles every level itself from the same seeded inputs.

Tolerance of one cycle: max |z - z_ref| <= 1e-12 max |z_ref|.  Both sides run the same
sweeps in FP64 and differ only in the order of the additions (SpMV rows, restriction
stencils, the assembly's element sums).  A few tens of sweeps, each contractive, keep
that rounding at a few units of 1e-16 times the operators' condition of one sweep
(measured: 4e-16 to 2.3e-15 over the cases below); the bar leaves more than two orders of
margin.
"""
import sys

import numpy as np
import pytest

import oracle as O
import oracle.multigrid as MG
import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = 1e-12


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def taus(n, U=1.0, nu=0.01):
    h = 1.0 / n
    tm = ((2 * U / h) ** 2 + 9 * (4 * nu / h ** 2) ** 2) ** -0.5
    return tm, h * h / (12 * tm)


def flow_params(n, levels):
    """The form's constants on each level (element size 2^l / n)."""
    out = []
    for l in range(levels):
        tm, tc = taus(n / 2 ** l)
        out.append(dict(rho=1.0, mu=0.01, tau_m=tm, tau_c=tc))
    return out


def flow_case(n, numbering, seed, jitter=0.1):
    mesh = W.structured_mesh((n, n, n), jitter=jitter, seed=seed)
    st, mask = W.flow_boundary(mesh, "cavity", field_major=numbering == O.FIELD_MAJOR)
    interior = 1 - W.boundary_node_mask(mesh.shape)
    st[:3] += 0.5 * W.fourier_velocity(mesh.coords, seed + 1) * interior[None, :]
    st[3] = W.uniform_nodal(1, mesh.n_nodes, -0.2, 0.2, seed + 2)[0]
    return mesh, st, mask


def gpu_cycle(mf, mesh, nf, form, prm_levels, state, mask, numbering, r, **opts):
    dev = torch.device("cuda:0")
    pat = mf.Pattern(torch.from_numpy(mesh.conn).to(dev), mesh.n_nodes, 3, nf, numbering=numbering)
    coords = torch.from_numpy(mesh.coords).to(dev)
    st = None if state is None else torch.from_numpy(state).to(dev).contiguous()
    dm = None if mask is None else torch.from_numpy(mask).to(dev)
    K, _ = pat.assemble(form, coords, precision=mf.F64, lin_state=st, dirichlet=dm)
    tm = [p.get("tau_m", 0.0) for p in prm_levels]
    tc = [p.get("tau_c", 0.0) for p in prm_levels]
    mg = mf.Multigrid(pat, tau_m=tm, tau_c=tc, **opts)
    mg.update(form, coords, K, lin_state=st, dirichlet=dm)
    z = mg.apply(torch.from_numpy(r).to(dev))
    torch.cuda.synchronize()
    return mg, z.cpu().numpy()


def oracle_cycle(dims, mesh, nf, kind, prm_levels, n_levels, state, mask, numbering, r, pre=2, post=2,
                 coarse_sweeps=20, omega=0.5):
    levels = MG.build_levels(dims, mesh.coords, nf, kind, prm_levels, n_levels, state=state, dirichlet=mask,
                             numbering=numbering)
    return MG.vcycle(levels, r, omega=omega, pre=pre, post=post, coarse_sweeps=coarse_sweeps)


def test_levels_follow_the_coarsening_rule(mf):
    say("multigrid levels")
    dev = torch.device("cuda:0")
    cases = [((16, 16, 16), 4, {}, [(16, 16, 16), (8, 8, 8), (4, 4, 4)]),
             ((12, 8, 6), 1, dict(coarse_rows=1), [(12, 8, 6), (6, 4, 3)]),
             ((16, 16, 16), 4, dict(max_levels=2), [(16, 16, 16), (8, 8, 8)]),
             ((6, 6, 6), 1, {}, [(6, 6, 6)])]
    for dims, nf, opts, expect in cases:
        mesh = W.structured_mesh(dims)
        pat = mf.Pattern(torch.from_numpy(mesh.conn).to(dev), mesh.n_nodes, 3, nf)
        assert mf.Multigrid(pat, **opts).levels() == expect, (dims, opts)


@pytest.mark.parametrize("numbering", [O.NODE_MAJOR, O.FIELD_MAJOR])
@pytest.mark.parametrize("coarse_rows", [0, 1])
def test_flow_cycle_matches_oracle(mf, numbering, coarse_rows):
    """16^3 jittered cavity at a random state: 3 levels down to 4^3 (default), or 5 down to
    1^3 (coarse_rows = 1)."""
    n = 16
    say(f"flow cycle {n}^3 numbering {numbering} coarse_rows {coarse_rows}")
    mesh, st, mask = flow_case(n, numbering, 7)
    n_levels = 3 if coarse_rows == 0 else 5
    prm = flow_params(n, n_levels)
    r = np.random.default_rng(8).standard_normal(mesh.n_nodes * 4)
    form = mf.Form(mf.NS_SUPG, **prm[0])
    mg, z = gpu_cycle(mf, mesh, 4, form, prm, st, mask, numbering, r, coarse_rows=coarse_rows)
    assert len(mg.levels()) == n_levels
    z_ref = oracle_cycle((n, n, n), mesh, 4, O.NS_SUPG, prm, n_levels, st, mask, numbering, r)
    err = np.abs(z - z_ref).max() / np.abs(z_ref).max()
    say(f"  rel err {err:.2e}")
    assert err <= TOL


@pytest.mark.parametrize("kind,nf,prm,dims,opts,n_levels", [
    (O.POISSON, 1, dict(coef=1.3), (8, 12, 6), dict(coarse_rows=1, pre_sweeps=1, post_sweeps=3), 2),
    (O.ELASTICITY, 3, dict(coef=1.0, nu=0.3), (8, 8, 4), dict(coarse_rows=1, coarse_sweeps=7, omega=0.6), 3),
    # the coarsest level has more rows than one workgroup holds: sweeps launched one by one
    (O.POISSON, 1, dict(coef=1.0), (32, 32, 32), dict(max_levels=2, coarse_sweeps=5), 2),
    (O.POISSON, 1, dict(coef=1.0), (18, 18, 18), dict(max_levels=1, coarse_sweeps=4), 1),
    (O.POISSON, 1, dict(coef=1.0), (8, 8, 8), dict(coarse_rows=1, pre_sweeps=0, post_sweeps=1,
                                                   coarse_sweeps=0), 4),
    # the benchmark's V(1,1) at omega 0.6, and an odd total of sweeps per level
    (O.POISSON, 1, dict(coef=1.0), (16, 16, 16), dict(pre_sweeps=1, post_sweeps=1, omega=0.6), 3),
    (O.ELASTICITY, 3, dict(coef=1.0, nu=0.3), (8, 8, 8), dict(coarse_rows=1, pre_sweeps=2, post_sweeps=1), 4),
])
def test_symmetric_form_cycle_matches_oracle(mf, kind, nf, prm, dims, opts, n_levels):
    say(f"cycle kind {kind} dims {dims} opts {opts}")
    mesh = W.structured_mesh(dims, jitter=0.12, seed=11)
    mask = W.dof_mask(W.boundary_node_mask(mesh.shape), nf, False)
    r = np.random.default_rng(12).standard_normal(mesh.n_nodes * nf)
    form = mf.Form({O.POISSON: mf.POISSON, O.ELASTICITY: mf.ELASTICITY}[kind], **prm)
    mg, z = gpu_cycle(mf, mesh, nf, form, [prm] * n_levels, None, mask, O.NODE_MAJOR, r, **opts)
    assert len(mg.levels()) == n_levels
    kw = dict(pre=opts.get("pre_sweeps", 2), post=opts.get("post_sweeps", 2),
              coarse_sweeps=opts.get("coarse_sweeps", 20), omega=opts.get("omega", 0.5))
    z_ref = oracle_cycle(dims, mesh, nf, kind, [prm] * n_levels, n_levels, None, mask, O.NODE_MAJOR, r, **kw)
    err = np.abs(z - z_ref).max() / np.abs(z_ref).max()
    say(f"  rel err {err:.2e}")
    assert err <= TOL


def test_bicgstab_with_multigrid_beats_jacobi(mf):
    """The 24^3 cavity tangent at a random state: multigrid-preconditioned BiCGStab meets
    1e-10 in a fraction of the Jacobi iterations; graph replay and eager launches give the
    same iterate bit for bit."""
    n = 24
    say(f"bicgstab multigrid {n}^3")
    dev = torch.device("cuda:0")
    mesh, st, mask = flow_case(n, O.NODE_MAJOR, 21, jitter=0.0)
    prm = flow_params(n, 4)
    pat = mf.Pattern(torch.from_numpy(mesh.conn).to(dev), mesh.n_nodes, 3, 4)
    coords = torch.from_numpy(mesh.coords).to(dev)
    stt = torch.from_numpy(st).to(dev).contiguous()
    dm = torch.from_numpy(mask).to(dev)
    form = mf.Form(mf.NS_SUPG, **prm[0])
    K, d = pat.assemble(form, coords, lin_state=stt, dirichlet=dm)
    mg = mf.Multigrid(pat, tau_m=[p["tau_m"] for p in prm], tau_c=[p["tau_c"] for p in prm])
    mg.update(form, coords, K, lin_state=stt, dirichlet=dm)
    rp, ci, _ = pat.device_arrays()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        x1, r1 = mf.bicgstab(rp, ci, K, d, tol=1e-10, precond=mf.PRECOND_MG, mg=mg, stream=s)
        x2, r2 = mf.bicgstab(rp, ci, K, d, tol=1e-10, precond=mf.PRECOND_MG, mg=mg, stream=s, use_graph=False)
        _, rj = mf.bicgstab(rp, ci, K, d, tol=1e-10, precond=mf.PRECOND_JACOBI, stream=s, raise_on_fail=False)
    s.synchronize()
    say(f"  mg {r1} jacobi {rj}")
    assert r1["converged"] and r1["true_relres"] <= 1e-10
    assert r2["iterations"] == r1["iterations"] and torch.equal(x1, x2)
    assert r1["iterations"] * 5 <= rj["iterations"]
    # the solution solves the oracle's own system
    opat = O.Pattern(mesh, 4)
    Ko, do = O.assemble(opat, O.NS_SUPG, prm[0], state=st, dirichlet=mask)
    assert np.linalg.norm(do - opat.to_scipy(Ko) @ x1.cpu().numpy()) <= 1e-9 * np.linalg.norm(do)


def test_pcg_with_multigrid_on_conduction(mf):
    """32^3 jittered conduction with Dirichlet walls: multigrid-preconditioned (flexible)
    PCG against Jacobi-PCG and the oracle's PCG solution."""
    n = 32
    say(f"pcg multigrid {n}^3")
    dev = torch.device("cuda:0")
    mesh = W.structured_mesh((n, n, n), jitter=0.15, seed=5)
    mask = W.boundary_node_mask(mesh.shape)
    f = W.uniform_nodal(1, mesh.n_nodes, 0, 1, 6)
    pat = mf.Pattern(torch.from_numpy(mesh.conn).to(dev), mesh.n_nodes, 3, 1)
    coords = torch.from_numpy(mesh.coords).to(dev)
    dm = torch.from_numpy(mask).to(dev)
    form = mf.Form(mf.POISSON, coef=1.0)
    K, d = pat.assemble(form, coords, nodal_src=torch.from_numpy(f).to(dev), dirichlet=dm)
    mg = mf.Multigrid(pat)
    mg.update(form, coords, K, dirichlet=dm)
    s = torch.cuda.Stream()
    rp, ci, _ = pat.device_arrays()
    with torch.cuda.stream(s):
        x, res = mf.pcg(rp, ci, K, d, tol=1e-10, precond=mf.PRECOND_MG, mg=mg, stream=s)
        _, rj = mf.pcg(rp, ci, K, d, tol=1e-10, stream=s)
    s.synchronize()
    say(f"  mg {res} jacobi {rj}")
    assert res["converged"] and res["iterations"] * 4 <= rj["iterations"]
    opat = O.Pattern(mesh, 1)
    Ko, do = O.assemble(opat, O.POISSON, {"coef": 1.0}, nodal_src=f, dirichlet=mask)
    xo, _, _ = O.pcg_jacobi(opat.row_ptr, opat.col_idx, Ko, do, tol=1e-12)
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-8 * np.linalg.norm(xo)


def test_multigrid_errors(mf):
    say("multigrid errors")
    dev = torch.device("cuda:0")
    mesh = W.structured_mesh((4, 4, 4))
    pat = mf.Pattern(torch.from_numpy(mesh.conn).to(dev), mesh.n_nodes, 3, 1)
    coords = torch.from_numpy(mesh.coords).to(dev)
    form = mf.Form(mf.POISSON, coef=1.0)
    K, d = pat.assemble(form, coords)
    rp, ci, _ = pat.device_arrays()
    # bad options
    for bad in (dict(omega=0.0), dict(omega=1.5), dict(pre_sweeps=-1), dict(max_levels=9)):
        with pytest.raises(mf.MFError) as e:
            mf.Multigrid(pat, **bad)
        assert e.value.status == mf.ERR_ARG
    mg = mf.Multigrid(pat, coarse_rows=1)
    # apply before update
    with pytest.raises(mf.MFError) as e:
        mg.apply(d)
    assert e.value.status == mf.ERR_ARG
    mg.update(form, coords, K)
    # r and z the same vector
    with pytest.raises(mf.MFError):
        mg.apply(d, d)
    # a solve on a different matrix than the one the cycle was updated for
    K2 = K.clone()
    with pytest.raises(mf.MFError) as e:
        mf.bicgstab(rp, ci, K2, d, precond=mf.PRECOND_MG, mg=mg)
    assert e.value.status == mf.ERR_ARG
    # no cycle given
    with pytest.raises(mf.MFError):
        mf.pcg(rp, ci, K, d, precond=mf.PRECOND_MG)
    # coarse levels take no right side
    with pytest.raises(mf.MFError) as e:
        lib = mf.load()
        F = mf._Fields(None, mf._ptr(torch.ones(pat.n_nodes, dtype=torch.float64, device=dev)), None, None)
        mf.check(lib.mf_mg_update(mg.handle, mf.C.byref(form.c), mf._ptr(coords), mf.C.byref(F),
                                  mf.C.byref(mf._Quad(2)), mf._ptr(K), mf._stream()))
    assert e.value.status == mf.ERR_UNSUPPORTED
    # not a structured grid: a permuted node numbering
    perm = np.random.default_rng(0).permutation(mesh.n_nodes)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(mesh.n_nodes)
    patp = mf.Pattern(torch.from_numpy(inv[mesh.conn].astype(np.int32)).to(dev), mesh.n_nodes, 3, 1)
    with pytest.raises(mf.MFError) as e:
        mf.Multigrid(patp)
    assert e.value.status == mf.ERR_UNSUPPORTED
    # the noalloc solver takes no cycle
    with pytest.raises(mf.MFError):
        mf.pcg_noalloc(rp, ci, K, d, torch.empty_like(d), precond=mf.PRECOND_MG)


def newton_mg(mf, n, multigrid=True, **kw):
    """The lid-driven cavity on an n^3 grid from rest; returns (state, result, st0, mask)."""
    dev = torch.device("cuda:0")
    mesh = W.structured_mesh((n, n, n))
    prm = flow_params(n, 8)
    pat = mf.Pattern(torch.from_numpy(mesh.conn).to(dev), mesh.n_nodes, 3, 4)
    st0, mask = W.flow_boundary(mesh, "cavity")
    state = torch.from_numpy(st0).to(dev).contiguous()
    coords = torch.from_numpy(mesh.coords).to(dev)
    form = mf.Form(mf.NS_SUPG, **prm[0])
    mgo = dict(tau_m=[p["tau_m"] for p in prm], tau_c=[p["tau_c"] for p in prm]) if multigrid else None
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        res = mf.ns_newton(pat, form, coords, state, dirichlet=torch.from_numpy(mask).to(dev), stream=s,
                           multigrid=mgo, **kw)
    s.synchronize()
    return mesh, state.cpu().numpy(), res, st0, mask


def test_newton_with_multigrid_matches_jacobi_newton(mf):
    """16^3 cavity: the multigrid and Jacobi Newton solves reach the same discrete solution
    with far fewer linear iterations."""
    say("newton multigrid vs jacobi 16^3")
    _, st_mg, r_mg, _, _ = newton_mg(mf, 16, rtol=1e-11, lin_tol=1e-11)
    _, st_j, r_j, _, _ = newton_mg(mf, 16, multigrid=False, rtol=1e-11, lin_tol=1e-11)
    say(f"  mg {r_mg['steps']} steps {r_mg['lin_iterations']} it; jacobi {r_j['steps']} steps "
        f"{r_j['lin_iterations']} it")
    assert r_mg["converged"] and r_j["converged"]
    assert r_mg["lin_iterations"] * 4 <= r_j["lin_iterations"]
    assert np.abs(st_mg - st_j).max() <= 1e-8 * np.abs(st_j).max()


def test_newton_cavity_48_with_multigrid_converges_reproducibly(mf):
    """The cavity on the flow Jacobian's 48^3 mesh (470,596 unknowns), where Jacobi-BiCGStab
    breaks down: Newton with the multigrid-preconditioned BiCGStab (5 levels, 48^3 to 3^3)
    converges to |R| / |R_0| <= 1e-10; two runs take the same linear iterations and end in
    the same state bit for bit; the oracle's own residual of that state meets the test."""
    n = 48
    say(f"newton multigrid cavity {n}^3")
    mesh, st, res, st0, mask = newton_mg(mf, n, rtol=1e-10, lin_tol=1e-10)
    say(f"  steps {res['steps']} lin {res['lin_iterations']} res {['%.2e' % r for r in res['res_norm']]}")
    assert res["converged"] and res["steps"] <= 8
    assert res["lin_iterations"] <= 400
    _, st2, res2, _, _ = newton_mg(mf, n, rtol=1e-10, lin_tol=1e-10)
    assert res2["lin_iterations"] == res["lin_iterations"] and np.array_equal(st2, st)
    pat = O.Pattern(mesh, 4)
    prm = flow_params(n, 1)[0]
    _, d0 = O.assemble(pat, O.NS_SUPG, prm, state=st0, dirichlet=mask, want_K=False)
    _, d = O.assemble(pat, O.NS_SUPG, prm, state=st, dirichlet=mask, want_K=False)
    assert abs(res["res_norm"][0] - np.linalg.norm(d0)) <= 1e-12 * np.linalg.norm(d0)
    assert np.linalg.norm(d) <= 1e-10 * np.linalg.norm(d0)


def weak_cavity_sets(dims, rho=1.0, mu=0.01):
    """The cavity's walls as weak boundary forms: the lid (side 5) as inflow with
    u^w = (1, 0, 0), the other five sides as fix."""
    import oracle.boundary as OB
    return [(OB.NS_INFLOW, W.box_faces(dims, sides=[5]), [1.0, 0.0, 0.0, rho, mu]),
            (OB.NS_FIX, W.box_faces(dims, sides=[0, 1, 2, 3, 4]), [0.0, 0.0, 0.0, rho, mu])]


@pytest.mark.parametrize("numbering", [O.NODE_MAJOR, O.FIELD_MAJOR])
def test_flow_cycle_with_face_sets_matches_oracle(mf, numbering):
    """A jittered 16^3 cavity whose walls are weak boundary forms (no Dirichlet rows), at a
    random state: the face sets coarsened onto every level (3 levels, 16^3 to 4^3)."""
    n = 16
    say(f"flow cycle with face sets {n}^3 numbering {numbering}")
    dev = torch.device("cuda:0")
    mesh, st, _ = flow_case(n, numbering, 31)
    prm = flow_params(n, 3)
    tau_b = 10.0
    sets = weak_cavity_sets((n, n, n))
    pat = mf.Pattern(torch.from_numpy(mesh.conn).to(dev), mesh.n_nodes, 3, 4, numbering=numbering)
    coords = torch.from_numpy(mesh.coords).to(dev)
    stt = torch.from_numpy(st).to(dev).contiguous()
    form = mf.Form(mf.NS_SUPG, **prm[0])
    K, d = pat.assemble(form, coords, lin_state=stt)
    bnd = [(k, torch.from_numpy(fe).to(dev), torch.from_numpy(fi).to(dev), tau_b, v, None) for k, (fe, fi), v in sets]
    for k, fe, fi, c, v, _ in bnd:
        pat.assemble_boundary(k, coords, fe, fi, coef=c, value=v, state=stt, K=K, d=d)
    mg = mf.Multigrid(pat, tau_m=[p["tau_m"] for p in prm], tau_c=[p["tau_c"] for p in prm])
    mg.update(form, coords, K, lin_state=stt, boundary=bnd)
    r = np.random.default_rng(32).standard_normal(pat.n_rows)
    z = mg.apply(torch.from_numpy(r).to(dev)).cpu().numpy()
    face_sets = [(k, tau_b, v, fe, fi, None) for k, (fe, fi), v in sets]
    levels = MG.build_levels((n, n, n), mesh.coords, 4, O.NS_SUPG, prm, 3, state=st, numbering=numbering,
                             face_sets=face_sets)
    z_ref = MG.vcycle(levels, r)
    err = np.abs(z - z_ref).max() / np.abs(z_ref).max()
    say(f"  rel err {err:.2e}")
    assert err <= TOL


def weak_newton(mf, n, multigrid, jitter=0.0, seed=None, **kw):
    dev = torch.device("cuda:0")
    dims = (n, n, n)
    mesh = W.structured_mesh(dims, jitter=jitter, seed=seed)
    prm = flow_params(n, 8)
    pat = mf.Pattern(torch.from_numpy(mesh.conn).to(dev), mesh.n_nodes, 3, 4)
    coords = torch.from_numpy(mesh.coords).to(dev)
    mask = np.zeros(pat.n_rows, np.uint8)
    mask[3] = 1  # the pressure of node 0
    bnd = [(k, torch.from_numpy(fe).to(dev), torch.from_numpy(fi).to(dev), 10.0, v, None)
           for k, (fe, fi), v in weak_cavity_sets(dims)]
    st = torch.zeros((4, mesh.n_nodes), dtype=torch.float64, device=dev)
    mgo = dict(tau_m=[p["tau_m"] for p in prm], tau_c=[p["tau_c"] for p in prm]) if multigrid else None
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        res = mf.ns_newton(pat, mf.Form(mf.NS_SUPG, **prm[0]), coords, st, dirichlet=torch.from_numpy(mask).to(dev),
                           boundary=bnd, multigrid=mgo, stream=s, **kw)
    s.synchronize()
    return st.cpu().numpy(), res


def test_weak_boundary_newton_with_multigrid(mf):
    """The weakly bounded cavity: on a jittered 8^3 mesh the multigrid Newton reaches the
    Jacobi Newton's state; on 32^3 it converges in a fraction of the Jacobi iterations, the
    same on two runs, bit for bit."""
    say("weak-boundary newton with multigrid")
    st_mg, r_mg = weak_newton(mf, 8, True, jitter=0.1, seed=12, rtol=1e-12, lin_tol=1e-12)
    st_j, r_j = weak_newton(mf, 8, False, jitter=0.1, seed=12, rtol=1e-12, lin_tol=1e-12)
    say(f"  8^3: mg {r_mg['steps']} steps {r_mg['lin_iterations']} it; jacobi {r_j['steps']} steps "
        f"{r_j['lin_iterations']} it")
    assert r_mg["converged"] and r_j["converged"]
    assert np.abs(st_mg - st_j).max() <= 1e-8 * np.abs(st_j).max()
    st1, r1 = weak_newton(mf, 32, True, rtol=1e-10, lin_tol=1e-10)
    st2, r2 = weak_newton(mf, 32, True, rtol=1e-10, lin_tol=1e-10)
    say(f"  32^3: {r1['steps']} steps {r1['lin_iterations']} it, res {['%.2e' % r for r in r1['res_norm']]}")
    assert r1["converged"] and r1["steps"] <= 8 and r1["lin_iterations"] <= 300
    assert r2["lin_iterations"] == r1["lin_iterations"] and np.array_equal(st1, st2)


@pytest.mark.parametrize("kind,nf,prm,dims,jitter", [
    (O.POISSON, 1, dict(coef=1.0), (16, 16, 16), 0.15),
    (O.ELASTICITY, 3, dict(coef=1.0, nu=0.3), (8, 8, 12), 0.1),
])
def test_cycle_with_a_coefficient_field_matches_oracle(mf, kind, nf, prm, dims, jitter):
    """A lognormal element coefficient (conductivity, Young's modulus) carried to the coarse
    levels as the mean of the children."""
    say(f"cycle with coefficient field kind {kind} dims {dims}")
    dev = torch.device("cuda:0")
    mesh = W.structured_mesh(dims, jitter=jitter, seed=41)
    k = W.lognormal_elem(mesh.n_elems, 1.0, 42)
    mask = W.dof_mask(W.boundary_node_mask(mesh.shape), nf, False)
    pat = mf.Pattern(torch.from_numpy(mesh.conn).to(dev), mesh.n_nodes, 3, nf)
    coords = torch.from_numpy(mesh.coords).to(dev)
    kt = torch.from_numpy(k).to(dev)
    dm = torch.from_numpy(mask).to(dev)
    form = mf.Form({O.POISSON: mf.POISSON, O.ELASTICITY: mf.ELASTICITY}[kind], **prm)
    K, _ = pat.assemble(form, coords, elem_param=kt, dirichlet=dm)
    mg = mf.Multigrid(pat, coarse_rows=1)
    mg.update(form, coords, K, dirichlet=dm, elem_param=kt)
    r = np.random.default_rng(43).standard_normal(pat.n_rows)
    z = mg.apply(torch.from_numpy(r).to(dev)).cpu().numpy()
    n_levels = len(mg.levels())
    levels = MG.build_levels(dims, mesh.coords, nf, kind, [prm] * n_levels, n_levels, dirichlet=mask, elem_param=k)
    z_ref = MG.vcycle(levels, r)
    err = np.abs(z - z_ref).max() / np.abs(z_ref).max()
    say(f"  levels {n_levels} rel err {err:.2e}")
    assert err <= TOL


def test_pcg_with_multigrid_on_lognormal_conduction(mf):
    """32^3 conduction with a lognormal Gaussian-field conductivity (sigma 1.5, correlation
    length 0.1, the learned preconditioner's workload at a smaller size): multigrid PCG in
    a fraction of the Jacobi iterations, within 1e-8 of the oracle's PCG solution."""
    n = 32
    say(f"pcg multigrid lognormal {n}^3")
    dev = torch.device("cuda:0")
    mesh = W.structured_mesh((n, n, n))
    k = W.grf_lognormal_elem((n, n, n), 1.5, 0.1, 7)
    f = W.uniform_nodal(1, mesh.n_nodes, 0, 1, 8)
    mask = W.boundary_node_mask(mesh.shape)
    pat = mf.Pattern(torch.from_numpy(mesh.conn).to(dev), mesh.n_nodes, 3, 1)
    coords = torch.from_numpy(mesh.coords).to(dev)
    kt, dm = torch.from_numpy(k).to(dev), torch.from_numpy(mask).to(dev)
    form = mf.Form(mf.POISSON, coef=1.0)
    K, d = pat.assemble(form, coords, elem_param=kt, nodal_src=torch.from_numpy(f).to(dev), dirichlet=dm)
    mg = mf.Multigrid(pat)
    mg.update(form, coords, K, dirichlet=dm, elem_param=kt)
    rp, ci, _ = pat.device_arrays()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        x, res = mf.pcg(rp, ci, K, d, tol=1e-10, precond=mf.PRECOND_MG, mg=mg, stream=s)
        _, rj = mf.pcg(rp, ci, K, d, tol=1e-10, stream=s)
    s.synchronize()
    say(f"  mg {res} jacobi {rj}")
    assert res["converged"] and res["iterations"] * 5 <= rj["iterations"]
    opat = O.Pattern(mesh, 1)
    Ko, do = O.assemble(opat, O.POISSON, {"coef": 1.0}, elem_param=k, nodal_src=f, dirichlet=mask)
    xo, _, _ = O.pcg_jacobi(opat.row_ptr, opat.col_idx, Ko, do, tol=1e-12)
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-8 * np.linalg.norm(xo)
