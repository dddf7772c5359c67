"""GPU parity of mf_pattern / mf_assemble against the oracle (through the C ABI).

Pattern: bit-exact.  K and d: row-scaled relative error <= 1e-12 (FP64) or 1e-5 (FP32).
In FP32 mode the oracle receives the same float-rounded inputs as the GPU (coordinates
stay FP64), so the comparison measures the arithmetic only.
"""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
from helpers import TOL, oracle_rows, rowscaled_error, vec_error

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def cuda(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def gpu_pattern(mf, mesh, nf, coupling=None, numbering=0):
    return mf.Pattern(cuda(mesh.conn), mesh.n_nodes, mesh.dim, nf, coupling=coupling, numbering=numbering)


# ------------------------------------------------------------------ pattern

PATTERN_CASES = [
    ("quad3x2", lambda: W.structured_mesh((3, 2)), 1, None, 0),
    ("quad7x5_fm", lambda: W.structured_mesh((7, 5)), 2, [[1, 0], [1, 1]], 1),
    ("hex1", lambda: W.structured_mesh((1, 1, 1)), 3, None, 0),
    ("hex9x7x6", lambda: W.structured_mesh((9, 7, 6)), 3, None, 0),
    ("hex9x7x6_fm", lambda: W.structured_mesh((9, 7, 6)), 4, None, 1),
    ("hex_perm", lambda: W.permute_mesh(W.structured_mesh((5, 4, 3)), 7)[0], 4,
     [[1, 1, 0, 1], [1, 1, 0, 1], [0, 0, 1, 1], [1, 1, 1, 1]], 0),
    ("hex_perm_fm", lambda: W.permute_mesh(W.structured_mesh((5, 4, 3)), 8)[0], 3, None, 1),
]


@pytest.mark.parametrize("name,make,nf,cpl,numbering", PATTERN_CASES, ids=[c[0] for c in PATTERN_CASES])
def test_pattern_bit_exact(mf, name, make, nf, cpl, numbering):
    say("pattern", name)
    mesh = make()
    cpl_arr = None if cpl is None else np.array(cpl, np.uint8)
    ref = O.Pattern(mesh, nf, cpl_arr, numbering)
    pat = gpu_pattern(mf, mesh, nf, cpl_arr, numbering)
    rp, ci, rk = pat.arrays()
    assert pat.n_rows == ref.n_rows and pat.nnz == ref.nnz
    assert np.array_equal(rp.astype(np.int64), ref.row_ptr)
    assert np.array_equal(ci, ref.col_idx)
    assert np.array_equal(rk, ref.rank)


def test_grid_detection(mf):
    say("grid detection")
    m = W.structured_mesh((6, 5, 4), jitter=0.1, seed=1)
    g, n = gpu_pattern(mf, m, 1).grid()
    assert g and n == (6, 5, 4)
    g2, n2 = gpu_pattern(mf, W.structured_mesh((6, 5)), 1).grid()
    assert g2 and n2[:2] == (6, 5)
    gp, _ = gpu_pattern(mf, W.permute_mesh(m, 3)[0], 1).grid()
    assert not gp


def test_bad_node_id_is_reported(mf):
    say("bad node id")
    m = W.structured_mesh((2, 2, 2))
    conn = m.conn.copy()
    conn[3, 2] = m.n_nodes  # out of range
    with pytest.raises(mf.MFError) as ei:
        mf.Pattern(cuda(conn), m.n_nodes, 3, 1)
    assert ei.value.status == mf.ERR_BAD_MESH


# ------------------------------------------------------------------ assembly

def make_inputs(kind, mesh, seed=0):
    dim = mesh.dim
    ep, src, state = None, None, None
    params = {}
    if kind == O.MASS:
        params = {"coef": 1.7}
        ep = W.lognormal_elem(mesh.n_elems, 0.3, seed + 1)
        src = W.uniform_nodal(1, mesh.n_nodes, 0, 1, seed + 2)
    elif kind == O.POISSON:
        params = {"coef": 1.3}
        ep = W.lognormal_elem(mesh.n_elems, 0.5, seed + 1)
        src = W.uniform_nodal(1, mesh.n_nodes, 0, 1, seed + 2)
    elif kind == O.ELASTICITY:
        params = {"coef": 1.0, "nu": 0.3}
        ep = W.lognormal_elem(mesh.n_elems, 0.5, seed + 1)
        src = W.uniform_nodal(dim, mesh.n_nodes, -1, 1, seed + 2)
    else:
        params = {"rho": 1.0, "mu": 0.01, "tau_m": 3.417e-3, "tau_c": 1.059e-2}
        state = np.zeros((dim + 1, mesh.n_nodes))
        state[:dim] = W.fourier_velocity(mesh.coords, seed + 5)
        state[dim] = W.uniform_nodal(1, mesh.n_nodes, -0.5, 0.5, seed + 3)[0]
    return params, ep, src, state


def run_gpu(mf, pat, kind, params, mesh, prec, ep, src, state, mask=None, scatter=0):
    dt = torch.float64 if prec == mf.F64 else torch.float32
    form = mf.Form(kind, **params)
    K, d = pat.assemble(form, cuda(mesh.coords), precision=prec,
                        elem_param=None if ep is None else cuda(ep, dt),
                        nodal_src=None if src is None else cuda(src, dt),
                        lin_state=None if state is None else cuda(state, dt),
                        dirichlet=None if mask is None else cuda(mask),
                        scatter=scatter)
    torch.cuda.synchronize()
    st, bad = pat.status()
    assert st == mf.OK, (st, bad)
    return K.double().cpu().numpy(), d.double().cpu().numpy()


def rounded(a, prec):
    if a is None or prec == 0:
        return a
    return np.asarray(a, np.float32).astype(np.float64)


FORMS = [("mass", O.MASS), ("poisson", O.POISSON), ("elasticity", O.ELASTICITY), ("ns", O.NS_SUPG)]
MESHES = [
    ("hex9x7x6_jit", lambda: W.structured_mesh((9, 7, 6), jitter=0.15, seed=2)),
    ("hex_perm", lambda: W.permute_mesh(W.structured_mesh((6, 5, 4), jitter=0.2, seed=3), 4)[0]),
    ("quad11x6_jit", lambda: W.structured_mesh((11, 6), jitter=0.2, seed=5)),
]


@pytest.mark.parametrize("prec", [0, 1], ids=["f64", "f32"])
@pytest.mark.parametrize("fname,kind", FORMS, ids=[f[0] for f in FORMS])
@pytest.mark.parametrize("mname,make", MESHES, ids=[m[0] for m in MESHES])
@pytest.mark.parametrize("scatter", [0, 1], ids=["auto", "atomic"])
def test_assembly_parity(mf, prec, fname, kind, mname, make, scatter):
    say("assemble", fname, mname, "f32" if prec else "f64", "scatter", scatter)
    mesh = make()
    nf = O.form_nf(kind, mesh.dim)
    params, ep, src, state = make_inputs(kind, mesh)
    ref_pat = O.Pattern(mesh, nf)
    Kr, dr = O.assemble(ref_pat, kind, params, elem_param=rounded(ep, prec), nodal_src=rounded(src, prec),
                        state=rounded(state, prec))
    pat = gpu_pattern(mf, mesh, nf)
    K, d = run_gpu(mf, pat, kind, params, mesh, prec, ep, src, state, scatter=scatter)
    ek, ed = rowscaled_error(ref_pat, K, Kr), vec_error(d, dr)
    say(f"  K err {ek:.3e}  d err {ed:.3e}")
    assert ek <= TOL[prec] and ed <= TOL[prec]


@pytest.mark.parametrize("numbering", [0, 1], ids=["node_major", "field_major"])
@pytest.mark.parametrize("prec", [0, 1], ids=["f64", "f32"])
def test_elasticity_dirichlet_and_numbering(mf, numbering, prec):
    say("elasticity dirichlet numbering", numbering, prec)
    mesh = W.structured_mesh((8, 6, 5), jitter=0.15, seed=9)
    params, ep, src, _ = make_inputs(O.ELASTICITY, mesh, seed=3)
    mask = W.dof_mask(W.boundary_node_mask(mesh.shape), 3, field_major=bool(numbering), fields=[0, 2])
    ref_pat = O.Pattern(mesh, 3, numbering=numbering)
    Kr, dr = O.assemble(ref_pat, O.ELASTICITY, params, elem_param=rounded(ep, prec),
                        nodal_src=rounded(src, prec), dirichlet=mask)
    pat = gpu_pattern(mf, mesh, 3, numbering=numbering)
    K, d = run_gpu(mf, pat, O.ELASTICITY, params, mesh, prec, ep, src, None, mask=mask)
    assert rowscaled_error(ref_pat, K, Kr) <= TOL[prec]
    assert vec_error(d, dr) <= TOL[prec]


def test_poisson_2d_32x32_dirichlet_f64(mf):
    """Thermal conduction on the unit square, 32x32 Q1, k = 1, f ~ U[0,1] (seed 1),
    u = 0 on the boundary: the whole system against the oracle."""
    say("poisson 2d 32x32")
    mesh = W.structured_mesh((32, 32))
    f = W.uniform_nodal(1, mesh.n_nodes, 0, 1, 1)
    mask = W.boundary_node_mask(mesh.shape)
    ref_pat = O.Pattern(mesh, 1)
    Kr, dr = O.assemble(ref_pat, O.POISSON, {"coef": 1.0}, nodal_src=f, dirichlet=mask)
    pat = gpu_pattern(mf, mesh, 1)
    K, d = run_gpu(mf, pat, O.POISSON, {"coef": 1.0}, mesh, 0, None, f, None, mask=mask)
    assert rowscaled_error(ref_pat, K, Kr) <= 1e-12
    assert vec_error(d, dr) <= 1e-12
    assert int(mask.sum()) == 128


def sampled_nodes(shape, n_random, seed):
    rng = np.random.default_rng(seed)
    npts = [v + 1 for v in shape]
    nn = int(np.prod(npts))
    picks = set(rng.integers(0, nn, n_random).tolist())
    for corner in range(8):  # corners and a few edge/face nodes
        ijk = [(npts[d] - 1) if (corner >> d) & 1 else 0 for d in range(3)]
        picks.add(ijk[0] + npts[0] * (ijk[1] + npts[1] * ijk[2]))
    picks.add(npts[0] // 2)                      # edge
    picks.add(npts[0] * (npts[1] // 2))          # face
    return sorted(picks)


@pytest.mark.parametrize("prec", [0, 1], ids=["f64", "f32"])
def test_elasticity_64cubed_whole_system(mf, prec):
    """Full-size 3D elasticity, 64^3 Q1, +-15% jitter, lognormal E, nu = 0.3, body force
    U[-1,1]: every one of the 64,701,513 values of K and every entry of d against the
    oracle's assembly of the whole mesh (row-scaled K error, d error scaled by |d_ref|_inf,
    1e-12 in FP64 and 1e-5 in FP32)."""
    say("elasticity 64^3 whole system", prec)
    mesh = W.structured_mesh((64, 64, 64), jitter=0.15, seed=2)
    E = W.lognormal_elem(mesh.n_elems, 0.5, 3)
    b = W.uniform_nodal(3, mesh.n_nodes, -1, 1, 4)
    params = {"coef": 1.0, "nu": 0.3}
    pat = gpu_pattern(mf, mesh, 3)
    K, d = run_gpu(mf, pat, O.ELASTICITY, params, mesh, prec, E, b, None)
    ref = O.Pattern(mesh, 3)
    rp, ci, _ = pat.arrays()
    assert np.array_equal(rp.astype(np.int64), ref.row_ptr) and np.array_equal(ci, ref.col_idx)
    del rp, ci
    Kr, dr = O.assemble(ref, O.ELASTICITY, params, elem_param=rounded(E, prec), nodal_src=rounded(b, prec))
    ek, ed = rowscaled_error(ref, K, Kr), vec_error(d, dr)
    say(f"  whole-system K err {ek:.3e} d err {ed:.3e}")
    assert ek <= TOL[prec] and ed <= TOL[prec]


def check_sampled(K, d, rp, ci, ref, nf, mask=None):
    """Worst row-scaled K error and d error of sampled rows against oracle rows; with a
    mask the oracle rows get the homogeneous Dirichlet elimination applied here."""
    worst_k = worst_d = 0.0
    for v, (cols, Krows, dref) in ref.items():
        dref = dref.copy()
        for i in range(nf):
            r = nf * v + i
            sl = slice(rp[r], rp[r + 1])
            assert np.array_equal(ci[sl], cols)
            want = Krows[i].copy()
            if mask is not None:
                if mask[r]:
                    want = (cols == r).astype(np.float64)
                    dref[i] = 0.0
                else:
                    want[mask[cols] != 0] = 0.0
            scale = np.max(np.abs(want))
            worst_k = max(worst_k, np.max(np.abs(K[sl] - want)) / scale)
        worst_d = max(worst_d, np.max(np.abs(d[nf * v:nf * v + nf] - dref)) / max(np.max(np.abs(dref)), 1e-300))
    return worst_k, worst_d


@pytest.mark.parametrize("prec", [0, 1], ids=["f64", "f32"])
def test_ns_48cubed_whole_system(mf, prec):
    """Full-size SUPG Navier-Stokes Jacobian, 48^3 Q1 on the unit cube, rho 1, mu 0.01,
    smooth random velocity, pressure U[-0.5,0.5]: all 48,778,000 values of K and all of
    d against the oracle's whole-mesh assembly, at the stated tolerances."""
    say("ns 48^3 whole system", prec)
    mesh = W.structured_mesh((48, 48, 48))
    params, _, _, state = make_inputs(O.NS_SUPG, mesh, seed=5)
    pat = gpu_pattern(mf, mesh, 4)
    K, d = run_gpu(mf, pat, O.NS_SUPG, params, mesh, prec, None, None, state)
    ref = O.Pattern(mesh, 4)
    Kr, dr = O.assemble(ref, O.NS_SUPG, params, state=rounded(state, prec))
    ek, ed = rowscaled_error(ref, K, Kr), vec_error(d, dr)
    say(f"  whole-system K err {ek:.3e} d err {ed:.3e}")
    assert ek <= TOL[prec] and ed <= TOL[prec]


def test_poisson_96cubed_sampled_rows_dirichlet(mf):
    """Full-size 3D Poisson, 96^3 Q1, lognormal Gaussian-field conductivity, f ~ U[0,1],
    u = 0 on the boundary (55,298 constrained rows), FP64: sampled rows against the
    oracle with the elimination applied."""
    say("poisson 96^3 sampled")
    n = (96, 96, 96)
    mesh = W.structured_mesh(n)
    k = W.grf_lognormal_elem(n, 1.5, 0.1, 10001)
    f = W.uniform_nodal(1, mesh.n_nodes, 0, 1, 10002)
    mask = W.boundary_node_mask(n)
    assert int(mask.sum()) == 55298
    pat = gpu_pattern(mf, mesh, 1)
    K, d = run_gpu(mf, pat, O.POISSON, {"coef": 1.0}, mesh, 0, k, f, None, mask=mask)
    rp, ci, _ = pat.arrays()
    nodes = sampled_nodes(n, 100, 17)
    ref = oracle_rows(mesh, nodes, O.POISSON, 1, {"coef": 1.0}, elem_param=k, nodal_src=f)
    wk, wd = check_sampled(K, d, rp, ci, ref, 1, mask=mask)
    say(f"  sampled K err {wk:.3e} d err {wd:.3e}")
    assert wk <= TOL[0] and wd <= TOL[0]


def test_inverted_element_sets_status(mf):
    say("inverted element")
    mesh = W.structured_mesh((3, 3, 3))
    conn = mesh.conn.copy()
    conn[[0, 1], 13] = conn[[1, 0], 13]
    bad = W.Mesh(mesh.coords, conn)
    pat = gpu_pattern(mf, bad, 1)
    form = mf.Form(mf.POISSON, coef=1.0)
    pat.assemble(form, cuda(bad.coords))
    st, e = pat.status()
    assert st == mf.ERR_BAD_JACOBIAN and e == 13
    # a good assembly on the same pattern clears the status
    pat2 = gpu_pattern(mf, mesh, 1)
    pat2.assemble(form, cuda(mesh.coords))
    assert pat2.status() == (mf.OK, -1)


NONFINITE_CASES = [
    ("gather_E", (5, 4, 3), O.ELASTICITY, "ep", 0),
    ("gather_src_f32", (5, 4, 3), O.POISSON, "src", 1),
    ("gather_ns_state_f32", (4, 3, 3), O.NS_SUPG, "state", 1),
    ("atomic_E", (5, 4, 3), O.ELASTICITY, "ep", 0),
    ("atomic_ns_state", (4, 3, 3), O.NS_SUPG, "state", 0),
    ("quad2d_src", (6, 5), O.POISSON, "src", 0),
]


@pytest.mark.parametrize("name,n,kind,what,prec", NONFINITE_CASES, ids=[c[0] for c in NONFINITE_CASES])
def test_nonfinite_input_sets_status(mf, name, n, kind, what, prec):
    """A NaN element parameter, source value or state value is reported by mf_status_poll
    as MF_ERR_NONFINITE with the smallest element that read it; the next clean assembly
    on the same pattern clears it."""
    say("non-finite input", name)
    mesh = W.structured_mesh(n, jitter=0.1, seed=4)
    nf = O.form_nf(kind, mesh.dim)
    params, ep, src, state = make_inputs(kind, mesh, seed=2)
    pat = gpu_pattern(mf, mesh, nf)
    scatter = mf.SCATTER_ATOMIC if name.startswith("atomic") else 0
    bad = {"ep": ep, "src": src, "state": state}[what].copy()
    if what == "ep":
        e = mesh.n_elems // 2
        bad[e] = np.nan
        want = e
    else:
        node = mesh.n_nodes // 2
        bad[-1 if what == "src" else 0, node] = np.nan
        want = int(np.min(np.nonzero(np.any(mesh.conn == node, axis=0))[0]))
    args = {"ep": ep, "src": src, "state": state}
    args[what] = bad
    dt = torch.float64 if prec == 0 else torch.float32
    form = mf.Form(kind, **params)
    opt = lambda a: None if a is None else cuda(a, dt)
    pat.assemble(form, cuda(mesh.coords), precision=prec, elem_param=opt(args["ep"]), nodal_src=opt(args["src"]),
                 lin_state=opt(args["state"]), scatter=scatter)
    st, first = pat.status()
    assert st == mf.ERR_NONFINITE and first == want, (st, first, want)
    pat.assemble(form, cuda(mesh.coords), precision=prec, elem_param=opt(ep), nodal_src=opt(src),
                 lin_state=opt(state), scatter=scatter)
    assert pat.status() == (mf.OK, -1)


def test_argument_errors(mf):
    say("argument errors")
    mesh = W.structured_mesh((2, 2, 2))
    pat = gpu_pattern(mf, mesh, 1)
    with pytest.raises(mf.MFError) as ei:
        pat.assemble(mf.Form(mf.ELASTICITY, coef=1.0, nu=0.3), cuda(mesh.coords))
    assert ei.value.status == mf.ERR_ARG
    with pytest.raises(mf.MFError) as ei:
        pat.assemble(mf.Form(mf.POISSON), cuda(mesh.coords), points_per_axis=3)
    assert ei.value.status == mf.ERR_UNSUPPORTED
    pat4 = gpu_pattern(mf, mesh, 4, coupling=np.tril(np.ones((4, 4))))
    with pytest.raises(mf.MFError):
        pat4.assemble(mf.Form(mf.NS_SUPG, rho=1.0), cuda(mesh.coords))


GATHER_MESHES = [(1, 1, 1), (2, 1, 1), (3, 5, 2), (7, 7, 3), (4, 4, 4), (5, 3, 11)]


@pytest.mark.parametrize("n", GATHER_MESHES, ids=["x".join(map(str, n)) for n in GATHER_MESHES])
@pytest.mark.parametrize("fname,kind", FORMS[:3], ids=[f[0] for f in FORMS[:3]])
@pytest.mark.parametrize("prec", [0, 1], ids=["f64", "f32"])
def test_gather_on_small_and_ragged_grids(mf, n, fname, kind, prec):
    """The owner-computes path on grids whose node counts are and are not multiples of
    the 4x2 node column, with Dirichlet rows on one face; against the oracle."""
    say("gather", n, fname, prec)
    mesh = W.structured_mesh(n, jitter=0.1, seed=sum(n))
    nf = O.form_nf(kind, 3)
    params, ep, src, state = make_inputs(kind, mesh, seed=7)
    nm = W.boundary_node_mask(mesh.shape) * (mesh.coords[0] == 0.0)
    mask = W.dof_mask(nm.astype(np.uint8), nf, field_major=False)
    ref_pat = O.Pattern(mesh, nf)
    Kr, dr = O.assemble(ref_pat, kind, params, elem_param=rounded(ep, prec), nodal_src=rounded(src, prec),
                        dirichlet=mask)
    pat = gpu_pattern(mf, mesh, nf)
    assert pat.grid()[0]
    K, d = run_gpu(mf, pat, kind, params, mesh, prec, ep, src, state, mask=mask, scatter=mf.SCATTER_GATHER)
    assert rowscaled_error(ref_pat, K, Kr) <= TOL[prec]
    assert vec_error(d, dr) <= TOL[prec]


@pytest.mark.parametrize("numbering", [0, 1], ids=["node_major", "field_major"])
@pytest.mark.parametrize("fname,kind", [FORMS[1], FORMS[2]], ids=["poisson", "elasticity"])
def test_gather_scattered_dirichlet(mf, fname, kind, numbering):
    """Dirichlet flags on random DOFs inside the grid (not only on faces), so every
    neighbour offset of the write-out's flag lookup meets constrained columns; the grid is
    tall enough that columns are split into several layer ranges."""
    say("gather scattered dirichlet", fname, numbering)
    mesh = W.structured_mesh((9, 6, 40), jitter=0.1, seed=11)
    nf = O.form_nf(kind, 3)
    params, ep, src, state = make_inputs(kind, mesh, seed=13)
    mask = (np.random.default_rng(14).random(nf * mesh.n_nodes) < 0.2).astype(np.uint8)
    ref_pat = O.Pattern(mesh, nf, numbering=numbering)
    Kr, dr = O.assemble(ref_pat, kind, params, elem_param=ep, nodal_src=src, dirichlet=mask)
    pat = gpu_pattern(mf, mesh, nf, numbering=numbering)
    assert pat.grid()[0]
    K, d = run_gpu(mf, pat, kind, params, mesh, 0, ep, src, state, mask=mask, scatter=mf.SCATTER_GATHER)
    assert rowscaled_error(ref_pat, K, Kr) <= TOL[0]
    assert vec_error(d, dr) <= TOL[0]


@pytest.mark.parametrize("mname,make,kinds", [(MESHES[0][0], MESHES[0][1], (O.NS_SUPG,)),
                                              (MESHES[1][0], MESHES[1][1], (O.ELASTICITY, O.NS_SUPG))],
                         ids=["grid_flow", "permuted"])
def test_coloured_scatter_is_deterministic(mf, mname, make, kinds):
    """Where the default path scatters element by element (meshes that are not grids, and
    the FP64 flow form, which has no gather kernel) it goes colour by colour with plain
    adds, so two assemblies are bitwise equal."""
    say("deterministic coloured scatter", mname)
    mesh = make()
    for kind in kinds:
        nf = O.form_nf(kind, mesh.dim)
        params, ep, src, state = make_inputs(kind, mesh)
        pat = gpu_pattern(mf, mesh, nf)
        K1, d1 = run_gpu(mf, pat, kind, params, mesh, 0, ep, src, state)
        K2, d2 = run_gpu(mf, pat, kind, params, mesh, 0, ep, src, state)
        assert np.array_equal(K1, K2) and np.array_equal(d1, d2)
