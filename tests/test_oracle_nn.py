"""Oracle pins for the learned-preconditioner network (numpy FP64 reference).

R and P are checked against their definitions (P interpolates linear fields exactly,
R = P^T), the convolution and its adjoints against a brute-force loop and the inner-
product identity, and the parameter gradient against central differences.
"""
import numpy as np
import pytest

import oracle as O
import oracle.nn_ref as N
import workloads as W


def test_prolong_is_exact_on_trilinear_fields_and_restrict_is_its_transpose():
    rng = np.random.default_rng(0)
    nc = (3, 4, 5)
    nf = tuple(2 * v - 1 for v in nc)
    zc, yc, xc = np.meshgrid(*[np.arange(v) * 2.0 for v in nc], indexing="ij")
    zf, yf, xf = np.meshgrid(*[np.arange(v) * 1.0 for v in nf], indexing="ij")
    lin = lambda z, y, x: 0.3 + 1.2 * x - 0.7 * y + 0.4 * z + 0.05 * x * y * z  # trilinear
    f = N.prolong(lin(zc, yc, xc), nf)
    assert np.max(np.abs(f - lin(zf, yf, xf))) < 1e-12
    a = rng.standard_normal(nc)
    b = rng.standard_normal(nf)
    assert abs(np.sum(N.prolong(a, nf) * b) - np.sum(a * N.restrict(b))) < 1e-12


def test_conv_against_loop_and_adjoints():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 4, 3, 5))
    w = rng.standard_normal((3, 2, 27))
    y = N.conv(x, w)
    # brute force at a few points
    for (o, z, yy, xx) in [(0, 0, 0, 0), (2, 3, 2, 4), (1, 2, 1, 2)]:
        s = 0.0
        for i in range(2):
            for t, (dz, dy, dx) in enumerate(N.TAPS):
                zz, y2, x2 = z + dz, yy + dy, xx + dx
                if 0 <= zz < 4 and 0 <= y2 < 3 and 0 <= x2 < 5:
                    s += w[o, i, t] * x[i, zz, y2, x2]
        assert abs(y[o, z, yy, xx] - s) < 1e-12
    gy = rng.standard_normal(y.shape)
    # <conv(x,w), gy> = <x, dgrad(gy,w)> = <w, wgrad(x,gy)>
    lhs = np.sum(y * gy)
    assert abs(lhs - np.sum(x * N.conv_dgrad(gy, w))) < 1e-10
    assert abs(lhs - np.sum(w * N.conv_wgrad(x, gy))) < 1e-10


def small_system(n=8, seed=3):
    mesh = W.structured_mesh((n, n, n))
    k = W.grf_lognormal_elem((n, n, n), 1.5, 0.1, seed)
    f = W.uniform_nodal(1, mesh.n_nodes, 0, 1, seed + 1)
    mask = W.boundary_node_mask(mesh.shape)
    pat = O.Pattern(mesh, 1)
    K, d = O.assemble(pat, O.POISSON, {"coef": 1.0}, elem_param=k, nodal_src=f, dirichlet=mask)
    S = pat.to_scipy(K)
    return S, d, S.diagonal().copy(), mask


def test_gradient_matches_central_differences():
    S, d, diag, mask = small_system(8)
    net = N.Net((9, 9, 9), [1, 2, 3])
    theta = N.init_params(net.channels, 5)
    rng = np.random.default_rng(2)
    r = np.where(mask != 0, 0.0, rng.standard_normal(d.shape))
    L, g = net.loss_and_grad(theta, r, diag, S, mask)
    eps = 1e-6
    idx = rng.choice(theta.size, 40, replace=False)
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        fd = (net.loss_and_grad(tp, r, diag, S, mask)[0] - net.loss_and_grad(tm, r, diag, S, mask)[0]) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_network_is_linear_and_identity_start_is_jacobi():
    S, d, diag, mask = small_system(8)
    net = N.Net((9, 9, 9), [1, 2])
    theta = N.init_params(net.channels, 1)
    rng = np.random.default_rng(4)
    a = np.where(mask != 0, 0.0, rng.standard_normal(d.shape))
    b = np.where(mask != 0, 0.0, rng.standard_normal(d.shape))
    za, zb, zab = net.forward(theta, a, diag, mask), net.forward(theta, b, diag, mask), \
        net.forward(theta, 2.0 * a - 3.0 * b, diag, mask)
    assert np.max(np.abs(zab - (2.0 * za - 3.0 * zb))) < 1e-12
    # level-0 identity stencil with the coarse levels zeroed is exactly Jacobi
    th = theta.copy()
    th[27:] = 0.0
    zj = net.forward(th, a, diag, mask)
    assert np.max(np.abs(zj - np.where(mask != 0, 0.0, a / diag))) < 1e-14


def test_energy_gradient_matches_central_differences():
    S, d, diag, mask = small_system(8, seed=6)
    net = N.Net((9, 9, 9), [1, 2, 2])
    theta = N.init_params(net.channels, 9)
    rng = np.random.default_rng(3)
    e = np.where(mask != 0, 0.0, rng.standard_normal(d.shape))
    L, r, g = N.energy_loss_and_grad(net, theta, e, diag, S, mask)
    # at the Jacobi start with coarse levels off the loss is that of z = D^-1 r
    th = theta.copy()
    th[27:] = 0.0
    zj = np.where(mask != 0, 0.0, r / diag)
    Lj = (zj - e) @ (S @ (zj - e)) / (e @ r)
    assert abs(N.energy_loss_and_grad(net, th, e, diag, S, mask)[0] - Lj) < 1e-12
    eps = 1e-6
    for i in rng.choice(theta.size, 30, replace=False):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        fd = (N.energy_loss_and_grad(net, tp, e, diag, S, mask)[0] -
              N.energy_loss_and_grad(net, tm, e, diag, S, mask)[0]) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i]))
