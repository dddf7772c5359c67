"""Oracle for the learned preconditioner: a plain numpy FP64 implementation of the network,
its loss and its parameter gradient.

TEST INFRASTRUCTURE ONLY.  Only `tests/` and the benchmark's CPU baseline leg may import
this module; the HIP library never does, and the two share no code.

The paper leaves the linear solver open (Sec. 2.2 D-4).  The preconditioner is a small
linear multilevel 3D convolution network on the node grid of a structured mesh:

    z = Dm^-1/2 * N(v),      v = Dm^-1/2 r
    N(v) = y_0 + P(y_1 + P(y_2 + ... P(y_{L-1})))
    y_0 = conv_0(v)                                  (1 -> 1 channel)
    y_l = conv_{l,3}(conv_{l,2}(conv_{l,1}(R^l v)))  (1 -> c_l -> c_l -> 1), l >= 1

where Dm = diag(K), R is full weighting from a (2n-1)-node grid to an n-node grid,
P = R^T is trilinear prolongation, and every conv is 3x3x3 with zero padding and no
bias.  z is set to 0 on constrained (Dirichlet) rows.  N is linear in v, so the
preconditioner is a fixed linear operator for each system.

Training losses for one residual r:  L = |K z - r|_2^2 / |r|_2^2, or, given the error e
with r = K e, the energy-norm error L = (z - e)^T K (z - e) / e^T K e.
"""
from __future__ import annotations

import numpy as np

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def level_shapes(shape, levels):
    """Node-grid shapes per level: (nz, ny, nx) -> ((nz+1)/2, ...)."""
    out = [tuple(shape)]
    for _ in range(levels - 1):
        s = out[-1]
        if any(v % 2 == 0 or v < 3 for v in s):
            raise ValueError(f"level grid {s} cannot be coarsened (odd sizes >= 3 needed)")
        out.append(tuple((v + 1) // 2 for v in s))
    return out


def param_layout(channels):
    """List of conv weight shapes (cout, cin, 27) in parameter order."""
    shapes = [(1, 1, 27)]
    for c in channels[1:]:
        shapes += [(c, 1, 27), (c, c, 27), (1, c, 27)]
    return shapes


def n_params(channels):
    return sum(a * b * t for a, b, t in param_layout(channels))


def unpack(theta, channels):
    ws, o = [], 0
    for a, b, t in param_layout(channels):
        ws.append(theta[o:o + a * b * t].reshape(a, b, t))
        o += a * b * t
    return ws


def shift(x, d):
    """y[p] = x[p + d] with zeros outside (x: [..., nz, ny, nx])."""
    y = np.zeros_like(x)
    src = [slice(None)] * x.ndim
    dst = [slice(None)] * x.ndim
    for ax, dd in zip(range(x.ndim - 3, x.ndim), d):
        n = x.shape[ax]
        if dd >= 0:
            src[ax], dst[ax] = slice(dd, n), slice(0, n - dd)
        else:
            src[ax], dst[ax] = slice(0, n + dd), slice(-dd, n)
    y[tuple(dst)] = x[tuple(src)]
    return y


def conv(x, w):
    """x [cin, nz, ny, nx], w [cout, cin, 27] -> [cout, nz, ny, nx]."""
    out = np.zeros((w.shape[0],) + x.shape[1:])
    for t, d in enumerate(TAPS):
        xs = shift(x, d)
        out += np.einsum("oi,izyx->ozyx", w[:, :, t], xs)
    return out


def conv_wgrad(x, gy):
    """dL/dw for y = conv(x, w) given dL/dy."""
    g = np.zeros((gy.shape[0], x.shape[0], 27))
    for t, d in enumerate(TAPS):
        g[:, :, t] = np.einsum("ozyx,izyx->oi", gy, shift(x, d))
    return g


def conv_dgrad(gy, w):
    """dL/dx for y = conv(x, w) given dL/dy."""
    out = np.zeros((w.shape[1],) + gy.shape[1:])
    for t, d in enumerate(TAPS):
        out += np.einsum("oi,ozyx->izyx", w[:, :, t], shift(gy, tuple(-v for v in d)))
    return out


def prolong(c, fine_shape):
    """Trilinear interpolation from an n-node grid to a (2n-1)-node grid."""
    f = c
    for ax in (-3, -2, -1):
        n = f.shape[ax]
        shp = list(f.shape)
        shp[ax] = 2 * n - 1
        g = np.zeros(shp)
        ev = [slice(None)] * f.ndim
        ev[ax] = slice(0, None, 2)
        g[tuple(ev)] = f
        od = [slice(None)] * f.ndim
        od[ax] = slice(1, None, 2)
        lo = [slice(None)] * f.ndim
        lo[ax] = slice(0, n - 1)
        hi = [slice(None)] * f.ndim
        hi[ax] = slice(1, n)
        g[tuple(od)] = 0.5 * (f[tuple(lo)] + f[tuple(hi)])
        f = g
    assert f.shape[-3:] == tuple(fine_shape)
    return f


def restrict(f):
    """Full weighting R = P^T from a (2n-1)-node grid to an n-node grid."""
    c = f
    for ax in (-3, -2, -1):
        n = (c.shape[ax] + 1) // 2
        shp = list(c.shape)
        shp[ax] = n
        g = np.zeros(shp)
        ev = [slice(None)] * c.ndim
        ev[ax] = slice(0, None, 2)
        g += c[tuple(ev)]
        od = [slice(None)] * c.ndim
        od[ax] = slice(1, None, 2)
        lo = [slice(None)] * c.ndim
        lo[ax] = slice(0, n - 1)
        hi = [slice(None)] * c.ndim
        hi[ax] = slice(1, n)
        g[tuple(lo)] += 0.5 * c[tuple(od)]
        g[tuple(hi)] += 0.5 * c[tuple(od)]
        c = g
    return c


class Net:
    def __init__(self, shape, channels):
        self.shape = tuple(shape)            # (nz, ny, nx) nodes
        self.channels = list(channels)
        self.levels = len(channels)
        self.shapes = level_shapes(self.shape, self.levels)

    def forward(self, theta, r, diag, mask=None, keep=False):
        """z for residual r [n_nodes] (node id = x + nx(y + ny z))."""
        ws = unpack(theta, self.channels)
        dm = 1.0 / np.sqrt(diag)
        v0 = (dm * r).reshape(self.shape)[None]
        s = 1.0
        vs, ys, acts = [v0], [], []
        for l in range(1, self.levels):
            vs.append(restrict(vs[-1]))
        ys.append(conv(v0, ws[0]))
        acts.append([v0])
        for l in range(1, self.levels):
            w1, w2, w3 = ws[1 + 3 * (l - 1): 4 + 3 * (l - 1)]
            h1 = conv(vs[l], w1)
            h2 = conv(h1, w2)
            ys.append(conv(h2, w3))
            acts.append([vs[l], h1, h2])
        acc = ys[-1]
        for l in range(self.levels - 2, -1, -1):
            acc = ys[l] + prolong(acc, self.shapes[l])
        z = s * dm * acc[0].reshape(-1)
        if mask is not None:
            z = np.where(mask != 0, 0.0, z)
        if keep:
            return z, (s, dm, acts)
        return z

    def loss_and_grad(self, theta, r, diag, Kmat, mask=None):
        """L = |K z - r|^2 / |r|^2 and dL/dtheta (adjoint through the linear network)."""
        ws = unpack(theta, self.channels)
        z, (s, dm, acts) = self.forward(theta, r, diag, mask, keep=True)
        res = Kmat @ z - r
        rn2 = float(r @ r)
        L = float(res @ res) / rn2
        gz = 2.0 * (Kmat.T @ res) / rn2
        if mask is not None:
            gz = np.where(mask != 0, 0.0, gz)
        gacc = (s * dm * gz).reshape(self.shape)[None]
        grads = [None] * len(ws)
        gy = [gacc]
        for l in range(1, self.levels):
            gy.append(restrict(gy[-1]))
        grads[0] = conv_wgrad(acts[0][0], gy[0])
        for l in range(1, self.levels):
            w1, w2, w3 = ws[1 + 3 * (l - 1): 4 + 3 * (l - 1)]
            v, h1, h2 = acts[l]
            b = 1 + 3 * (l - 1)
            grads[b + 2] = conv_wgrad(h2, gy[l])
            g2 = conv_dgrad(gy[l], w3)
            grads[b + 1] = conv_wgrad(h1, g2)
            g1 = conv_dgrad(g2, w2)
            grads[b] = conv_wgrad(v, g1)
        return L, np.concatenate([g.reshape(-1) for g in grads])


def energy_loss_and_grad(net, theta, e, diag, Kmat, mask=None):
    """L = (z - e)^T K (z - e) / (e^T K e) for r = K e, and dL/dtheta."""
    r = Kmat @ e
    ws = unpack(theta, net.channels)
    z, (s, dm, acts) = net.forward(theta, r, diag, mask, keep=True)
    den = float(e @ r)
    L = float((z - e) @ (Kmat @ (z - e))) / den
    gz = 2.0 * (Kmat @ (z - e)) / den
    if mask is not None:
        gz = np.where(mask != 0, 0.0, gz)
    gy = [(s * dm * gz).reshape(net.shape)[None]]
    for l in range(1, net.levels):
        gy.append(restrict(gy[-1]))
    grads = [conv_wgrad(acts[0][0], gy[0])]
    for l in range(1, net.levels):
        w1, w2, w3 = ws[1 + 3 * (l - 1): 4 + 3 * (l - 1)]
        v, h1, h2 = acts[l]
        g3 = conv_wgrad(h2, gy[l])
        g2 = conv_dgrad(gy[l], w3)
        gw2 = conv_wgrad(h1, g2)
        g1 = conv_dgrad(g2, w2)
        grads += [conv_wgrad(v, g1), gw2, g3]
    return L, r, np.concatenate([g.reshape(-1) for g in grads])


def init_params(channels, seed):
    """Small random weights; the level-0 stencil starts as the identity (Jacobi)."""
    rng = np.random.default_rng(seed)
    parts = []
    for a, b, t in param_layout(channels):
        w = rng.normal(0.0, 0.1 / np.sqrt(b * t), size=(a, b, t))
        parts.append(w)
    parts[0][:] = 0.0
    parts[0][0, 0, 13] = 1.0
    return np.concatenate([p.reshape(-1) for p in parts])
