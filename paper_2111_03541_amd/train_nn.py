"""Train the learned PCG preconditioner on systems assembled by the library.

    python -m paper_2111_03541_amd.train_nn --n 96 --systems 2000 --out weights/poisson96

Training data: 3D Poisson on an n^3 Q1 hex mesh of the unit cube with u = 0 on the
boundary and a lognormal conductivity k = exp(sigma g), sigma ~ U[1,2], g a unit-variance
Gaussian field with correlation length 0.1.  Each system's g is a random unit-norm
combination of two fields from a pool of independent draws (again such a field), so
thousands of systems come from a small pool.  K is assembled on the GPU by mf_assemble;
each step draws a multiscale error e, forms r = K e with mf_spmv, and takes one Adam step
on the energy-norm loss (z - e)^T K (z - e) / e^T K e with the library's training kernels.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

DEFAULT_CHANNELS = [1, 4, 8, 8, 8]


def levels_for(n_nodes, want):
    lv, m = 1, n_nodes
    while lv < want and m % 2 == 1 and m >= 5:
        m = (m + 1) // 2
        lv += 1
    return lv


class PoissonFamily:
    """Structured-mesh Poisson systems sharing one pattern; assembled on demand."""

    def __init__(self, n, dev, pool=64, seed=0):
        import torch
        import paper_2111_03541_amd as mf
        import workloads as W
        self.n = n
        self.dev = dev
        self.mesh = W.structured_mesh((n, n, n))
        self.pat = mf.Pattern(torch.from_numpy(self.mesh.conn).to(dev), self.mesh.n_nodes, 3, 1)
        self.coords = torch.from_numpy(self.mesh.coords).to(dev)
        self.mask_np = W.boundary_node_mask(self.mesh.shape)
        self.mask = torch.from_numpy(self.mask_np).to(dev)
        self.form = mf.Form(mf.POISSON, coef=1.0)
        self.pool = [W.grf_elem((n, n, n), 0.1, seed * 100_003 + 7 * i) for i in range(pool)]
        self.rp, self.ci, _ = self.pat.device_arrays()
        self.K = torch.empty(self.pat.nnz, dtype=torch.float64, device=dev)
        self.d = torch.empty(self.pat.n_rows, dtype=torch.float64, device=dev)

    def system(self, sys_seed):
        """Assemble system number sys_seed into self.K / self.d; returns sigma."""
        import torch
        import paper_2111_03541_amd as mf
        import workloads as W
        rng = np.random.default_rng(sys_seed)
        sigma = float(rng.uniform(1.0, 2.0))
        i, j = rng.choice(len(self.pool), 2, replace=False)
        th = rng.uniform(0.0, 2.0 * np.pi)
        g = np.cos(th) * self.pool[i] + np.sin(th) * self.pool[j]
        k = torch.from_numpy(np.exp(sigma * g)).to(self.dev)
        f = torch.from_numpy(W.uniform_nodal(1, self.mesh.n_nodes, 0, 1, sys_seed + 1)).to(self.dev)
        self.pat.assemble(self.form, self.coords, precision=mf.F64, elem_param=k, nodal_src=f,
                          dirichlet=self.mask, K=self.K, d=self.d)
        return sigma


def checkpoint_step(path):
    """Training step recorded in a checkpoint file (header word 2, see mf_nn_save)."""
    return int(np.fromfile(path, dtype=np.int64, count=3)[2])


def train(n=96, n_systems=2000, channels=None, lr=2e-3, pool=64, seed=0, log_every=100, dev=None,
          net=None, epochs=1, checkpoint=None, checkpoint_every=0, resume=None):
    """Train on n_systems systems per epoch.  The system and the error of global step k
    are functions of k alone, so a run resumed from a checkpoint (parameters, Adam state
    and step, mf_nn_save) continues exactly where the interrupted one stopped."""
    import torch
    import paper_2111_03541_amd as mf
    import workloads as W
    dev = dev or torch.device("cuda:0")
    nn_nodes = n + 1
    channels = list(channels or DEFAULT_CHANNELS)
    channels = channels[:levels_for(nn_nodes, len(channels))]
    fam = PoissonFamily(n, dev, pool=pool, seed=seed)
    if net is None:
        net = mf.Net((nn_nodes,) * 3, channels, seed=seed + 1)
    start = 0
    if resume:
        net.load_checkpoint(resume)
        start = checkpoint_step(resume)
    mask = fam.mask_np != 0
    hist = []
    t0 = time.perf_counter()
    step = 0
    for ep in range(epochs):
        for s in range(n_systems):
            if step < start:
                step += 1
                continue
            fam.system(s)
            net.set_system(fam.rp, fam.ci, fam.K, fam.mask)
            e_np = W.multiscale_nodal(nn_nodes, len(channels), 1_000_000 + ep * n_systems + s)
            e_np[mask] = 0.0
            e = torch.from_numpy(e_np).to(dev)
            r = mf.spmv(fam.rp, fam.ci, fam.K, e)
            cur_lr = lr * 0.5 * (1.0 + np.cos(np.pi * step / (epochs * n_systems)))
            loss = net.train_step(r, cur_lr, e=e)
            hist.append(loss)
            step += 1
            if checkpoint and checkpoint_every and step % checkpoint_every == 0:
                net.save_checkpoint(checkpoint)
            if log_every and step % log_every == 0:
                print(f"[train] step {step} loss {np.mean(hist[-log_every:]):.4f} "
                      f"({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    return net, hist, fam


def compare(net, fam, seeds, tol=1e-8, check_every=8):
    """Iterations and wall time to tol: learned (flexible) PCG vs Jacobi PCG."""
    import torch
    import paper_2111_03541_amd as mf
    stream = torch.cuda.Stream(fam.dev)
    out = []
    x = torch.empty_like(fam.d)
    for s in seeds:
        fam.system(s)
        net.set_system(fam.rp, fam.ci, fam.K, fam.mask)
        row = {"seed": s}
        for name, pc in (("jacobi", mf.PRECOND_JACOBI), ("learned", mf.PRECOND_NN)):
            times = []
            for rep in range(2):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, res = mf.pcg(fam.rp, fam.ci, fam.K, fam.d, x=x, tol=tol, maxit=20000, precond=pc,
                                net=net if pc == mf.PRECOND_NN else None, check_every=check_every,
                                use_graph=True, stream=stream)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
            row[name] = {"iterations": res["iterations"], "ms": 1e3 * min(times),
                         "true_relres": res["true_relres"], "fallbacks": res["fallbacks"]}
        out.append(row)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=96)
    ap.add_argument("--systems", type=int, default=2000)
    ap.add_argument("--epochs", type=int, default=1)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--pool", type=int, default=64)
    ap.add_argument("--channels", type=str, default=",".join(map(str, DEFAULT_CHANNELS)))
    ap.add_argument("--out", type=str, default=None)
    ap.add_argument("--eval", type=int, default=3)
    ap.add_argument("--checkpoint", type=str, default=None, help="training-state file written every --every steps")
    ap.add_argument("--every", type=int, default=500)
    ap.add_argument("--resume", type=str, default=None, help="continue from this training-state file")
    args = ap.parse_args()
    net, hist, fam = train(args.n, args.systems, [int(v) for v in args.channels.split(",")], args.lr,
                           args.pool, epochs=args.epochs, checkpoint=args.checkpoint, checkpoint_every=args.every,
                           resume=args.resume)
    res = compare(net, fam, [10_000 + i for i in range(args.eval)])
    print(json.dumps({"final_loss": float(np.mean(hist[-100:])) if hist else None, "eval": res}), flush=True)
    if args.out:
        os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
        net.save(args.out, trained_with={"command": " ".join(["python -m paper_2111_03541_amd.train_nn"] + sys.argv[1:]),
                                         "n": args.n, "systems": args.systems, "epochs": args.epochs, "lr": args.lr,
                                         "pool": args.pool, "loss": "energy norm", "seed": 0})


if __name__ == "__main__":
    main()
