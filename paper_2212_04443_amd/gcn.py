"""Learned warm start for the solver (not part of the paper).

A three-layer graph-convolution network (widths 17 -> 64 -> 64 -> 32, FP32)
maps 16 Gaussian channels plus sqrt(deg / mean deg) to an n x 32 block.  After
Rayleigh-Ritz the block, sorted by Rayleigh quotient, is passed to the solver
as V_init, which Alg. 2 filters progressively (steps 2 and 17).  The random
start stays the fallback: the solver's answer is accepted only by its residual
certificate.

Training runs on the GPU through the library's own kernels
(chebdav_gcn_forward / chebdav_gcn_backward / chebdav_subspace_loss /
chebdav_adam_step): the targets are the k = 32 eigenvectors the FP64 solver
computes for seeded SBM graphs with N in [10k, 50k], 8..32 blocks, intra-block
degree 10..30 and inter-block degree 2..6; the loss is the rotation-invariant
subspace loss.  An optional 64-wide head (17 -> 64 -> 64 -> 64, k = 64
targets; gcn_weights_k64.npz) serves the k = 64 workloads.

    python -m paper_2212_04443_amd.gcn train --graphs 512 --epochs 20 --lr 5e-3 --fixed-features --schedule step
    python -m paper_2212_04443_amd.gcn evaluate --workload sbm1m --seeds 6     (random / untrained / trained)
"""

from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np
import torch

from . import chebdav as cd

DIMS = (17, 64, 64, 32)
N_GAUSS = 16
WEIGHTS_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "gcn_weights.npz")
# optional 64-wide head for the k = 64 workloads (same inputs and hidden widths)
DIMS_K64 = (17, 64, 64, 64)
WEIGHTS_FILE_K64 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "gcn_weights_k64.npz")


def _sizes(dims=DIMS):
    return [dims[l] * dims[l + 1] for l in range(3)]


class Net:
    """Weights of the three layers in one flat device buffer (views per layer)."""

    def __init__(self, flat: torch.Tensor, dims=DIMS):
        self.dims = tuple(dims)
        self.flat = flat
        off = 0
        self.W = []
        for l, sz in enumerate(_sizes(dims)):
            self.W.append(flat[off:off + sz].view(dims[l], dims[l + 1]))
            off += sz

    @classmethod
    def glorot(cls, seed: int, dims=DIMS, device="cuda"):
        rng = np.random.Generator(np.random.PCG64(seed))
        parts = []
        for l in range(3):
            a = np.sqrt(6.0 / (dims[l] + dims[l + 1]))
            parts.append(rng.uniform(-a, a, size=dims[l] * dims[l + 1]))
        flat = torch.from_numpy(np.concatenate(parts).astype(np.float32)).to(device)
        return cls(flat, dims)

    def save(self, path: str, **meta):
        np.savez(path, flat=self.flat.cpu().numpy(), dims=np.array(self.dims), **meta)

    @classmethod
    def load(cls, path: str = WEIGHTS_FILE, device="cuda"):
        z = np.load(path, allow_pickle=False)
        return cls(torch.from_numpy(z["flat"]).to(device), tuple(int(x) for x in z["dims"]))


def training_graph(index: int, base_seed: int = 424242):
    """Parameters and edges of training graph `index` (seeded)."""
    import synth
    rng = np.random.Generator(np.random.PCG64(base_seed + index))
    n = int(rng.integers(10_000, 50_001))
    blocks = int(rng.integers(8, 33))
    d_in = float(rng.uniform(10, 30))
    d_out = float(rng.uniform(2, 6))
    edges, _ = synth.sbm(n, blocks, d_in=d_in, d_out=d_out, uneven=True, seed=base_seed + 100_000 + index)
    return edges, n, dict(n=n, blocks=blocks, d_in=d_in, d_out=d_out)


def build_dataset(n_graphs: int, base_seed: int = 424242, k: int = 32, kb: int = 32, m: int = 15, log=None):
    data = []
    for i in range(n_graphs):
        edges, n, meta = training_graph(i, base_seed)
        g = cd.build_laplacian(edges, n)
        r = cd.solve(g, cd.make_params(k_want=k, kb=kb, m=m, tol=1e-8, seed=base_seed + i))
        X0 = cd.gcn_features(g, seed=base_seed + 7 * i + 1, n_gauss=N_GAUSS)
        data.append(dict(g=g, X0=X0, U=r.evecs, meta=meta, iterations=r.stats["iterations"]))
        if log and (i + 1) % 64 == 0:
            log("  dataset %d/%d" % (i + 1, n_graphs))
    return data


def train(data, epochs: int = 20, lr: float = 3e-3, seed: int = 5, log=None, net: Net | None = None,
          fresh_features: bool = True, schedule: str = "cosine", targets: str = "all"):
    """Adam, one graph per step, graphs in a seeded random order each epoch.
    The input channels are random by design, so with fresh_features every epoch
    draws new ones for every graph (seed = the epoch and graph index), instead of
    reusing one draw per graph, which the network could fit.  The learning rate
    follows a cosine decay to lr/20 over the epochs ("cosine") or halves every
    third of them ("step")."""
    net = net or Net.glorot(seed)
    dims = net.dims
    m = torch.zeros_like(net.flat)
    v = torch.zeros_like(net.flat)
    grad = torch.zeros_like(net.flat)
    sizes = _sizes(dims)
    dW = []
    off = 0
    for l, sz in enumerate(sizes):
        dW.append(grad[off:off + sz].view(dims[l], dims[l + 1]))
        off += sz
    rng = np.random.Generator(np.random.PCG64(seed))
    history = []
    step = 0
    ws_cache = {}
    for ep in range(epochs):
        order = rng.permutation(len(data))
        losses = []
        if schedule == "cosine":
            lr_ep = lr * (0.05 + 0.95 * 0.5 * (1.0 + np.cos(np.pi * ep / max(1, epochs))))
        else:
            lr_ep = lr * (0.5 ** (ep // max(1, epochs // 3)))
        for i in order:
            d = data[i]
            g = d["g"]
            ws = ws_cache.get(g.n)
            if ws is None:
                ws = ws_cache[g.n] = cd.gcn_workspace(g, dims)
            X0 = d["X0"]
            if fresh_features:
                X0 = cd.gcn_features(g, seed=(seed << 32) + ep * 1_000_003 + int(i), n_gauss=N_GAUSS)
            out, acts = cd.gcn_forward(g, dims, X0, net.W, workspace=ws)
            kt = min(dims[3], d["U"].shape[1])
            if targets == "cluster":  # the eigenvectors of the planted clusters only
                kt = min(kt, int(d["meta"]["blocks"]))
            U = d["U"] if kt == d["U"].shape[1] else d["U"][:, :kt].contiguous()
            loss, dX = cd.subspace_loss(out, U, grad=True)
            cd.gcn_backward(g, dims, X0, net.W, acts, dX, dW=dW, workspace=ws)
            step += 1
            cd.adam_step(net.flat, grad, m, v, lr_ep, step=step)
            losses.append(loss)
        history.append(float(np.mean(losses)))
        if log:
            log("  epoch %d: mean loss %.4f (lr %.2e)" % (ep, history[-1], lr_ep))
    return net, history


def warm_start(g, net: Net, seed: int = 0):
    """V_init for chebdav_solve: Ritz vectors of the network's output block,
    ascending by Rayleigh quotient.  Returns (V_init, ritz)."""
    X0 = cd.gcn_features(g, seed=seed, n_gauss=N_GAUSS)
    out, _ = cd.gcn_forward(g, net.dims, X0, net.W)
    return cd.rayleigh_ritz(g, out, seed=seed)


def evaluate(g, starts: dict, k: int, kb: int, m: int, seeds, filter_dtype=cd.F64):
    """Solves from each start with the same solver settings, for each seed (the
    seed drives the random vectors and the networks' input channels).  starts:
    name -> Net, or None for the random start.  Returns a list of dicts, one per
    seed and start: iterations, sparse products, seconds (a network start's time
    includes feature generation, inference and Rayleigh-Ritz), the eigenvalues'
    largest difference from the random start's and the residual certificate."""
    rows = []
    for sd in seeds:
        p = cd.make_params(k_want=k, kb=kb, m=m, tol=1e-8, seed=sd, filter_dtype=filter_dtype)
        ref = None
        for name, net in starts.items():
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if net is None:
                r = cd.solve(g, p)
            else:
                V0, _ = warm_start(g, net, seed=sd)
                r = cd.solve(g, p, V_init=V0.contiguous())
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            if ref is None:
                ref = r.evals
            rows.append(dict(seed=sd, start=name, iterations=r.stats["iterations"],
                             spmm=r.stats["n_spmm_filter"] + r.stats["n_spmm_other"], seconds=t,
                             max_dlambda=float((r.evals - ref).abs().max().item()),
                             max_residual=r.stats["max_residual"]))
    return rows


def summarize(rows):
    """Mean iterations and sparse products, median seconds, per start."""
    out = {}
    for name in dict.fromkeys(r["start"] for r in rows):
        rs = [r for r in rows if r["start"] == name]
        out[name] = dict(iterations=float(np.mean([r["iterations"] for r in rs])),
                         spmm=float(np.mean([r["spmm"] for r in rs])),
                         ms=1e3 * float(np.median([r["seconds"] for r in rs])),
                         max_dlambda=max(r["max_dlambda"] for r in rs),
                         max_residual=max(r["max_residual"] for r in rs))
    return out


def subspace_losses(data, net: Net):
    """The subspace loss of the network's output against each graph's targets."""
    out = []
    for d in data:
        o, _ = cd.gcn_forward(d["g"], net.dims, d["X0"], net.W)
        out.append(cd.subspace_loss(o, d["U"][:, :net.dims[3]].contiguous())[0])
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description="train or evaluate the warm-start network on the GPU")
    ap.add_argument("cmd", choices=["train", "evaluate"])
    ap.add_argument("--workload", default="sbm1m")
    ap.add_argument("--seeds", type=int, default=6)
    ap.add_argument("--graphs", type=int, default=512)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--k", type=int, default=32, choices=[32, 64],
                    help="output width: 32 (the default network) or 64 (the optional 64-wide head)")
    ap.add_argument("--filter", default="f64", choices=["f64", "f32"])
    ap.add_argument("--fixed-features", action="store_true",
                    help="one draw of input channels per graph for the whole training (default: fresh every epoch)")
    ap.add_argument("--schedule", default="cosine", choices=["cosine", "step"])
    ap.add_argument("--targets", default="all", choices=["all", "cluster"],
                    help="all k eigenvectors, or only those of the planted clusters (min(blocks, k))")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    dims = DIMS if a.k == 32 else DIMS_K64
    wfile = a.out or (WEIGHTS_FILE if a.k == 32 else WEIGHTS_FILE_K64)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    if a.cmd == "evaluate":
        import json
        import synth
        edges, n, cfg = synth.make_config_graph(a.workload)
        g = cd.build_laplacian(edges, n)
        trained = Net.load(wfile)
        z = np.load(wfile, allow_pickle=False)
        init_seed = int(z["seed"]) if "seed" in z.files else a.seed
        starts = {"random": None, "untrained": Net.glorot(init_seed, trained.dims), "trained": trained}
        rows = evaluate(g, starts, cfg["k"], cfg["kb"], cfg["m"], seeds=range(1, a.seeds + 1),
                        filter_dtype=cd.F64 if a.filter == "f64" else cd.F32)
        for r in rows:
            log(json.dumps(r))
        print(json.dumps(dict(workload=a.workload, seeds=a.seeds, filter=a.filter, network=os.path.basename(wfile),
                              starts=summarize(rows))), flush=True)
        return

    t0 = time.time()
    data = build_dataset(a.graphs, k=a.k, kb=32, log=log)
    t1 = time.time()
    log("dataset of %d graphs (targets from the FP64 solver, k = %d) in %.1f s" % (len(data), a.k, t1 - t0))
    net, hist = train(data, epochs=a.epochs, lr=a.lr, seed=a.seed, log=log, net=Net.glorot(a.seed, dims),
                      fresh_features=not a.fixed_features, schedule=a.schedule, targets=a.targets)
    torch.cuda.synchronize()
    t2 = time.time()
    log("trained %d epochs in %.1f s" % (a.epochs, t2 - t1))
    net.save(wfile, history=np.array(hist), graphs=a.graphs, epochs=a.epochs, lr=a.lr, seed=a.seed,
             fresh_features=not a.fixed_features, schedule=a.schedule, targets=a.targets,
             train_seconds=t2 - t1, dataset_seconds=t1 - t0)
    log("saved %s" % wfile)


if __name__ == "__main__":
    main()
