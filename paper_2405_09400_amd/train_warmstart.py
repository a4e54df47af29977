"""Train the learned warm-start net on cell solves that the method itself produces.

Data: domain decomposition on a 256x256 mixture workload (8-blob Gaussian mixtures, s = 4)
brought to kappa = 1 (eps = h^2) in one of two ways:
  mix256: Knothe-Rosenblatt start, eps-scaling kappa = 64 ... 2 with 4 half-iterations per
          stage;
  ms256:  coarse to fine (layers 8^2 ... 128^2 of 2x2 block sums, kappa = 2, 1, 1/2 with 8
          half-iterations each, refinement between layers), then 8 half-iterations at
          kappa = 2 on the 256^2 layer,
then half-iterations at kappa = 1 with the Sinkhorn tolerance 1e-5.  After every kappa = 1
half-iteration (previous-iterate start) the features of each composite cell and the
correction that takes the start's Y potential g0 to the solved one are taken
(domdec_net_samples).  Several seeds give different mixtures.

Training: Adam on the gauge-invariant weighted squared error of the predicted correction
(dd_net_train_step), mini-batches drawn from a seeded permutation, cosine learning rate.
The last layer starts at zero, so the untrained net gives the correction 0 (one Sinkhorn
iteration from the previous-iterate start).
Every step runs in the library's kernels; this script only orchestrates.

    python -m paper_2405_09400_amd.train_warmstart --out weights.npz
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def generate(seeds, n_k1, N, tol, name="mix256"):
    import torch

    import paper_2405_09400_amd as dd
    import synth

    xs, ts, ws = [], [], []
    for seed in seeds:
        t0 = time.perf_counter()
        w = synth.workload(name, seed=seed, N=N)
        levels = w.extra.get("levels", 0)
        ctx = dd.DomDec(w.mu, w.nu, w.s, w.init, levels=levels)
        k = 0
        for _ in range(levels):
            for kappa in w.extra["layer_kappas"]:
                for _ in range(w.extra["layer_iters"]):
                    ctx.iterate("AB"[k % 2], kappa / ctx.N ** 2, tol=tol)
                    k += 1
            ctx.refine()
        for kappa, its in zip(w.kappas[:-1], w.stage_iters[:-1]):
            for _ in range(its):
                ctx.iterate("AB"[k % 2], kappa / w.N ** 2, tol=tol)
                k += 1
        eps = w.kappas[-1] / w.N ** 2
        for _ in range(n_k1):
            ctx.iterate("AB"[k % 2], eps, tol=tol)
            k += 1
            x, t, wt = ctx.net_samples()
            xs.append(x)
            ts.append(t)
            ws.append(wt)
        ctx.close()
        torch.cuda.synchronize()
        log(f"[train] seed {seed}: {sum(len(x) for x in xs)} samples "
            f"({time.perf_counter() - t0:.1f}s)")
    return torch.cat(xs), torch.cat(ts), torch.cat(ws)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--seeds", type=int, default=10)
    ap.add_argument("--seed0", type=int, default=100)
    ap.add_argument("--k1-iters", type=int, default=20)
    ap.add_argument("--N", type=int, default=256)
    ap.add_argument("--workload", default="ms256", choices=("mix256", "ms256"))
    ap.add_argument("--tol", type=float, default=1e-5)
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--init-seed", type=int, default=0)
    ap.add_argument("--target-scale", type=float, default=0.0,
                    help="train on the targets times this factor and divide the last layer by "
                         "it afterwards (the output layer is linear); 0: one over the RMS of the "
                         "weighted mean-free targets, so that small corrections keep Adam's "
                         "steps in proportion")
    args = ap.parse_args()

    import torch

    import paper_2405_09400_amd as dd

    torch.cuda.set_device(0)
    seeds = list(range(args.seed0, args.seed0 + args.seeds))
    X, T, W = generate(seeds, args.k1_iters, args.N, args.tol, args.workload)
    n = len(X)
    # hold out the last seed's samples for validation
    n_val = max(1, n // args.seeds)
    n_tr = n - n_val
    log(f"[train] {n_tr} training / {n_val} validation samples; target |g| "
        f"p50={T.abs().median().item():.2e} max={T.abs().max().item():.2e}")
    rms = [X[:n_tr, c].pow(2).mean().sqrt().item() for c in range(X.shape[1])]
    log("[train] input channel RMS " + " ".join(f"{r:.2e}" for r in rms))
    e0 = 0.0
    for s0 in range(0, n_tr, 4096):
        e1 = min(n_tr, s0 + 4096)
        sw = W[s0:e1].sum(dim=(1, 2), keepdim=True).clamp_min(1e-30)
        c = (W[s0:e1] * T[s0:e1]).sum(dim=(1, 2), keepdim=True) / sw
        e0 += (W[s0:e1] * (T[s0:e1] - c) ** 2).sum().item()
    e0 /= n_tr
    scale = args.target_scale if args.target_scale > 0 else 1.0 / math.sqrt(max(e0, 1e-30))
    log(f"[train] weighted target energy {e0:.3e}; training on targets x {scale:.3g}")
    T = T * scale
    p0 = dd.net_init_params(args.init_seed)
    p0[-(4 * 32 * 9 + 4):] = 0.0  # last layer (weights [4][32][3][3], bias [4])
    net = dd.WarmStartNet(p0)
    gen = torch.Generator(device="cpu").manual_seed(args.init_seed)
    steps = args.epochs * (n_tr // args.batch)
    step = 0
    hist = []

    def val_loss():
        tot, cnt = 0.0, 0
        for s in range(n_tr, n, 1024):
            e = min(n, s + 1024)
            y = net.forward(X[s:e])
            r = (y - T[s:e])
            sw = W[s:e].sum(dim=(1, 2), keepdim=True).clamp_min(1e-30)
            c = (W[s:e] * r).sum(dim=(1, 2), keepdim=True) / sw
            tot += (W[s:e] * (r - c) ** 2).sum().item()
            cnt += e - s
        return tot / cnt / scale ** 2  # in the units of the targets

    v0 = val_loss()
    log(f"[train] validation loss before training {v0:.4e}")
    t0 = time.perf_counter()
    for ep in range(args.epochs):
        perm = torch.randperm(n_tr, generator=gen).cuda()
        run = 0.0
        nb = n_tr // args.batch
        for b in range(nb):
            idx = perm[b * args.batch:(b + 1) * args.batch]
            lr = args.lr * 0.5 * (1.0 + math.cos(math.pi * step / max(steps, 1)))
            run += net.train_step(X[idx].contiguous(), T[idx].contiguous(), W[idx].contiguous(),
                                  max(lr, 1e-6))
            step += 1
        v = val_loss()
        tr = run / max(nb, 1) / scale ** 2
        hist.append((tr, v))
        log(f"[train] epoch {ep}: train {tr:.4e} val {v:.4e} ({time.perf_counter() - t0:.1f}s)")
    p = net.params()
    p[-(4 * 32 * 9 + 4):] /= scale
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    np.savez(args.out, params=p, val_loss=np.array([v0] + [h[1] for h in hist]),
             train_loss=np.array([h[0] for h in hist]), seeds=np.array(seeds),
             samples=np.array([n_tr, n_val]), k1_iters=np.array(args.k1_iters),
             grid=np.array(args.N), workload=np.array(args.workload),
             target_scale=np.array(scale))
    log(f"[train] wrote {args.out}")
    net.close()


if __name__ == "__main__":
    main()
