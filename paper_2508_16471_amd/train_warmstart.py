#!/usr/bin/env python3
"""Train the learned warm start on solutions the solver generates, then
evaluate it against the plain start on held-out bodies.

1. Data: bodies of the Pancharatnam-Berry fin-metasurface family on a
   128^3 grid (seed 5), several random channels each (20 deg cap about +z,
   random elliptical polarisation), solved by the library (FP32 product with
   FP64 refinement, tol 1e-7).  Each (body, channel) gives one sample: the
   network input features and the scaled solution, kept on the device.
2. Training: Adam on the masked relative-L2 loss with the library's own
   forward/backward kernels, cosine learning-rate decay.
3. Evaluation: held-out bodies (seed 55, the benchmark's bodies): iterations,
   solves/s and fallback rate with and without the warm start, same
   tolerance; the final FP64 true residual judges both.

Writes the fp32 parameter vector (numpy .npy) and a JSON summary.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

K0 = 2 * np.pi
DEFAULT_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights",
                               "warmstart_metasurface128.npy")


def log(*a):
    print(*a, flush=True)


def family(seed, nbodies, nch, n):
    from synth import metasurface_family, random_planewave

    rng = np.random.default_rng(seed)
    bodies, chans = [], []
    for _ in range(nbodies):
        g, eps = metasurface_family(rng, n, 1.0 / 32 * 128 / n)
        bodies.append((eps, g.h, g.origin))
        for _ in range(nch):
            chans.append(random_planewave(rng, cap_deg=20.0, elliptical=True))
    return bodies, chans


def generate(V, torch, bodies, chans, nch, chunk, tol):
    samples = []
    for c0 in range(0, len(bodies), chunk):
        bs = bodies[c0:c0 + chunk]
        cs = chans[c0 * nch:(c0 + len(bs)) * nch]
        t0 = time.perf_counter()
        ctx = V.vie_setup(bs, V.make_options(K0, precision=V.VIE_MIXED, tol=tol, max_iter=20000))
        try:
            _, st = V.vie_solve(ctx, cs, [nch] * len(bs))
            for b in range(len(bs)):
                for q in range(nch):
                    d = V.vie_cnn_sample_dev(ctx, b, q)
                    ft = torch.empty((d[2], d[1], d[0], 32), dtype=torch.bfloat16, device="cuda")
                    tt = torch.empty((d[2], d[1], d[0], 6), dtype=torch.float32, device="cuda")
                    V.vie_cnn_sample_dev(ctx, b, q, ft.data_ptr(), tt.data_ptr())
                    samples.append((d, ft, tt))
        finally:
            V.vie_destroy(ctx)
        log(f"data: bodies {c0 + len(bs)}/{len(bodies)}, mean iters {np.mean([s['iters'] for s in st]):.0f}, "
            f"{time.perf_counter() - t0:.1f} s")
    return samples


def train(V, torch, samples, epochs, lr, seed):
    net = V.vie_cnn_create(seed)
    rng = np.random.default_rng(seed)
    nsteps = epochs * len(samples)
    step = 0
    t0 = time.perf_counter()
    hist = []
    for ep in range(epochs):
        order = rng.permutation(len(samples))
        losses = []
        for i in order:
            d, ft, tt = samples[i]
            lr_t = lr * 0.5 * (1 + np.cos(np.pi * step / nsteps))
            losses.append(V.vie_cnn_train_step_dev(net, d, ft.data_ptr(), tt.data_ptr(), lr_t))
            step += 1
        hist.append(float(np.mean(losses)))
        log(f"train: epoch {ep + 1}/{epochs} mean loss {hist[-1]:.4f} ({time.perf_counter() - t0:.1f} s)")
    return net, hist, time.perf_counter() - t0


def evaluate(V, torch, net, bodies, chans, nch, tol, inner_tol):
    out = {}
    for name, warm in (("plain_start", 0), ("warm_start", 1)):
        ctx = V.vie_setup(bodies, V.make_options(K0, precision=V.VIE_MIXED, tol=tol, max_iter=20000,
                                                 inner_tol=inner_tol, warm_start=warm))
        try:
            if warm:
                V.vie_attach_cnn(ctx, net)
            V.vie_solve(ctx, chans, [nch] * len(bodies))  # warm-up (autotuning)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, st = V.vie_solve(ctx, chans, [nch] * len(bodies))
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        finally:
            V.vie_destroy(ctx)
        out[name] = {
            "solves_per_s": len(chans) / dt,
            "iters_mean": float(np.mean([s["iters"] for s in st])),
            "products_mean": float(np.mean([s["matvecs"] for s in st])),
            "max_rel_res": float(max(s["rel_res"] for s in st)),
            "converged": bool(all(s["converged"] for s in st)),
            "fallback_rate": float(np.mean([s["fallback"] for s in st])) if warm else None,
            "rel_res_x0_mean": float(np.mean([s["rel_res_x0"] for s in st])) if warm else 1.0,
        }
        log(f"eval {name}: {out[name]}")
    out["iteration_ratio"] = out["warm_start"]["iters_mean"] / out["plain_start"]["iters_mean"]
    out["speedup"] = out["warm_start"]["solves_per_s"] / out["plain_start"]["solves_per_s"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-bodies", type=int, default=96)
    ap.add_argument("--channels", type=int, default=4)
    ap.add_argument("--heldout-bodies", type=int, default=8)
    ap.add_argument("--heldout-channels", type=int, default=2)
    ap.add_argument("--chunk", type=int, default=8)
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--grid", type=int, default=128)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--data-tol", type=float, default=1e-7)
    ap.add_argument("--inner-tol", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--summary", default=None)
    args = ap.parse_args()

    import torch

    from paper_2508_16471_amd import vie as V

    torch.cuda.set_device(0)
    V.lib()
    tb, tc = family(args.seed, args.train_bodies, args.channels, args.grid)
    samples = generate(V, torch, tb, tc, args.channels, args.chunk, args.data_tol)
    net, hist, ttrain = train(V, torch, samples, args.epochs, args.lr, args.seed)
    p = V.vie_cnn_params(net)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    np.save(args.out, p.astype(np.float32))
    log(f"saved {p.size} parameters to {args.out}")
    del samples
    torch.cuda.empty_cache()
    hb, hc = family(55, args.heldout_bodies, args.heldout_channels, args.grid)
    ev = evaluate(V, torch, net, hb, hc, args.heldout_channels, args.tol, args.inner_tol)
    summary = {"train_samples": args.train_bodies * args.channels, "epochs": args.epochs,
               "train_seconds": ttrain, "loss_history": hist, "heldout": ev,
               "heldout_bodies": args.heldout_bodies, "heldout_channels": args.heldout_channels,
               "tol": args.tol}
    V.vie_cnn_destroy(net)
    js = json.dumps(summary)
    log(js)
    if args.summary:
        with open(args.summary, "w") as f:
            f.write(js + "\n")


if __name__ == "__main__":
    main()
