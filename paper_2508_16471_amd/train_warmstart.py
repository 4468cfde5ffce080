#!/usr/bin/env python3
"""Train the learned warm start on solutions the solver generates, then
evaluate it against the plain start on held-out bodies.

1. Data: bodies of the Pancharatnam-Berry fin-metasurface family on a
   128^3 grid (seed 5), random channels (20 deg cap about +z, random
   elliptical polarisation), solved by the library to a true FP64 relative
   residual of data_tol (BiCGSTAB, or the block-Jacobi FGMRES of the fast
   path; FP32 products inside FP64 refinement).  Each (body, channel) gives
   one sample: the network input features and the scaled solution, kept on
   the device (about 53 MB per W128 sample).
2. Training: Adam on the masked relative-L2 loss with the library's own
   forward/backward kernels, cosine learning-rate decay.
3. Evaluation: held-out bodies (seed 55, drawn like the benchmark's):
   iterations, solves/s and fallback rate with and without
   the warm start, same solver and tolerance, solved in chunks of `chunk`
   bodies; the final FP64 true residual decides for both.

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


def family(seed, nch, n):
    """Bodies of the family with their nch channels each, drawn one at a time
    from one generator (the same sequence however they are chunked)."""
    from synth import metasurface_family, random_planewave

    rng = np.random.default_rng(seed)
    while True:
        g, eps = metasurface_family(rng, n, 1.0 / 32 * 128 / n)
        chans = [random_planewave(rng, cap_deg=20.0, elliptical=True) for _ in range(nch)]
        yield (eps, g.h, g.origin), chans


def take(it, k):
    bodies, chans = [], []
    for _ in range(k):
        b, c = next(it)
        bodies.append(b)
        chans += c
    return bodies, chans


def solve_fn(V, solver):
    """The solve call of `solver` ("bicgstab", or "fgmres": restart 60, 2 x 2
    block-Jacobi, 8 inner GMRES steps in FP32, as the fast path)."""
    if solver == "fgmres":
        fo = V.fgmres_options(60, (2, 2), 8, V.VIE_MIXED)
        return lambda ctx, cs, nr: V.vie_solve_fgmres(ctx, cs, nr, fo)
    return lambda ctx, cs, nr: V.vie_solve(ctx, cs, nr)


def generate(V, torch, it, nbodies, nch, chunk, tol, solver):
    samples = []
    solve = solve_fn(V, solver)
    t_start = time.perf_counter()
    for c0 in range(0, nbodies, chunk):
        bs, cs = take(it, min(chunk, nbodies - c0))
        t0 = time.perf_counter()
        ctx = V.vie_setup(bs, V.make_options(K0, precision=V.VIE_MIXED, tol=tol, max_iter=20000))
        try:
            _, st = solve(ctx, cs, [nch] * len(bs))
            for b in range(len(bs)):
                for q in range(nch):
                    d = V.vie_cnn_sample_dev(ctx, b, q)
                    ft = torch.empty((d[2], d[1], d[0], 32), dtype=torch.bfloat16, device="cuda")
                    tt = torch.empty((d[2], d[1], d[0], 6), dtype=torch.float32, device="cuda")
                    V.vie_cnn_sample_dev(ctx, b, q, ft.data_ptr(), tt.data_ptr())
                    samples.append((d, ft, tt))
        finally:
            V.vie_destroy(ctx)
        log(f"data: bodies {c0 + len(bs)}/{nbodies}, mean iters {np.mean([s['iters'] for s in st]):.0f}, "
            f"max rel res {max(s['rel_res'] for s in st):.2e}, {time.perf_counter() - t0:.1f} s "
            f"(total {time.perf_counter() - t_start:.0f} s)")
    return samples


def train(V, torch, samples, epochs, lr, seed, checkpoint=None, resume=None, stop_after=None):
    """Adam with cosine decay over epochs x samples steps.  checkpoint: .npz
    path written after every epoch (parameters, Adam moments and step, epoch,
    step, shuffling generator state, loss history); resume: such a file to
    continue from, bit for bit; stop_after: return after that many epochs."""
    net = V.vie_cnn_create(seed)
    rng = np.random.default_rng(seed)
    nsteps = epochs * len(samples)
    step = 0
    ep0 = 0
    hist = []
    if resume:
        with np.load(resume, allow_pickle=False) as z:
            V.vie_cnn_params(net, z["params"])
            V.vie_cnn_adam_state(net, (z["adam_m"], z["adam_v"], int(z["adam_step"])))
            rng.bit_generator.state = json.loads(str(z["rng_state"]))
            ep0, step = int(z["epoch"]), int(z["step"])
            hist = [float(v) for v in z["hist"]]
            if int(z["nsteps"]) != nsteps:
                raise ValueError("checkpoint was written for another schedule")
        log(f"train: resumed after epoch {ep0} from {resume}")
    t0 = time.perf_counter()
    for ep in range(ep0, epochs):
        if stop_after is not None and ep >= stop_after:
            break
        order = rng.permutation(len(samples))
        losses = []
        for i in order:
            d, ft, tt = samples[i]
            lr_t = lr * 0.5 * (1 + np.cos(np.pi * step / nsteps))
            losses.append(V.vie_cnn_train_step_dev(net, d, ft.data_ptr(), tt.data_ptr(), lr_t))
            step += 1
        hist.append(float(np.mean(losses)))
        log(f"train: epoch {ep + 1}/{epochs} mean loss {hist[-1]:.4f} ({time.perf_counter() - t0:.1f} s)")
        if checkpoint:
            m, v, astep = V.vie_cnn_adam_state(net)
            tmp = checkpoint + ".tmp.npz"
            np.savez(tmp, params=V.vie_cnn_params(net), adam_m=m, adam_v=v, adam_step=astep,
                     epoch=ep + 1, step=step, nsteps=nsteps, hist=np.asarray(hist),
                     rng_state=json.dumps(rng.bit_generator.state))
            os.replace(tmp, checkpoint)
    return net, hist, time.perf_counter() - t0


def evaluate(V, torch, net, it, nbodies, nch, tol, inner_tol, solver, chunk):
    """Solve the held-out bodies in chunks, one context per chunk (untimed
    setup), with the plain and then the learned start: per start a warm-up
    solve (autotuning, graph capture), then the timed solve."""
    solve = solve_fn(V, solver)
    legs = (("plain_start", 0), ("warm_start", 1))
    st = {name: [] for name, _ in legs}
    dt = {name: 0.0 for name, _ in legs}
    nsol = 0
    for c0 in range(0, nbodies, chunk):
        bs, cs = take(it, min(chunk, nbodies - c0))
        nsol += len(cs)
        ctx = V.vie_setup(bs, V.make_options(K0, precision=V.VIE_MIXED, tol=tol, max_iter=20000,
                                             inner_tol=inner_tol))
        try:
            V.vie_attach_cnn(ctx, net)
            for name, warm in legs:
                V.vie_set_options(ctx, V.make_options(K0, precision=V.VIE_MIXED, tol=tol,
                                                      max_iter=20000, inner_tol=inner_tol,
                                                      warm_start=warm))
                solve(ctx, cs, [nch] * len(bs))
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, s = solve(ctx, cs, [nch] * len(bs))
                torch.cuda.synchronize()
                dt[name] += time.perf_counter() - t0
                st[name] += s
        finally:
            V.vie_destroy(ctx)
        log(f"eval: bodies {c0 + len(bs)}/{nbodies}, mean iters plain "
            f"{np.mean([x['iters'] for x in st['plain_start']]):.1f} warm "
            f"{np.mean([x['iters'] for x in st['warm_start']]):.1f}")
    out = {}
    for name, warm in legs:
        ss = st[name]
        out[name] = {
            "solves_per_s": nsol / dt[name],
            "iters_mean": float(np.mean([x["iters"] for x in ss])),
            "products_mean": float(np.mean([x["matvecs"] for x in ss])),
            "max_rel_res": float(max(x["rel_res"] for x in ss)),
            "converged": bool(all(x["converged"] for x in ss)),
            "fallback_rate": float(np.mean([x["fallback"] for x in ss])) if warm else None,
            "rel_res_x0_mean": float(np.mean([x["rel_res_x0"] for x in ss])) if warm else 1.0,
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
    ap.add_argument("--solver", choices=["bicgstab", "fgmres"], default="bicgstab",
                    help="data generation and held-out evaluation")
    ap.add_argument("--eval-chunk", type=int, default=8, help="held-out bodies per context")
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--summary", default=None)
    ap.add_argument("--checkpoint", default=None, help=".npz written after every epoch")
    ap.add_argument("--resume", default=None, help="continue training from a checkpoint")
    args = ap.parse_args()

    import torch

    from paper_2508_16471_amd import vie as V

    torch.cuda.set_device(0)
    V.lib()
    samples = generate(V, torch, family(args.seed, args.channels, args.grid), args.train_bodies,
                       args.channels, args.chunk, args.data_tol, args.solver)
    net, hist, ttrain = train(V, torch, samples, args.epochs, args.lr, args.seed,
                              checkpoint=args.checkpoint, resume=args.resume)
    p = V.vie_cnn_params(net)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    np.save(args.out, p.astype(np.float32))
    log(f"saved {p.size} parameters to {args.out}")
    del samples
    torch.cuda.empty_cache()
    ev = evaluate(V, torch, net, family(55, args.heldout_channels, args.grid), args.heldout_bodies,
                  args.heldout_channels, args.tol, args.inner_tol, args.solver, args.eval_chunk)
    summary = {"train_samples": args.train_bodies * args.channels, "epochs": args.epochs,
               "train_bodies": args.train_bodies, "channels_per_body": args.channels,
               "data_tol": args.data_tol, "solver": args.solver, "lr": args.lr,
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
