#!/usr/bin/env python3
"""Benchmark of the FFT-VIE hot path on one MI355X.

Workload (W128): held-out bodies of the Pancharatnam-Berry fin-metasurface
family on a 128^3 grid (h = lambda/32, FFT 256^3), two plane-wave channels
per body (directions in a 20 deg cap about +z, random elliptical
polarisation), solved to a true relative residual of 1e-6 (FP64 operator).
One step = the whole path for one batch: batched solve of every
(body, channel) -> far field on a 181-point detector scan per body ->
circular (L/R) transfer coefficients -> g2 scan and coincidence curve.

value  = solves/s of the fast path (FP32 FFT product inside FP64 iterative
         refinement, all right-hand sides batched per launch);
plain  = solves/s of the plain path (FP64 product, FP64 BiCGSTAB, x0 = 0,
         one right-hand side per call), reported beside it.
roofline: the dominant kernel's algorithmic bytes (per right-hand-side
         execution, counted from the solver's own product counts) over its
         HIP-event time inside the timed region.
cpu_baseline: the CPU oracle's direct FP64 operator rows (O(N_b) each) timed
         on the host, extrapolated to a full product and scaled by the plain
         path's measured product count per solve.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

K0 = 2 * np.pi
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--bodies", type=int, default=4)
    ap.add_argument("--channels", type=int, default=2)
    ap.add_argument("--grid", type=int, default=128)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--inner-tol", type=float, default=1e-3)
    ap.add_argument("--plain-solves", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="end with 512 MiB fill / sum kernels (HBM counter calibration)")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_2508_16471_amd", "weights",
                                                      "warmstart_metasurface128.npy"))
    ap.add_argument("--mode", choices=["solve", "matvec", "farfield", "uneven", "metasurface",
                                       "sphere", "precond", "paperscale", "cnn", "rooftop"],
                    default="solve",
                    help="matvec: time device-resident operator products only; farfield: "
                         "the 64,800-direction sweep of one body only (profiling); uneven: "
                         "random ellipsoid-union bodies on mixed grids, batched per grid; "
                         "precond: block-Jacobi FGMRES against GMRES and BiCGSTAB on one body")
    ap.add_argument("--nrhs", type=int, default=1, help="matvec mode: vectors per product")
    ap.add_argument("--paper-iters", type=int, default=1024,
                    help="paperscale mode: BiCGSTAB iteration cap of the time-boxed solve")
    ap.add_argument("--directions", type=int, default=64,
                    help="metasurface mode: incident directions of the 64-point (u, v) grid (x 2 circular polarisations)")
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp32")
    ap.add_argument("--solver", choices=["fgmres", "bicgstab"], default=None,
                    help="fast leg: block-Jacobi FGMRES (vie_solve_fgmres) or BiCGSTAB with FP64 "
                         "refinement (vie_solve); default FGMRES, BiCGSTAB in --mode uneven")
    ap.add_argument("--restart", type=int, default=40, help="FGMRES steps per cycle")
    ap.add_argument("--blocks", default="2,2", help="FGMRES lateral block partition bx,by")
    ap.add_argument("--inner-iters", type=int, default=8, help="GMRES steps per block solve")
    ap.add_argument("--block-basis", choices=["fp32", "bf16"], default="bf16",
                    help="storage of the block solves' Arnoldi basis (FP32 products either way)")
    ap.add_argument("--precond-body", choices=["family", "metasurface"], default="family",
                    help="precond mode: the benchmark family (--bodies x --channels) or the "
                         "256x256x48 PB metasurface (one body, --channels uv directions x L/R)")
    ap.add_argument("--no-window", action="store_true",
                    help="solve and precond modes: compute on the full grid instead of the z "
                         "window that holds the bodies (VIE_FLAG_Z_WINDOW)")
    ap.add_argument("--configs", default="",
                    help="precond mode: comma-separated configuration names to run "
                         "(the BiCGSTAB reference always runs)")
    return ap.parse_args()


def make_workload(nb, nch, n):
    from synth import metasurface_family, random_planewave

    rng = np.random.default_rng(55)  # held-out seed of the metasurface family
    bodies, chans = [], []
    for _ in range(nb):
        g, eps = metasurface_family(rng, n, 1.0 / 32 * 128 / n)
        bodies.append((eps, g.h, g.origin, g))
        for _ in range(nch):
            chans.append(random_planewave(rng, cap_deg=20.0, elliptical=True))
    return bodies, chans


def detector_scan():
    psi = np.deg2rad(np.linspace(-90.0, 90.0, 181))
    theta = np.abs(psi)
    phi = np.where(psi < 0, np.pi, 0.0)
    return psi, theta, phi


def post_process(V, ctx, nb, nch, theta, phi, dtau):
    """Far field -> circular transfer coefficients -> g2 scan, classical
    intensity-product scan (eq. 27) and Nc curve."""
    out = []
    i_m10 = 80  # psi = -10 deg
    i_p10 = 100  # psi = +10 deg
    for b in range(nb):
        F = V.vie_farfield(ctx, b, theta, phi, nch)  # [nch][181][2]
        EL = (F[..., 0] + 1j * F[..., 1]) / np.sqrt(2)
        ER = (F[..., 0] - 1j * F[..., 1]) / np.sqrt(2)
        g2s, p2s = [], []
        for j in range(len(theta)):
            T = (ER[0, i_m10], ER[1, i_m10], EL[0, j], EL[1, j])
            g, _, _ = V.hom_g2(T)
            g2s.append(g)
            p2s.append(V.hom_classical_p2(T))
        T = (ER[0, i_m10], ER[1, i_m10], EL[0, i_p10], EL[1, i_p10])
        _, raw, nrm = V.hom_g2(T, 1.2, dtau, V.VIE_NORM_R1)
        out.append((np.array(g2s), np.array(p2s), nrm))
    return out


# ------------------------------------------------------------ byte model
def fft_length(n):
    """The library's circulant length per axis: the smallest 2^k >= 8 or
    3 * 2^k >= 12 that is >= 2n - 1."""
    need = max(8, 2 * n - 1)
    p2, p3 = 8, 12
    while p2 < need:
        p2 *= 2
    while p3 < need:
        p3 *= 2
    return min(p2, p3)


def kernel_bytes(kind, N, P, Q, epi_extra=0, nb=None, vb=16, vin=None):
    """Algorithmic HBM bytes of one right-hand-side execution of a pass
    (spectrum excluded; it is charged once per launch).  nb: body voxels when
    the solver's vectors are body-compressed (x passes read/write 3 nb
    values plus the voxel index and line pointers), None for box vectors.
    vb: bytes of a vector element (16, or 8 for the FP32 vectors of the
    FGMRES products); vin: bytes of an input-vector element when it differs
    (4 for the bfloat16 basis vectors the block products read).  Kinds
    ending in h16 are the packed-FP16 passes: FP16 scratch (4 bytes a
    point), FP32 vectors."""
    N1, N2, N3 = N
    P1, P2, P3 = P
    n = N1 * N2 * N3
    c = 16 if kind.endswith("f64") else (4 if kind.endswith("h16") else 8)
    A = 3 * N3 * N2 * P1
    B = 3 * N3 * P2 * P1
    if kind.startswith("fft_xy_fwd"):  # fused packed x-y: compressed input to y/z scratch
        return 3 * nb * ((vin or vb) + 4) + 3 * (N2 * N3 + 1) * 4 + B * c
    if kind.startswith("fft_yx_inv"):  # fused packed y-x: y/z scratch to compressed output
        return B * c + 3 * nb * (vb + (vin or vb) + 8 + 4) + 3 * (N2 * N3 + 1) * 4 + epi_extra
    if kind.startswith("fft_x_fwd"):
        if nb is not None:
            return 3 * nb * ((vin or vb) + 4) + 3 * (N2 * N3 + 1) * 4 + A * c
        return 3 * n * 16 + A * c
    if kind.startswith("fft_y_fwd"):
        return A * c + B * c
    if kind.startswith(("fft_z_green", "fft_z_h16")):
        return 2 * B * c
    if kind.startswith("fft_y_inv"):
        return B * c + A * c
    if kind.startswith("fft_x_inv"):
        if nb is not None:
            return A * c + 3 * nb * (vb + (vin or vb) + 8 + 4) + 3 * (N2 * N3 + 1) * 4 + epi_extra
        return A * c + 3 * n * 16 * 2 + n * 8 + epi_extra
    raise KeyError(kind)


def spectrum_bytes(kind, Q):
    if kind.endswith("h16"):  # pair-packed FP16 copy: six 8-byte records per column pair
        return 6 * Q[1] * Q[2] * (Q[0] - 1) * 8
    c = 16 if kind.endswith("f64") else 8
    return 6 * Q[0] * Q[1] * Q[2] * c


def roofline_from_times(times, stats, N, P, Q, mixed, nb):
    """Achieved GB/s of every FFT pass over the timed region (nb: mean body
    voxels per right-hand side; the solver's vectors are body-compressed)."""
    iters = np.array([s["iters"] for s in stats])
    cyc = np.array([s["cycles"] for s in stats])
    rows = {}
    for kind, (ms, cnt) in times.items():
        if not kind.startswith("fft_") or cnt == 0 or ms <= 0:
            continue
        f32 = kind.endswith("f32")
        if mixed:
            execs = int((2 * iters).sum()) if f32 else int(cyc.sum())
            launches_active = int(2 * iters.max()) if f32 else int(cyc.max())
        else:
            execs = int((2 * iters + cyc).sum())
            launches_active = int(2 * iters.max() + cyc.max())
        extra = 0
        if kind.startswith("fft_x_inv"):
            extra = 3 * nb * 16 // 2  # rhat read (v = A p) or written (restart), on average
        by = execs * kernel_bytes(kind, N, P, Q, extra, nb=nb)
        if kind.startswith("fft_z_green"):
            by += launches_active * spectrum_bytes(kind, Q)
        rows[kind] = {"ms_total": ms, "launches": int(cnt), "rhs_execs": execs,
                      "bytes": float(by), "GBps": by / (ms * 1e-3) / 1e9,
                      "avg_launch_ms": ms / cnt}
    return rows


def block_geometry(bodies, blocks):
    """The block-Jacobi sub-problem grid the library builds for these bodies
    (same lateral partition, every non-empty block cropped to its bounding
    box, the common grid the largest box extent per axis), the block count of
    every body and the mean body voxels per block."""
    bx, by = blocks

    def bounds(n, parts):
        return [(p * n) // parts for p in range(parts + 1)]

    ext = [1, 1, 1]
    nblk, nbv = [], []
    for e, _, _, g in bodies:
        body = e != 1.0  # (N3, N2, N1)
        n1, n2 = g.n[0], g.n[1]
        xb, yb = bounds(n1, bx), bounds(n2, by)
        cnt = 0
        for py in range(by):
            for px in range(bx):
                sub = body[:, yb[py]:yb[py + 1], xb[px]:xb[px + 1]]
                if not sub.any():
                    continue
                cnt += 1
                nbv.append(int(sub.sum()))
                for a, ax in ((0, (1, 2)), (1, (0, 2)), (2, (0, 1))):
                    idx = np.nonzero(sub.any(axis=ax))[0]
                    ext[2 - a] = max(ext[2 - a], int(idx[-1] - idx[0] + 1))
        nblk.append(cnt)
    P = tuple(fft_length(v) for v in ext)
    return {"N": tuple(ext), "P": P, "Q": tuple(p // 2 + 1 for p in P), "blocks_per_body": nblk,
            "nb_mean": float(np.mean(nbv)) if nbv else 0.0}


def roofline_fgmres(times, stats, N, P, Q, nb, geom, k, nch, block_vin=8, nrm_fused=False):
    """Achieved GB/s of every FFT pass of the FGMRES solve: FP32 outer
    products (one per Arnoldi step), FP64 true-residual products (one per
    cycle) and the FP32 block products (k per step, one execution per block
    of the right-hand side's body).  FP32 products read and write FP32
    vectors, except that block products read their bfloat16 basis vectors
    (block_vin = 4).  nrm_fused: k - 1 of the k fused forward passes of every
    block solve read the FP32 work vector instead (8 bytes) and write the
    normalised bfloat16 basis vector (4 bytes)."""
    iters = np.array([s["iters"] for s in stats])
    cyc = np.array([s["cycles"] for s in stats])
    per_step = len(geom["blocks_per_body"]) * nch  # stats repeat once per timed step
    nblk = np.array([geom["blocks_per_body"][(i % per_step) // nch] for i in range(len(stats))])
    rows = {}
    for kind, (ms, cnt) in times.items():
        blk = kind.startswith("block_")
        base = kind[len("block_"):] if blk else kind
        if not base.startswith("fft_") or cnt == 0 or ms <= 0:
            continue
        f32 = base.endswith(("f32", "h16"))  # FP32 vectors
        if blk:
            Nk, Pk, Qk, nbk = geom["N"], geom["P"], geom["Q"], geom["nb_mean"]
            execs = int((iters * k * nblk).sum())
            launches_active = int(iters.max() * k)
        else:
            Nk, Pk, Qk, nbk = N, P, Q, nb
            execs = int(iters.sum()) if f32 else int(cyc.sum())
            launches_active = int(iters.max()) if f32 else int(cyc.max())
        extra = 3 * nbk * 16 if (base.startswith("fft_x_inv") and not f32 and not blk) else 0
        by = execs * kernel_bytes(base, Nk, Pk, Qk, extra, nb=nbk, vb=8 if f32 else 16,
                                  vin=block_vin if (blk and f32) else None)
        if base.startswith(("fft_z_green", "fft_z_h16")):
            by += launches_active * spectrum_bytes(base, Qk)
        if blk and nrm_fused and base.startswith("fft_xy_fwd"):
            by += int((iters * (k - 1) * nblk).sum()) * 3 * nbk * (8 - block_vin + 4)
        rows[kind] = {"ms_total": ms, "launches": int(cnt), "rhs_execs": execs,
                      "bytes": float(by), "GBps": by / (ms * 1e-3) / 1e9,
                      "avg_launch_ms": ms / cnt}
    return rows


def arnoldi_bytes(stats, nbv, nch, restart, k, block_vb=8, block_nrm_fused=False):
    """Algorithmic HBM bytes of the FGMRES Gram-Schmidt kernels (timing kind
    "arnoldi": one classical Gram-Schmidt pass per step in the mixed path,
    FP32 work vector, basis elements of vb bytes): at step j of a cycle, per
    vector element, the multi-dot reads V_0..V_j and w, the multi-axpy reads
    V_0..V_j and w and writes w, the normalisation reads w and writes
    V_{j+1}: 2 vb j + 3 vb + 32 bytes (16 j + 56 with the FP32 basis).
    Outer process (FP32 basis): every cycle's steps; block solves (basis of
    block_vb bytes: 8, or 4 in bfloat16): k steps per outer step over the
    same elements (the blocks partition the body).  block_nrm_fused: the
    block solves' normalisation runs inside the next packed product (its bytes
    are that kernel's), so a block step is 2 vb j + 2 vb + 24 bytes.  nbv:
    body voxels of each body, stats in body-major order."""
    total = 0.0
    per = len(nbv) * nch
    for i, st in enumerate(stats):
        n = 3 * nbv[(i % per) // nch]
        steps = st["iters"]
        full, rem = divmod(steps, restart)
        cyc = [restart] * full + ([rem] if rem else [])
        outer = sum(8 * c * (c - 1) + 56 * c for c in cyc)
        if block_nrm_fused:
            inner = steps * (block_vb * k * (k - 1) + (2 * block_vb + 24) * k)
        else:
            inner = steps * (block_vb * k * (k - 1) + (3 * block_vb + 32) * k)
        total += n * (outer + inner)
    return total


# ------------------------------------------------------------ CPU oracle
_G = {}


def _oracle_rows(idx):
    from oracle import vie_dense as vd

    return vd.matvec_rows(_G["chi"], _G["pos"], _G["h"], K0, _G["x"], idx)


def cpu_product_time(body, seconds):
    """Oracle rows of the FP64 product on the host (before any GPU use),
    extrapolated to one full product.  Returns (seconds, info)."""
    import multiprocessing as mp

    from oracle import vie_dense as vd

    eps, h, origin, g = body
    chi = (eps - 1).ravel()
    pos = vd.voxel_centres(g.n, g.h, g.origin)
    rng = np.random.default_rng(1)
    bodyvox = np.nonzero(chi)[0]
    x = np.zeros((3, chi.size), complex)
    x[:, bodyvox] = rng.standard_normal((3, len(bodyvox))) + 1j * rng.standard_normal((3, len(bodyvox)))
    _G.update(chi=chi, pos=pos, h=h, x=x)
    workers = max(1, min(16, os.cpu_count() or 1))
    # calibrate on one chunk in this process
    t0 = time.perf_counter()
    _oracle_rows(bodyvox[:8])
    per_row = (time.perf_counter() - t0) / 8
    nrows = int(max(workers * 8, min(len(bodyvox), seconds * workers / max(per_row, 1e-6))))
    sel = rng.choice(bodyvox, size=nrows, replace=False)
    chunks = np.array_split(sel, workers * 4)
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        pool.map(_oracle_rows, chunks)
    wall = time.perf_counter() - t0
    t_product = wall / nrows * len(bodyvox)  # rows off the body are the identity
    return t_product, {"workers": workers, "rows": nrows, "body_rows": len(bodyvox), "wall": wall}


def host_info():
    """CPU model and the cores this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cores": usable}


def cpu_c1_solve():
    """The oracle's dense LU solve of C1 (16^3 sphere, r = lambda/2, eps 2.25,
    6,528 unknowns), timed whole on the host: matrix assembly + LU + solve,
    and one dense product (no extrapolation)."""
    from oracle import vie_dense as vd
    from synth import Grid, sphere

    g = Grid.centred(16, 1.0 / 16)
    chi = (sphere(g, 0.5, 2.25) - 1.0).ravel()
    pos = vd.voxel_centres(g.n, g.h, g.origin)
    t0 = time.perf_counter()
    vd.solve_lu(chi, pos, g.h, K0, (0.0, 0.0, 1.0), (1.0, 0.0, 0.0))
    t_lu = time.perf_counter() - t0
    x = np.zeros((3, chi.size), complex)
    x[:, chi != 0] = 1.0
    t0 = time.perf_counter()
    vd.matvec(chi, pos, g.h, K0, x)
    t_mv = time.perf_counter() - t0
    return {"workload": "C1: 16^3 sphere r=lambda/2, eps 2.25 (2,176 body voxels, 6,528 unknowns)",
            "lu_solve_s": t_lu, "lu_solves_per_s": 1.0 / t_lu, "dense_product_s": t_mv}


def cpu_baseline(t_product, info, plain_products, c1=None):
    solve_s = t_product * plain_products
    out = {"value": 1.0 / solve_s, "unit": "solves/s", "cores": info["workers"], "kind": "oracle",
           "sample": (f"{info['rows']} of {info['body_rows']} body rows of the FP64 product (direct "
                      f"O(N_b) sum per row) on one held-out 128^3 body in {info['wall']:.1f} s wall; "
                      f"scaled to a full product ({t_product:.1f} s) x {plain_products:.0f} "
                      f"products per plain solve (the GPU plain path's measured count)"),
           "host": host_info()}
    if c1 is not None:
        out["c1_measured"] = c1
    return out


# ------------------------------------------------------- product timing
def matvec_mode(args):
    """Time `steps` device-resident operator products of one W128 body."""
    import torch

    from paper_2508_16471_amd import vie as V

    torch.cuda.set_device(0)
    bodies, _ = make_workload(1, 1, args.grid)
    eps, h, o, g = bodies[0]
    prec = V.VIE_MIXED if args.precision == "fp32" else V.VIE_FP64
    ctx = V.vie_setup([(eps, h, o)], V.make_options(K0, flags=V.VIE_FLAG_TIMING))
    N, P, _ = V.vie_grid(ctx, 0)  # the z window the passes run on
    Q = tuple(p // 2 + 1 for p in P)
    n = g.n[0] * g.n[1] * g.n[2]  # box vectors stay in the body's grid
    x = torch.randn(args.nrhs, 3 * n, dtype=torch.complex128, device="cuda")
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream().cuda_stream
    V.vie_set_stream(ctx, stream)
    for _ in range(max(1, args.warmup)):
        V.vie_matvec_dev(ctx, 0, x.data_ptr(), y.data_ptr(), args.nrhs, prec)
    torch.cuda.synchronize()
    V.vie_kernel_times(ctx, reset=True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        V.vie_matvec_dev(ctx, 0, x.data_ptr(), y.data_ptr(), args.nrhs, prec)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    times = V.vie_kernel_times(ctx, reset=True)
    V.vie_destroy(ctx)
    calib_copy(torch)  # FETCH_SIZE / WRITE_SIZE calibration kernels
    rows = {}
    for kind, (ms, cnt) in times.items():
        if not kind.startswith("fft_") or cnt == 0:
            continue
        by = args.steps * args.nrhs * kernel_bytes(kind, N, P, Q)
        if kind.startswith("fft_z_green"):
            by += args.steps * spectrum_bytes(kind, Q)
        rows[kind] = {"avg_launch_ms": ms / cnt, "GBps": by / (ms * 1e-3) / 1e9, "launches": cnt}
    total = sum(v["avg_launch_ms"] for v in rows.values())
    print(json.dumps({"mode": "matvec", "precision": args.precision, "nrhs": args.nrhs,
                      "calibration": {"fill_bytes_written": 512 << 20, "sum_bytes_read": 512 << 20},
                      "grid": list(g.n), "window": list(N), "fft": list(P),
                      "ms_per_product": dt / args.steps * 1e3,
                      "kernel_ms_per_product": total, "kernels": rows}))


# ------------------------------------------------------- HBM counters
def calib_copy(torch):
    """Kernels of known HBM traffic for the FETCH_SIZE / WRITE_SIZE counters:
    a device fill writes 512 MiB, a device sum reads 512 MiB (three each)."""
    cbytes = 512 << 20
    ca = torch.empty(cbytes // 4, dtype=torch.float32, device="cuda")
    for _ in range(3):
        ca.fill_(1.0)
    for _ in range(3):
        float(ca.sum())
    torch.cuda.synchronize()


def measured_traffic(kind, avg_launch_ms):
    """HBM bytes per launch of `kind` from the committed counter summary
    (profiles/traffic_<kind>.json, written by profsum traffic), or None when
    it is missing or the product sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kind}.json")
    if not os.path.exists(path):
        return None
    from paper_2508_16471_amd.profsum import sources_sha

    with open(path) as f:
        rec = json.load(f)
    if rec.get("sources_sha256") != sources_sha():
        return None
    return {"bytes_per_launch": rec["bytes_per_dispatch"],
            "GBps": rec["bytes_per_dispatch"] / (avg_launch_ms * 1e-3) / 1e9,
            "fetch_scale": rec["fetch_scale"], "write_scale": rec["write_scale"],
            "source": os.path.relpath(path, ROOT)}


# ------------------------------------------------------- extra legs
def other_rows(times):
    """Time of the non-FFT kernel kinds over the timed region."""
    return {k: {"ms_total": ms, "launches": int(cnt)} for k, (ms, cnt) in times.items()
            if not k.startswith(("fft_", "block_fft_")) and cnt > 0}


def learned_leg(V, torch, ctx, args, chans, nb, nch, theta, phi, dtau, fast_value, solve):
    """The fast path (solver `solve`) with the trained warm-start network
    attached (same bodies, same step); the plain start stays the fallback."""
    net = V.vie_cnn_create(0)
    try:
        V.vie_cnn_params(net, np.load(args.weights))
        V.vie_attach_cnn(ctx, net)
        V.vie_set_options(ctx, V.make_options(K0, precision=V.VIE_MIXED, tol=args.tol,
                                              max_iter=20000, inner_tol=args.inner_tol,
                                              warm_start=1, flags=args.wflag))
        solve()  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = []
        for _ in range(args.steps):
            _, s = solve()
            post_process(V, ctx, nb, nch, theta, phi, dtau)
            st += s
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        val = args.steps * nb * nch / dt
        return {"solves_per_s": val, "vs_fast": val / fast_value,
                "iters_mean": float(np.mean([x["iters"] for x in st])),
                "fallback_rate": float(np.mean([x["fallback"] for x in st])),
                "rel_res_x0_mean": float(np.mean([x["rel_res_x0"] for x in st])),
                "converged": all(x["converged"] for x in st),
                "max_rel_res": max(x["rel_res"] for x in st),
                "weights": os.path.relpath(args.weights, ROOT)}
    finally:
        V.vie_attach_cnn(ctx, None)
        V.vie_cnn_destroy(net)


def farfield_sweep(V, torch, ctx, args, chans, nch, nbv, reps=3):
    """360 x 180 far-field sweep (64,800 directions) of body 0's channels on
    the FP64-MFMA contraction; achieved rate from the kernel-kind time."""
    V.vie_set_options(ctx, V.make_options(K0, precision=V.VIE_MIXED, tol=args.tol, max_iter=20000,
                                          inner_tol=args.inner_tol,
                                          flags=V.VIE_FLAG_TIMING | args.wflag))
    V.vie_solve(ctx, chans[:nch], [nch] + [0] * (len(chans) // nch - 1))
    th1 = (np.arange(180) + 0.5) * np.pi / 180
    ph1 = np.arange(360) * 2 * np.pi / 360 - np.pi
    TH, PH = np.meshgrid(th1, ph1, indexing="ij")
    V.vie_farfield(ctx, 0, TH.ravel(), PH.ravel(), nch)
    V.vie_kernel_times(ctx, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        V.vie_farfield(ctx, 0, TH.ravel(), PH.ravel(), nch)
    wall = (time.perf_counter() - t0) / reps
    ms, cnt = V.vie_kernel_times(ctx, reset=True).get("farfield", (0.0, 0))
    flop = 8.0 * TH.size * nbv * 3 * nch  # complex multiply-adds of the voxel sum
    dev_s = ms / max(cnt, 1) * 1e-3
    return {"directions": int(TH.size), "channels": nch, "body_voxels": nbv,
            "device_ms": dev_s * 1e3, "wall_ms": wall * 1e3,
            "tflops": flop / dev_s / 1e12 if dev_s > 0 else None,
            "frac_fp64_peak": flop / dev_s / 78.6e12 if dev_s > 0 else None}


def na_detection(V, torch, ctx, nch):
    """Finite-aperture detection on body 0: detector a (R circular, psi = -10 deg)
    and detector b (L circular, psi = +10 deg) in the xz plane, uniform cones of
    NA = sin(alpha) (12 x 24 quadrature nodes each), g2 of the two channels per NA."""
    rows = []
    for na in (0.0, 0.05, 0.1, 0.2, 0.3, 0.5):
        al = float(np.arcsin(na))
        dets = []
        for psi, sgn in ((-10.0, -1.0), (10.0, 1.0)):
            t0, p0 = np.deg2rad(abs(psi)), (np.pi if psi < 0 else 0.0)
            th = np.array([np.cos(t0) * np.cos(p0), np.cos(t0) * np.sin(p0), -np.sin(t0)])
            ph = np.array([-np.sin(p0), np.cos(p0), 0.0])
            dets.append((t0, p0, al, (th + 1j * sgn * ph) / np.sqrt(2)))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        T = V.vie_transfer_na(ctx, 0, dets, nch, 12, 24)
        sec = time.perf_counter() - t1
        g2 = V.hom_g2((T[0, 0], T[1, 0], T[0, 1], T[1, 1]))[0] if nch >= 2 else None
        rows.append({"NA": na, "g2": g2, "seconds": sec})
    return {"detectors": "R at psi=-10 deg, L at psi=+10 deg, uniform cone, 12x24 nodes",
            "body": 0, "rows": rows}


def sphere_leg(V, torch, args):
    """The secondary W128 body: a sphere r = 2 lambda, eps 2.25 on the same
    128^3 grid (h = lambda/32, about 52 % fill), k = z, x-polarised, tol as the
    main run: plain FP64 against the fast (mixed) path, one solve each after a
    warm-up."""
    from synth import Grid, sphere

    g = Grid.centred(args.grid, 1.0 / 32 * 128 / args.grid)
    eps = sphere(g, 2.0, 2.25)
    ch = [((0, 0, 1.0), (1.0, 0, 0))]
    out = {"workload": f"sphere r=2 lambda, eps 2.25, {args.grid}^3, h=lambda/32, k=z, x-pol",
           "body_voxels": int((eps != 1.0).sum())}
    for label, prec in (("plain_fp64", V.VIE_FP64), ("fast", V.VIE_MIXED)):
        ctx = V.vie_setup([(eps, g.h, g.origin)], V.make_options(K0, precision=prec, tol=args.tol,
                                                                max_iter=20000, inner_tol=args.inner_tol))
        try:
            V.vie_solve(ctx, ch, [1])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, st = V.vie_solve(ctx, ch, [1])
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        finally:
            V.vie_destroy(ctx)
        out[label] = {"solves_per_s": 1.0 / dt, "iters": st[0]["iters"], "rel_res": st[0]["rel_res"]}
    out["speedup"] = out["fast"]["solves_per_s"] / out["plain_fp64"]["solves_per_s"]
    return out


def farfield_mode(args):
    """Solve body 0 of the workload (its channels), then time the far-field
    sweep alone (`steps` sweeps)."""
    import torch

    from paper_2508_16471_amd import vie as V

    torch.cuda.set_device(0)
    V.lib()
    bodies, chans = make_workload(1, args.channels, args.grid)
    eps, h, o, g = bodies[0]
    ctx = V.vie_setup([(eps, h, o)], V.make_options(K0, precision=V.VIE_MIXED, tol=args.tol,
                                                   max_iter=20000, inner_tol=args.inner_tol,
                                                   flags=V.VIE_FLAG_TIMING))
    try:
        sweep = farfield_sweep(V, torch, ctx, args, chans, args.channels, int((eps != 1.0).sum()),
                               reps=max(1, args.steps))
    finally:
        V.vie_destroy(ctx)
    print(json.dumps({"mode": "farfield", "grid": list(g.n), "farfield_sweep": sweep}))


def cnn_flops_per_voxel(backward=False):
    """Algorithmic flops of the network per box voxel: 2 x 27 taps x Cin x
    Cout per layer (forward); a training step adds the weight gradient of
    every layer and the data gradient of all but the first."""
    ch = [32, 32, 32, 32, 16]
    macs = [27 * ci * co for ci, co in zip(ch[:-1], ch[1:])]
    f = 2 * sum(macs)
    if backward:
        f += 2 * sum(macs) + 2 * sum(macs[1:])
    return f


def cnn_mode(args):
    """The warm-start network alone on the box of one W128 benchmark body
    (bounding box + 4-voxel halo): `steps` forward inferences, then `steps`
    training steps (forward, masked loss, backward, Adam), on synthetic bf16
    features and fp32 targets; HIP events on the stream the library runs on."""
    import torch

    from paper_2508_16471_amd import vie as V

    torch.cuda.set_device(0)
    V.lib()
    bodies, chans = make_workload(1, 1, args.grid)
    eps, h, o, g = bodies[0]
    ctx = V.vie_setup([(eps, h, o)], V.make_options(K0, precision=V.VIE_MIXED, tol=1e-2))
    try:
        V.vie_solve(ctx, chans, [1])  # sizes the body's channel storage
        d = V.vie_cnn_sample_dev(ctx, 0, 0)
    finally:
        V.vie_destroy(ctx)
    nv = d[0] * d[1] * d[2]
    gen = torch.Generator(device="cuda").manual_seed(7)
    feat = torch.randn((d[2], d[1], d[0], 32), generator=gen, device="cuda").to(torch.bfloat16)
    feat[..., 0] = (torch.rand((d[2], d[1], d[0]), generator=gen, device="cuda") < 0.3).to(
        torch.bfloat16)  # channel 0 doubles as the loss mask (body voxels)
    tgt = torch.randn((d[2], d[1], d[0], 6), generator=gen, device="cuda")
    out = torch.empty((d[2], d[1], d[0], 16), device="cuda")
    net = V.vie_cnn_create(0)
    st = torch.cuda.current_stream()
    res = {}
    try:
        def timed(fn, reps):
            fn()
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(st)
            for _ in range(reps):
                fn()
            b.record(st)
            b.synchronize()
            return a.elapsed_time(b) / reps

        reps = max(1, args.steps)
        ms_f = timed(lambda: V.vie_cnn_infer_dev(net, d, feat.data_ptr(), out.data_ptr(),
                                                 st.cuda_stream), 4 * reps)
        ms_t = timed(lambda: V.vie_cnn_train_step_dev(net, d, feat.data_ptr(), tgt.data_ptr(),
                                                      1e-4, st.cuda_stream), reps)
        for name, ms, bw in (("forward", ms_f, False), ("train_step", ms_t, True)):
            fl = cnn_flops_per_voxel(bw) * nv
            res[name] = {"ms": ms, "flop": fl, "TFLOPs": fl / (ms * 1e-3) / 1e12,
                         "frac_bf16_mfma_peak": fl / (ms * 1e-3) / 1e12 / 2500.0}
    finally:
        V.vie_cnn_destroy(net)
    print(json.dumps({"mode": "cnn", "box": list(d), "voxels": nv, "data": "synthetic",
                      "peak_TFLOPs": 2500.0, **res}))


def uneven_mode(args):
    """Uneven batch: `bodies` random ellipsoid unions (1-6 ellipsoids, semi-axes
    U[0.2, 1], eps U[1.5, 6]) on grids drawn from {32, 48, 64, 96}^3 (h = 1/16),
    4 channels each (k uniform on the sphere, random linear polarisation).
    Bodies sharing a grid form one batched group; groups are solved in grid
    order, one call each, and a solve's latency is the time from the first
    call's start to its own completion (its group call's start plus the
    device-measured completion time `seconds` the library reports), beside
    the end of its group's call.  Solver as --solver (FGMRES:
    --blocks, --inner-iters, --restart, --block-basis).  Run with replayed
    graphs and, for comparison, with eager launches."""
    import torch

    from paper_2508_16471_amd import vie as V
    from synth import Grid, random_ellipsoid_body

    torch.cuda.set_device(0)
    V.lib()
    rng = np.random.default_rng(4)
    sizes = [32, 48, 64, 96]
    nb = args.bodies
    nch = 4
    grid_of = [int(rng.choice(sizes)) for _ in range(nb)]
    bodies, chans = [], []
    for n in grid_of:
        g = Grid.centred(n, 1.0 / 16)
        bodies.append((random_ellipsoid_body(rng, g), g.h, g.origin))
        for _ in range(nch):
            k = rng.standard_normal(3)
            k /= np.linalg.norm(k)
            p = np.cross(k, rng.standard_normal(3))
            chans.append((k, p / np.linalg.norm(p)))
    out = {"mode": "uneven", "bodies": nb, "channels_per_body": nch,
           "grids": {str(n): grid_of.count(n) for n in sizes}, "tol": args.tol,
           "solver": args.solver or "bicgstab"}
    fo = None
    if args.solver == "fgmres":
        fo = V.fgmres_options(args.restart, tuple(int(v) for v in args.blocks.split(",")),
                              args.inner_iters,
                              V.VIE_MIXED_BF16 if args.block_basis == "bf16" else V.VIE_MIXED)
        out["fgmres"] = {"restart": args.restart, "blocks": args.blocks,
                         "inner_iters": args.inner_iters, "block_basis": args.block_basis}

    def solve(ctx, ch, cnt):
        if fo is not None:
            return V.vie_solve_fgmres(ctx, ch, cnt, fo)
        return V.vie_solve(ctx, ch, cnt)

    for label, flags in (("graph", 0), ("eager", V.VIE_FLAG_NO_GRAPH)):
        opt = V.make_options(K0, precision=V.VIE_MIXED, tol=args.tol, max_iter=20000,
                             inner_tol=args.inner_tol, flags=flags)
        t0 = time.perf_counter()
        ctx = V.vie_setup(bodies, opt)
        setup = time.perf_counter() - t0
        try:
            for n in sizes:  # warm-up: tuning and graph capture per group
                cnt = [nch if grid_of[b] == n else 0 for b in range(nb)]
                if sum(cnt):
                    solve(ctx, [c for b, c in enumerate(chans) if cnt[b // nch]], cnt)
                    print(f"uneven {label} warm-up grid {n} done", file=sys.stderr, flush=True)
            torch.cuda.synchronize()
            lat, lat_end, groups, iters = [], [], {}, []
            t0 = time.perf_counter()
            for n in sizes:
                cnt = [nch if grid_of[b] == n else 0 for b in range(nb)]
                if not sum(cnt):
                    continue
                tg = time.perf_counter()
                _, st = solve(ctx, [c for b, c in enumerate(chans) if cnt[b // nch]], cnt)
                now = time.perf_counter()
                groups[str(n)] = {"rhs": sum(cnt), "seconds": now - tg,
                                  "iters_mean": float(np.mean([x["iters"] for x in st])),
                                  "converged": all(x["converged"] for x in st)}
                lat += [tg - t0 + x["seconds"] for x in st]
                lat_end += [now - t0] * len(st)
                iters += [x["iters"] for x in st]
                print(f"uneven {label} grid {n}: {groups[str(n)]}", file=sys.stderr, flush=True)
            total = time.perf_counter() - t0
        finally:
            V.vie_destroy(ctx)
        lat, lat_end = np.array(lat), np.array(lat_end)
        out[label] = {"solves_per_s": len(lat) / total, "seconds": total, "setup_s": setup,
                      "latency_s": {"p50": float(np.percentile(lat, 50)),
                                    "p90": float(np.percentile(lat, 90)),
                                    "p99": float(np.percentile(lat, 99))},
                      "group_end_s": {"p50": float(np.percentile(lat_end, 50)),
                                      "p90": float(np.percentile(lat_end, 90)),
                                      "p99": float(np.percentile(lat_end, 99))},
                      "iters_mean": float(np.mean(iters)), "groups": groups}
        print(json.dumps({label: out[label]}), file=sys.stderr, flush=True)
    # launch-bound case: one 16^3 sphere (r = lambda/2, eps 2.25), one channel
    g = Grid.centred(16, 1.0 / 16)
    from synth import sphere

    body = [(sphere(g, 0.5, 2.25), g.h, g.origin)]
    small = {}
    for label, flags in (("graph", 0), ("eager", V.VIE_FLAG_NO_GRAPH)):
        ctx = V.vie_setup(body, V.make_options(K0, precision=V.VIE_FP64, tol=1e-8, max_iter=5000,
                                               flags=flags))
        try:
            V.vie_solve(ctx, [((0, 0, 1.0), (1.0, 0, 0))], [1])
            ts = []
            for _ in range(20):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, st = V.vie_solve(ctx, [((0, 0, 1.0), (1.0, 0, 0))], [1])
                ts.append(time.perf_counter() - t0)
        finally:
            V.vie_destroy(ctx)
        small[label] = {"median_ms": float(np.median(ts)) * 1e3, "iters": st[0]["iters"]}
    out["small_single_solve"] = {"workload": "16^3 sphere r=0.5, eps 2.25, 1 channel, FP64, tol 1e-8",
                                 **small}
    print(json.dumps(out))


def paperscale_mode(args):
    """The paper's full-wave PB metasurface at its stated size (Sec. III-B:
    40 x 12 x 2 wavelengths at 62 cells per wavelength, 2480 x 744 x 124
    voxels, 91 x 27 silicon fins (eps 11.83) with the 13.44 deg PB rotation
    step of eq. 32 on a glass substrate; 17.5 M body voxels, 52.5 M unknowns)
    on one GPU, computed on the z window (FFT 6144 x 1536 x 96).  Setup,
    device memory, FP32 and FP64 product times (device vectors, 1 RHS), then
    a time-boxed mixed-precision BiCGSTAB solve of both circular
    polarisations at normal incidence (batched), `--paper-iters` iterations
    at most: the true residual reached and the time per iteration."""
    import torch

    from paper_2508_16471_amd import vie as V
    from synth import circular_pol_basis, paper_metasurface

    torch.cuda.set_device(0)
    V.lib()
    t0 = time.perf_counter()
    g, eps = paper_metasurface()
    t_gen = time.perf_counter() - t0
    nb = int((eps != 1.0).sum())
    k = np.array([0.0, 0.0, 1.0])
    _, _, L, R = circular_pol_basis(k)
    chans = [(k, L), (k, R)]
    free0 = torch.cuda.mem_get_info()[0]
    t0 = time.perf_counter()
    ctx = V.vie_setup([(eps, g.h, g.origin)],
                      V.make_options(K0, precision=V.VIE_MIXED, tol=args.tol,
                                     max_iter=args.paper_iters, flags=V.VIE_FLAG_Z_WINDOW))
    t_setup = time.perf_counter() - t0
    win, fft, _ = V.vie_grid(ctx, 0)
    print(f"paper scale: {nb} body voxels, window {win}, fft {fft}, setup {t_setup:.2f} s",
          file=sys.stderr, flush=True)
    x = torch.zeros((3, eps.size), dtype=torch.complex128, device="cuda")
    x[:, torch.from_numpy(np.nonzero(eps.ravel() != 1.0)[0]).cuda()] = 1.0
    y = torch.empty_like(x)
    prod = {}
    for label, prec in (("fp32", V.VIE_MIXED), ("fp64", V.VIE_FP64)):
        V.vie_matvec_dev(ctx, 0, x.data_ptr(), y.data_ptr(), 1, prec)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(3):
            V.vie_matvec_dev(ctx, 0, x.data_ptr(), y.data_ptr(), 1, prec)
        torch.cuda.synchronize()
        prod[label + "_ms"] = (time.perf_counter() - t1) / 3 * 1e3
    del x, y
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, st = V.vie_solve(ctx, chans, [2], allow_noconv=True)
    t_solve = time.perf_counter() - t0
    used = (free0 - torch.cuda.mem_get_info()[0]) / 2**30
    V.vie_destroy(ctx)
    iters = max(s["iters"] for s in st)
    line = {"mode": "paperscale",
            "workload": ("paper-scale PB metasurface: 40x12x2 lambda at 62 cells/lambda "
                         "(2480x744x124), 91x27 Si fins (eps 11.83) on glass (eps 2.25), "
                         f"{nb} body voxels ({3 * nb} unknowns); z window {list(win)}, "
                         f"FFT {list(fft)}; normal incidence, L and R, batched, mixed"),
            "generate_s": t_gen, "setup_s": t_setup, "device_GiB": used,
            "product_ms_device_vectors": prod,
            "solve": {"iterations": [s["iters"] for s in st], "converged": [s["converged"] for s in st],
                      "true_rel_res": [s["rel_res"] for s in st], "seconds": t_solve,
                      "ms_per_iteration": t_solve / max(iters, 1) * 1e3, "tol": args.tol,
                      "iteration_cap": args.paper_iters},
            "paper": "31.9 h (24 h with the 7x7 block preconditioner) on 24 CPU threads, 54,041,130 unknowns"}
    print(json.dumps(line))


def metasurface_mode(args):
    """PB metasurface on the 256 x 256 x 48 grid (h = lambda/60, 8 x 8 fins of
    eps 5.8 on an eps 2.1 slab, 1.28 M body voxels): incident directions
    (u, v, sqrt(1 - u^2 - v^2)) with u, v in {-0.3, ..., 0.4} (64, normal
    incidence included; `directions` < 64 takes an evenly strided subset),
    each with both circular polarisations, solved as one batched call (FP32
    product inside FP64 refinement, replayed graphs; the call includes the
    one-off z-shape tuning and graph capture), then a 362-direction far-field
    scan (theta in [0, 180] deg in the phi = 0 and phi = 90 deg planes) of
    every right-hand side."""
    import torch

    from paper_2508_16471_amd import vie as V
    from synth import circular_pol_basis, pb_metasurface, uv_directions

    torch.cuda.set_device(0)
    V.lib()
    g, eps = pb_metasurface()
    chans = []
    dirs = uv_directions()
    if args.directions < len(dirs):
        pick = np.linspace(0, len(dirs) - 1, args.directions).round().astype(int)
        normal = int(np.argmin(np.abs(dirs[:, 0]) + np.abs(dirs[:, 1])))
        if normal not in pick:
            pick[np.argmin(np.abs(pick - normal))] = normal  # keep normal incidence
        dirs = dirs[np.unique(pick)]
    for k in dirs:
        _, _, L, R = circular_pol_basis(k)
        chans += [(k, L), (k, R)]
    nrhs = len(chans)
    nb = int((eps != 1.0).sum())
    N = g.n
    P = tuple(fft_length(v) for v in N)
    free0 = torch.cuda.mem_get_info()[0]
    opt = V.make_options(K0, precision=V.VIE_MIXED, tol=args.tol, max_iter=20000,
                         inner_tol=args.inner_tol)
    t0 = time.perf_counter()
    ctx = V.vie_setup([(eps, g.h, g.origin)], opt)
    setup = time.perf_counter() - t0
    print(f"metasurface: setup {setup:.2f} s, {nrhs} right-hand sides, {nb} body voxels",
          file=sys.stderr, flush=True)
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, st = V.vie_solve(ctx, chans, [nrhs], allow_noconv=True)
        torch.cuda.synchronize()
        solve_s = time.perf_counter() - t0
        used = (free0 - torch.cuda.mem_get_info()[0]) / 1e9
        print(f"metasurface: solve {solve_s:.2f} s rc {rc}", file=sys.stderr, flush=True)
        th = np.deg2rad(np.linspace(0.0, 180.0, 181))
        theta = np.concatenate([th, th])
        phi = np.concatenate([np.zeros(181), np.full(181, np.pi / 2)])
        V.vie_farfield(ctx, 0, theta, phi, nrhs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        V.vie_farfield(ctx, 0, theta, phi, nrhs)
        torch.cuda.synchronize()
        ff_s = time.perf_counter() - t0
        # two photons in H and V at normal incidence (linear combinations of the
        # L and R solutions), L detection at +psi, R detection at -psi, in the
        # xz plane along the rotation gradient
        i0 = int(np.argmin(np.abs(dirs[:, 0]) + np.abs(dirs[:, 1])))
        psi = np.deg2rad(np.linspace(-90.0, 90.0, 181))
        Fs = V.vie_farfield(ctx, 0, np.abs(psi), np.where(psi < 0, np.pi, 0.0), nrhs)
        FL, FR = Fs[2 * i0], Fs[2 * i0 + 1]  # [psi][theta/phi component]
        FH = (FL + FR) / np.sqrt(2)
        FV = (FL - FR) / (1j * np.sqrt(2))
        projL = lambda F: (F[..., 0] + 1j * F[..., 1]) / np.sqrt(2)  # noqa: E731
        projR = lambda F: (F[..., 0] - 1j * F[..., 1]) / np.sqrt(2)  # noqa: E731
        # first diffraction order of the 8-fin supercell (it spans the grid: n[0] h)
        design = float(np.degrees(np.arcsin(1.0 / (g.n[0] * g.h))))
        g2lr = {}
        for ang in (design, 10.0):
            a = np.deg2rad(ang)
            Fd = V.vie_farfield(ctx, 0, np.array([a, a]), np.array([0.0, np.pi]), nrhs)
            dH = (Fd[2 * i0] + Fd[2 * i0 + 1]) / np.sqrt(2)
            dV = (Fd[2 * i0] - Fd[2 * i0 + 1]) / (1j * np.sqrt(2))
            T = (projL(dH)[0], projL(dV)[0], projR(dH)[1], projR(dV)[1])
            g2lr[f"{ang:.2f}"] = {"g2": V.hom_g2(T)[0], "P2_classical": V.hom_classical_p2(T)}
        ia = int(np.argmin(np.abs(np.degrees(psi) - design)))
        scan = np.array([V.hom_g2((projL(FH)[ia], projL(FV)[ia], projR(FH)[j], projR(FV)[j]))[0]
                         for j in range(len(psi))])
        g2_out = {"channels": "H, V at normal incidence (from the L/R solutions)",
                  "detectors": "L at +psi, R at -psi, xz plane (scan: R detector on 1-deg steps)",
                  "design_order_deg": design, "at": g2lr,
                  "scan_b_min": float(np.nanmin(scan)), "scan_b_max": float(np.nanmax(scan))}
    finally:
        V.vie_destroy(ctx)
    it = [x["iters"] for x in st]
    flops = 8.0 * theta.size * nb * 3 * nrhs
    print(json.dumps({
        "mode": "metasurface", "workload": "PB metasurface 256x256x48, h=lambda/60, 8x8 fins eps 5.8 "
        "(9x24x36 cells, period 32 cells), slab eps 2.1 (12 cells), directions u,v in -0.3..0.4 x L/R", "grid": list(N), "fft": list(P), "body_voxels": nb, "rhs": nrhs,
        "tol": args.tol, "precision": "fp32 product + fp64 refinement", "setup_s": setup,
        "solve_s": solve_s, "solves_per_s": nrhs / solve_s, "rc": rc,
        "iters_mean": float(np.mean(it)), "iters_max": int(np.max(it)),
        "all_converged": all(x["converged"] for x in st),
        "max_rel_res": float(max(x["rel_res"] for x in st)), "device_mem_GB": used,
        "farfield": {"directions": int(theta.size), "seconds": ff_s,
                     "TFLOPs": flops / ff_s / 1e12},
        "g2_LR": g2_out}))


def sphere_mode(args):
    """The paper's sphere study at full size: r = 1 lambda, eps 4, 64^3 voxels
    (h = 2.05/64), two channels at theta = +-30 deg (y-polarised), both
    precisions.  Far-field sweep 360 x 180 per channel, z-detection
    (c = (-sin theta, 0)) transfer coefficients, the g2 map (eq. 10) and the
    classical intensity-product map (eq. 27) over (phi1, phi2) in 1 deg steps at
    theta1 = 45, theta2 = 135 deg, the g2 map over (theta1, theta2) at
    (phi1, phi2) = (0, 180 deg), and coincidence curves (200 delays) at the
    (phi1, phi2) map's minimum, median and maximum g2 and at its pair closest
    to a single path."""
    import torch

    from paper_2508_16471_amd import vie as V
    from synth import Grid, sphere

    torch.cuda.set_device(0)
    V.lib()
    g = Grid.centred((64, 64, 64), 2.05 / 64)
    eps = sphere(g, 1.0, 4.0)
    a = np.deg2rad(30.0)
    chans = [((np.sin(a), 0, np.cos(a)), (0, 1.0, 0)), ((-np.sin(a), 0, np.cos(a)), (0, 1.0, 0))]
    out = {"mode": "sphere", "workload": "sphere r=1 lambda, eps 4, 64^3, h=2.05/64, channels "
           "theta=+-30 deg (y-pol), z-detection", "body_voxels": int((eps != 1.0).sum())}
    th1 = (np.arange(180) + 0.5) * np.pi / 180
    ph1 = np.arange(360) * 2 * np.pi / 360 - np.pi
    TH, PH = np.meshgrid(th1, ph1, indexing="ij")
    for label, prec in (("fp64", V.VIE_FP64), ("mixed", V.VIE_MIXED)):
        ctx = V.vie_setup([(eps, g.h, g.origin)], V.make_options(K0, precision=prec, tol=1e-6,
                                                                max_iter=20000))
        try:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, st = V.vie_solve(ctx, chans, [2])
            torch.cuda.synchronize()
            ts = time.perf_counter() - t0
            t0 = time.perf_counter()
            V.vie_farfield(ctx, 0, TH.ravel(), PH.ravel(), 2)
            tf = time.perf_counter() - t0
            phis = np.deg2rad(np.arange(360.0))
            t0 = time.perf_counter()
            Fa = V.vie_farfield(ctx, 0, np.full(360, np.pi / 4), phis, 2)[..., 0]
            Fb = V.vie_farfield(ctx, 0, np.full(360, 3 * np.pi / 4), phis, 2)[..., 0]
            Ta = -np.sin(np.pi / 4) * Fa  # [channel][phi1]
            Tb = -np.sin(3 * np.pi / 4) * Fb
            g2 = np.empty((360, 360))
            p2 = np.empty((360, 360))
            for i in range(360):
                for j in range(360):
                    T = (Ta[0, i], Ta[1, i], Tb[0, j], Tb[1, j])
                    g2[i, j] = V.hom_g2(T)[0]
                    p2[i, j] = V.hom_classical_p2(T)
            # (theta1, theta2) map at (phi1, phi2) = (0, 180 deg)
            ths = (np.arange(180) + 0.5) * np.pi / 180
            Fa2 = V.vie_farfield(ctx, 0, ths, np.zeros(180), 2)[..., 0] * -np.sin(ths)
            Fb2 = V.vie_farfield(ctx, 0, ths, np.full(180, np.pi), 2)[..., 0] * -np.sin(ths)
            g2t = np.array([[V.hom_g2((Fa2[0, i], Fa2[1, i], Fb2[0, j], Fb2[1, j]))[0]
                             for j in range(180)] for i in range(180)])
            tm = time.perf_counter() - t0
        finally:
            V.vie_destroy(ctx)
        # the (theta1, theta2) detectors see only solver-tolerance noise when the
        # channels' fields have no theta component in the xz plane (y-polarised
        # channels on a body symmetric under y -> -y): no physical g2 there
        bright = float(max(np.abs(Fa2).max(), np.abs(Fb2).max()) / np.abs(Ta).max())
        theta_map = ({"dark": True, "relative_brightness": bright} if bright < 10 * 1e-6 else
                     {"dark": False, "relative_brightness": bright, "g2_min": float(np.nanmin(g2t)),
                      "g2_max": float(np.nanmax(g2t))})
        flat = np.argsort(g2, axis=None)
        # single-path point: the pair where one path amplitude is smallest
        # relative to the other (|A_dir| = |T_a1 T_b2|, |A_ex| = |T_a2 T_b1|)
        ad = np.abs(Ta[0][:, None] * Tb[1][None, :])
        ae = np.abs(Ta[1][:, None] * Tb[0][None, :])
        single = int(np.argmin(np.minimum(ad, ae) / np.maximum(np.maximum(ad, ae), 1e-300)))
        picks = {"min": flat[0], "median": flat[len(flat) // 2], "max": flat[-1],
                 "single_path": single}
        dtau = np.linspace(-5, 5, 200)
        curves = {}
        for k, idx in picks.items():
            i, j = divmod(int(idx), 360)
            T = (Ta[0, i], Ta[1, i], Tb[0, j], Tb[1, j])
            _, _, nrm = V.hom_g2(T, 1.2, dtau, V.VIE_NORM_R2)
            curves[k] = {"phi1_deg": i, "phi2_deg": j, "g2": float(g2[i, j]),
                         "Nc_R2_near_0": float(nrm[int(np.argmin(np.abs(dtau)))]),
                         "Nc_R2_at_5sigma": float(nrm[-1])}
        out[label] = {"solve_s": ts, "iters": [x["iters"] for x in st],
                      "rel_res": [x["rel_res"] for x in st],
                      "sweep_64800_s": tf, "maps_s": tm,
                      "g2_min": float(np.nanmin(g2)), "g2_max": float(np.nanmax(g2)),
                      "theta_map": theta_map,
                      "p2_norm_min": float(np.nanmin(p2) / np.nanmax(p2)), "coincidence": curves}
        print(json.dumps({label: out[label]}), file=sys.stderr, flush=True)
    print(json.dumps(out))


def rooftop_mode(args):
    """The rooftop-basis operator (eq. Js_expand) on the paper's sphere (r = 1
    lambda, eps 4, 64^3, h = 2.05/64, padded grid 66^3, circulant 192^3): setup,
    per precision (FP64, and FP32 products inside FP64 refinement) --steps
    products of host vectors (PCIe copies included; the device time per
    product is in the kernel trace) and the two theta = +-30 deg channels
    solved to 1e-6 with BiCGSTAB, then a 180 x 360 far-field sweep per channel
    of the mixed solution."""
    import torch

    from paper_2508_16471_amd import vie as V
    from synth import Grid, sphere

    torch.cuda.set_device(0)
    V.lib()
    g = Grid.centred((64, 64, 64), 2.05 / 64)
    eps = sphere(g, 1.0, 4.0)
    a = np.deg2rad(30.0)
    chans = [((np.sin(a), 0, np.cos(a)), (0, 1.0, 0)), ((-np.sin(a), 0, np.cos(a)), (0, 1.0, 0))]
    t0 = time.perf_counter()
    rt = V.vie_rt_setup(eps, g.h, g.origin, K0)
    t_setup = time.perf_counter() - t0
    try:
        E, P = V.vie_rt_grid(rt)
        rng = np.random.default_rng(0)
        x = rng.standard_normal((3, E[2], E[1], E[0])) + 1j * rng.standard_normal((3, E[2], E[1], E[0]))
        prod_ms, solves = {}, {}
        for label, prec in (("fp64", V.VIE_FP64), ("mixed", V.VIE_MIXED)):
            V.vie_rt_matvec(rt, x, precision=prec)
            ts = []
            for _ in range(max(1, args.steps)):
                t0 = time.perf_counter()
                V.vie_rt_matvec(rt, x, precision=prec)
                ts.append(time.perf_counter() - t0)
            prod_ms[label] = 1e3 * float(np.median(ts))
            print(f"rooftop: {len(ts)} {label} products done", file=sys.stderr, flush=True)
            t0 = time.perf_counter()
            rc, w, st = V.vie_rt_solve(rt, chans, tol=1e-6, max_iter=8000, allow_noconv=True,
                                       precision=prec)
            solves[label] = {"solve_s": time.perf_counter() - t0, "status": int(rc),
                             "iters": [v["iters"] for v in st], "cycles": [v["cycles"] for v in st],
                             "matvecs": [v["matvecs"] for v in st],
                             "rel_res": [v["rel_res"] for v in st]}
            print(f"rooftop: {label} solve done", file=sys.stderr, flush=True)
        th = (np.arange(180) + 0.5) * np.pi / 180
        ph = np.arange(360) * 2 * np.pi / 360 - np.pi
        TH, PH = np.meshgrid(th, ph, indexing="ij")
        t0 = time.perf_counter()
        V.vie_rt_farfield(rt, w, TH.ravel(), PH.ravel())
        t_far = time.perf_counter() - t0
    finally:
        V.vie_rt_destroy(rt)
    M = P[0] * P[1] * P[2]
    out = {"mode": "rooftop", "workload": "rooftop basis, sphere r=1 lambda, eps 4, 64^3, "
           "h=2.05/64, channels theta=+-30 deg (y-pol)", "padded_grid": E, "circulant": P,
           "body_voxels": int((eps != 1.0).sum()), "setup_s": t_setup,
           "product_ms_host_vectors": prod_ms, "fp64": solves["fp64"], "mixed": solves["mixed"],
           "farfield_64800x2_s": t_far, "spectrum_bytes_fp64": 16 * M}
    print(json.dumps(out))


# ------------------------------------------------------------------ main
def precond_mode(args):
    """The paper's block preconditioner (7 x 7 lateral blocks, read as block
    Jacobi with k-step GMRES block solves) inside restarted FGMRES, against
    plain restarted GMRES and the mixed BiCGSTAB path, on the benchmark
    workload (--bodies bodies of --grid^3, --channels each), mixed precision,
    tol --tol; the best configurations also with the learned warm start.
    Each configuration is run once untimed (sub-problem setup, autotuning)
    and once timed."""
    if args.precond_body == "metasurface":
        from synth import circular_pol_basis, pb_metasurface, uv_directions

        g, eps = pb_metasurface()
        dirs = uv_directions()
        order = [27] + [i for i in range(len(dirs)) if i != 27]  # normal incidence first
        chans = []
        for i in order[:max(1, args.channels // 2)]:
            _, _, L, R = circular_pol_basis(dirs[i])
            chans += [(dirs[i], L), (dirs[i], R)]
        bodies = [(eps, g.h, g.origin, g)]
        nb, nch = 1, len(chans)
        workload = (f"PB metasurface 256x256x48, h = lambda/60, {nch} channels "
                    f"({nch // 2} directions x L/R), mixed precision")
    else:
        bodies, chans = make_workload(args.bodies, args.channels, args.grid)
        nb, nch = args.bodies, args.channels
        workload = (f"metasurface family {args.grid}^3, h = lambda/32, {nb} bodies x {nch} "
                    f"channels, mixed precision")
    import torch

    from paper_2508_16471_amd import vie as V

    torch.cuda.set_device(0)
    V.lib()
    wflag = 0 if args.no_window else V.VIE_FLAG_Z_WINDOW
    opt = V.make_options(K0, precision=V.VIE_MIXED, tol=args.tol, max_iter=20000,
                         inner_tol=args.inner_tol, flags=wflag)
    opt_warm = V.make_options(K0, precision=V.VIE_MIXED, tol=args.tol, max_iter=20000,
                              inner_tol=args.inner_tol, warm_start=1, flags=wflag)
    ctx = V.vie_setup([(e, h, o) for e, h, o, _ in bodies], opt)
    net = V.vie_cnn_create(0)
    V.vie_cnn_params(net, np.load(args.weights))
    configs = [("bicgstab_mixed", None, 0, 0), ("gmres30", V.fgmres_options(30, (0, 0)), 0, 0)]
    for m, bl, k in ((30, (7, 7), 2), (30, (7, 7), 4), (30, (8, 8), 2), (30, (8, 8), 4),
                     (30, (4, 4), 4), (30, (4, 4), 8), (30, (2, 2), 2), (30, (2, 2), 4),
                     (30, (2, 2), 8), (60, (2, 2), 8), (20, (2, 2), 8), (40, (2, 2), 8),
                     (30, (2, 2), 16), (30, (1, 1), 4), (60, (2, 2), 6), (60, (2, 2), 10),
                     (60, (3, 3), 8), (60, (2, 1), 8), (60, (1, 2), 8), (60, (3, 3), 12),
                     (40, (2, 2), 10), (30, (2, 2), 10), (60, (2, 2), 12)):
        configs.append((f"fgmres{m}_bj{bl[0]}x{bl[1]}_k{k}",
                        V.fgmres_options(m, bl, k, V.VIE_MIXED), k, 0))
    configs += [("bicgstab_mixed_learned", None, 0, 1),
                ("fgmres60_bj2x2_k8_learned", V.fgmres_options(60, (2, 2), 8, V.VIE_MIXED), 8, 1)]
    if args.configs:
        keep = set(args.configs.split(","))
        configs = [c for c in configs if c[0] in keep or c[0] == "bicgstab_mixed"]
    res = {}
    try:
        for name, fo, k, warm in configs:
            V.vie_set_options(ctx, opt_warm if warm else opt)
            V.vie_attach_cnn(ctx, net if warm else None)

            def run():
                if fo is None:
                    return V.vie_solve(ctx, chans, [nch] * nb, allow_noconv=True)[1]
                return V.vie_solve_fgmres(ctx, chans, [nch] * nb, fo, allow_noconv=True)[1]

            run()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = run()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            it = float(np.mean([s["iters"] for s in st]))
            r = {"solves_per_s": nb * nch / dt, "ms_per_solve": 1e3 * dt / (nb * nch),
                 "iterations": it, "operator_products": float(np.mean([s["matvecs"] for s in st])),
                 "block_products": it * k, "converged": all(s["converged"] for s in st),
                 "max_rel_res": max(s["rel_res"] for s in st)}
            if warm:
                r["initial_rel_res"] = float(np.mean([s["rel_res_x0"] for s in st]))
                r["fallbacks"] = int(sum(s["fallback"] for s in st))
            res[name] = r
            print(f"precond {name}: {r}", file=sys.stderr, flush=True)
    finally:
        V.vie_destroy(ctx)
        V.vie_cnn_destroy(net)
    base = res["bicgstab_mixed"]["solves_per_s"]
    print(json.dumps({"metric": "VIE solves/s at rel. residual %g" % args.tol,
                      "value": max(r["solves_per_s"] for r in res.values()), "unit": "solves/s",
                      "n_gpus": 1, "mode": "precond", "data": "synthetic",
                      "config": {"workload": workload},
                      "configs": res,
                      "speedup_vs_bicgstab": {k: v["solves_per_s"] / base for k, v in res.items()}}))


def main():
    args = parse()
    if args.mode in ("matvec", "farfield", "uneven", "metasurface", "sphere", "precond",
                     "paperscale", "cnn", "rooftop"):
        if args.gpus != 1:
            sys.exit(2)
        return {"matvec": matvec_mode, "farfield": farfield_mode, "uneven": uneven_mode,
                "metasurface": metasurface_mode, "sphere": sphere_mode,
                "precond": precond_mode, "paperscale": paperscale_mode,
                "cnn": cnn_mode, "rooftop": rooftop_mode}[args.mode](args)
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; the path shards by "
                          "right-hand side / body (see DESIGN.md), --gpus must be 1"}))
        sys.exit(2)
    bodies, chans = make_workload(args.bodies, args.channels, args.grid)
    cpu_t = c1 = None
    if not args.no_cpu:  # host oracle first, before this process touches the GPU
        cpu_t = cpu_product_time(bodies[0], args.cpu_seconds)
        c1 = cpu_c1_solve()
    import torch

    from paper_2508_16471_amd import vie as V

    torch.cuda.set_device(0)
    V.lib()
    N0 = bodies[0][3].n
    nb, nch = args.bodies, args.channels
    psi, theta, phi = detector_scan()
    dtau = np.linspace(-5, 5, 200)

    args.wflag = 0 if args.no_window else V.VIE_FLAG_Z_WINDOW
    # timed as shipped: graphs on, no timing events
    fast = V.make_options(K0, precision=V.VIE_MIXED, tol=args.tol, max_iter=20000,
                          inner_tol=args.inner_tol, flags=args.wflag)
    fast_timed = V.make_options(K0, precision=V.VIE_MIXED, tol=args.tol, max_iter=20000,
                                inner_tol=args.inner_tol, flags=V.VIE_FLAG_TIMING | args.wflag)
    t0 = time.perf_counter()
    ctx = V.vie_setup([(e, h, o) for e, h, o, _ in bodies], fast)
    setup_s = time.perf_counter() - t0
    N, P, _ = V.vie_grid(ctx, 0)  # the z window of the group (all bodies share it)
    Q = tuple(p // 2 + 1 for p in P)

    use_fgmres = args.solver in (None, "fgmres")
    blocks = tuple(int(v) for v in args.blocks.split(","))
    inner_prec = V.VIE_MIXED_BF16 if args.block_basis == "bf16" else V.VIE_MIXED
    fo = V.fgmres_options(args.restart, blocks, args.inner_iters, inner_prec)
    geom = block_geometry(bodies, blocks) if use_fgmres else None

    def solve():
        if use_fgmres:
            return V.vie_solve_fgmres(ctx, chans, [nch] * nb, fo)
        return V.vie_solve(ctx, chans, [nch] * nb)

    def step():
        rc, st = solve()
        post_process(V, ctx, nb, nch, theta, phi, dtau)
        return st

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    all_stats = []
    for _ in range(args.steps):
        all_stats += step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    solves = args.steps * nb * nch
    value = solves / dt
    # Per-kernel times: the same steps again with HIP events around every
    # launch on the library's stream (instrumented: graphs off, events between
    # launches); the kernels and their launches are the same as in the timed
    # region above.
    V.vie_set_options(ctx, fast_timed)
    step()
    V.vie_kernel_times(ctx, reset=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    inst_stats = []
    for _ in range(args.steps):
        inst_stats += step()
    torch.cuda.synchronize()
    dt_inst = time.perf_counter() - t1
    times = V.vie_kernel_times(ctx, reset=True)
    V.vie_set_options(ctx, fast)
    iters_match = [s["iters"] for s in inst_stats] == [s["iters"] for s in all_stats]
    nb_mean = float(np.mean([(e > 1).sum() for e, _, _, _ in bodies]))
    if use_fgmres:
        nrm_fused = (args.block_basis == "bf16"
                     and times.get("block_fft_xy_fwd_h16", (0.0, 0))[1] > 0)
        fast_rows = roofline_fgmres(times, inst_stats, N, P, Q, nb_mean, geom, args.inner_iters, nch,
                                    block_vin=4 if args.block_basis == "bf16" else 8,
                                    nrm_fused=nrm_fused)
    else:
        fast_rows = roofline_from_times(times, inst_stats, N, P, Q, mixed=True, nb=nb_mean)
    dom = max(fast_rows, key=lambda k: fast_rows[k]["ms_total"])
    d = fast_rows[dom]
    # the whole FP32 operator product of the body grid: its five passes'
    # algorithmic bytes over their summed kernel time in the timed region
    mv_keys = sorted(k for k in fast_rows if k.endswith("_f32") and not k.startswith("block_"))
    mv_rows = [fast_rows[k] for k in mv_keys]
    mv_bytes = sum(v["bytes"] for v in mv_rows)
    mv_ms = sum(v["ms_total"] for v in mv_rows)
    zrow = fast_rows.get("fft_z_green_f32", {"rhs_execs": 0})
    matvec = {"passes": mv_keys,
              "GBps": mv_bytes / (mv_ms * 1e-3) / 1e9 if mv_ms > 0 else None,
              "frac": mv_bytes / (mv_ms * 1e-3) / 1e9 / HBM_PEAK_GBS if mv_ms > 0 else None,
              "rhs_products": zrow["rhs_execs"],
              "rhs_products_per_s": zrow["rhs_execs"] / (mv_ms * 1e-3) if mv_ms > 0 else None}
    arn = None
    if use_fgmres and "arnoldi" in times:
        a_ms = times["arnoldi"][0]
        a_by = arnoldi_bytes(inst_stats, [int((e != 1.0).sum()) for e, _, _, _ in bodies], nch,
                             args.restart, args.inner_iters,
                             block_vb=4 if args.block_basis == "bf16" else 8,
                             block_nrm_fused=use_fgmres and nrm_fused)
        arn = {"ms_total": a_ms, "launches": int(times["arnoldi"][1]), "bytes": a_by,
               "GBps": a_by / (a_ms * 1e-3) / 1e9, "frac": a_by / (a_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
               "model": ("2 vb j + 3 vb + 32 bytes per element at Gram-Schmidt step j (FP32 w; "
                         "basis element vb = 8 B outer, " +
                         ("4 B (bfloat16)" if args.block_basis == "bf16" else "8 B") +
                         " in the block solves" +
                         ("; 2 vb j + 2 vb + 24 there, their normalisation being done by the "
                          "next packed product" if use_fgmres and nrm_fused else "") + ")")}
    conv = all(s["converged"] for s in all_stats)
    max_res = max(s["rel_res"] for s in all_stats)
    prod_fast = np.mean([s["matvecs"] for s in all_stats])

    plain = None
    if not args.no_plain:
        def plain_solves():
            ps = []
            for i in range(args.plain_solves):
                b, q = divmod(i % (nb * nch), nch)
                cnt = [0] * nb
                cnt[b] = 1
                _, st = V.vie_solve(ctx, [chans[b * nch + q]], cnt)
                ps += st
            return ps

        popt = dict(precision=V.VIE_FP64, tol=args.tol, max_iter=20000)
        V.vie_set_options(ctx, V.make_options(K0, flags=args.wflag, **popt))
        V.vie_solve(ctx, [chans[0]], [1] + [0] * (nb - 1))  # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ps = plain_solves()
        torch.cuda.synchronize()
        pdt = time.perf_counter() - t0
        # per-kernel times from an instrumented re-run of the same solves
        V.vie_set_options(ctx, V.make_options(K0, flags=V.VIE_FLAG_TIMING | args.wflag, **popt))
        V.vie_kernel_times(ctx, reset=True)
        ps_inst = plain_solves()
        ptimes = V.vie_kernel_times(ctx, reset=True)
        prow = roofline_from_times(ptimes, ps_inst, N, P, Q, mixed=False, nb=nb_mean)
        plain = {"solves_per_s": args.plain_solves / pdt,
                 "iters_mean": float(np.mean([s["iters"] for s in ps])),
                 "products_mean": float(np.mean([s["matvecs"] for s in ps])),
                 "max_rel_res": max(s["rel_res"] for s in ps),
                 "kernels": prow}
    learned = None
    if not args.no_learned and os.path.exists(args.weights):
        learned = learned_leg(V, torch, ctx, args, chans, nb, nch, theta, phi, dtau, value, solve)
    sweep = None
    if not args.no_sweep:
        sweep = farfield_sweep(V, torch, ctx, args, chans, nch, int((bodies[0][0] != 1.0).sum()))
    na = na_detection(V, torch, ctx, nch)
    V.vie_destroy(ctx)
    secondary = None if args.no_plain else sphere_leg(V, torch, args)
    probe = V.vie_hbm_probe(4 << 30, 10)  # achievable HBM on this device
    if args.calib_copy:
        calib_copy(torch)

    cpu = None
    if cpu_t is not None:
        prods = plain["products_mean"] if plain else prod_fast
        cpu = cpu_baseline(cpu_t[0], cpu_t[1], prods, c1)

    mt = measured_traffic(dom, d["avg_launch_ms"])
    line = {
        "metric": "VIE solves/s at rel. residual 1e-6 (128^3 grid), plain FP64 vs mixed+learned",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 FFT product / f64 Krylov",
        "data": "synthetic",
        "config": {"workload": (f"W128: {nb} held-out PB-phase fin-metasurface bodies (seed 55) on "
                                f"{N0[0]}x{N0[1]}x{N0[2]} voxels (computed on the {N[0]}x{N[1]}x{N[2]} "
                                f"z window that holds the bodies), h=lambda/32, FFT {P[0]}x{P[1]}x{P[2]}, "
                                f"{nch} channels each, true rel. residual <= {args.tol:g}, far field "
                                f"on a 181-point detector scan, circular g2 scan + 200-delay Nc"),
                   "bodies": nb, "channels_per_body": nch, "grid": list(N0), "window": list(N),
                   "fft": list(P),
                   "tol": args.tol, "precision": "mixed (FP32 product, FP64 refinement)",
                   "solver": ({"method": "FGMRES, block-Jacobi right preconditioner",
                               "restart": args.restart, "blocks": list(blocks),
                               "inner_gmres_steps": args.inner_iters,
                               "block_basis": args.block_basis,
                               "block_grid": list(geom["N"]), "block_fft": list(geom["P"]),
                               "blocks_per_body": geom["blocks_per_body"]}
                              if use_fgmres else {"method": "BiCGSTAB with FP64 refinement",
                                                  "inner_tol": args.inner_tol}),
                   "z_window": not args.no_window, "warm_start": False},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": d["GBps"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": d["GBps"] / HBM_PEAK_GBS,
                     "traffic": (mt or {}).get("bytes_per_launch"),
                     "traffic_detail": mt,
                     "algorithmic_bytes_per_launch": d["bytes"] / d["launches"],
                     "avg_launch_ms": d["avg_launch_ms"],
                     "timing": ("HIP events around every launch on the library's stream, over "
                                "an instrumented re-run of the timed steps (graphs off)"),
                     "instrumented_ms_per_step": dt_inst / args.steps * 1e3,
                     "instrumented_iters_match": iters_match,
                     "achievable_GBps": probe,
                     "frac_of_achievable_copy": d["GBps"] / probe["copy"]},
        "arnoldi": arn,
        "matvec": matvec,
        "cpu_baseline": cpu,
        "fast": {"converged": conv, "max_rel_res": max_res, "products_mean": float(prod_fast),
                 "iters_mean": float(np.mean([s["iters"] for s in all_stats])),
                 "block_products_mean": (float(np.mean([s["iters"] for s in all_stats]))
                                         * args.inner_iters if use_fgmres else 0.0),
                 "kernels": fast_rows},
        "other_kernels": other_rows(times),
        "plain_fp64": plain,
        "speedup_vs_plain": (value / plain["solves_per_s"]) if plain else None,
        "learned": learned,
        "farfield_sweep": sweep,
        "na_detection": na,
        "secondary_sphere": secondary,
        "setup_s": setup_s,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
