"""What the trained warm-start network gains over the plain start.

Held-out bodies of its training family (seed 55: 128^3 PB-phase fin
metasurfaces, h = lambda/32), 4 bodies x 2 channels, mixed path, tol 1e-6.
The committed weights are loaded and both starts solve the same right-hand
sides.  The test prints the initial residual, iterations and fallback rate
of each, and asserts what the network does deliver: its guesses are
accepted (no fallback to w = 0), they cut the initial residual below 0.7
against 1 for the plain start, and both solves meet the tolerance with the
FP64 residual.  It also bounds the cost: at most 10 % more iterations than
the plain start.  It claims no iteration saving; the measured ratio is about
1.0, because the slow modes of these bodies are global resonances that a
9^3 receptive field cannot represent.
"""

import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
K0 = 2 * np.pi
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "paper_2508_16471_amd", "weights", "warmstart_metasurface128.npy")


def test_trained_warm_start_against_plain_start():
    import torch

    assert torch.cuda.is_available()
    from paper_2508_16471_amd import vie as V
    from synth import metasurface_family, random_planewave

    rng = np.random.default_rng(55)
    bodies, chans = [], []
    for _ in range(4):
        g, eps = metasurface_family(rng, 128, 1.0 / 32)
        bodies.append((eps, g.h, g.origin))
        for _ in range(2):
            chans.append(random_planewave(rng, cap_deg=20.0, elliptical=True))
    res = {}
    net = V.vie_cnn_create(0)
    try:
        V.vie_cnn_params(net, np.load(WEIGHTS))
        for name, warm in (("plain", 0), ("warm", 1)):
            ctx = V.vie_setup(bodies, V.make_options(K0, precision=V.VIE_MIXED, tol=1e-6,
                                                     max_iter=20000, warm_start=warm))
            try:
                if warm:
                    V.vie_attach_cnn(ctx, net)
                rc, st = V.vie_solve(ctx, chans, [2] * 4)
            finally:
                V.vie_destroy(ctx)
            assert rc == 0 and all(s["converged"] and s["rel_res"] <= 1e-6 for s in st)
            res[name] = st
    finally:
        V.vie_cnn_destroy(net)
    it_p = np.mean([s["iters"] for s in res["plain"]])
    it_w = np.mean([s["iters"] for s in res["warm"]])
    x0 = np.mean([s["rel_res_x0"] for s in res["warm"]])
    fb = np.mean([s["fallback"] for s in res["warm"]])
    print(f"plain iterations {it_p:.1f}, warm iterations {it_w:.1f} (ratio {it_w / it_p:.3f}), "
          f"initial residual {x0:.3f}, fallback rate {fb:.2f}")
    assert fb == 0.0
    assert all(s["warm"] == 1 for s in res["warm"])
    assert x0 < 0.7
    assert it_w <= 1.1 * it_p


def test_trained_warm_start_inside_preconditioned_fgmres():
    """The same held-out bodies and channels through the block-preconditioned
    FGMRES path (2 x 2 blocks, 8 block steps) with and without the network's
    start: every guess is accepted, both starts meet the tolerance, and the
    warm start takes at most as many Arnoldi steps (plus one cycle's slack)."""
    import torch

    assert torch.cuda.is_available()
    from paper_2508_16471_amd import vie as V
    from synth import metasurface_family, random_planewave

    rng = np.random.default_rng(55)
    bodies, chans = [], []
    for _ in range(4):
        g, eps = metasurface_family(rng, 128, 1.0 / 32)
        bodies.append((eps, g.h, g.origin))
        for _ in range(2):
            chans.append(random_planewave(rng, cap_deg=20.0, elliptical=True))
    fo = V.fgmres_options(60, (2, 2), 8, V.VIE_MIXED)
    res = {}
    net = V.vie_cnn_create(0)
    try:
        V.vie_cnn_params(net, np.load(WEIGHTS))
        for name, warm in (("plain", 0), ("warm", 1)):
            ctx = V.vie_setup(bodies, V.make_options(K0, precision=V.VIE_MIXED, tol=1e-6,
                                                     max_iter=20000, warm_start=warm))
            try:
                if warm:
                    V.vie_attach_cnn(ctx, net)
                rc, st = V.vie_solve_fgmres(ctx, chans, [2] * 4, fo)
            finally:
                V.vie_destroy(ctx)
            assert rc == 0 and all(s["converged"] and s["rel_res"] <= 1e-6 for s in st)
            res[name] = st
    finally:
        V.vie_cnn_destroy(net)
    it_p = np.mean([s["iters"] for s in res["plain"]])
    it_w = np.mean([s["iters"] for s in res["warm"]])
    print(f"FGMRES steps: plain {it_p:.1f}, warm {it_w:.1f}; initial residual "
          f"{np.mean([s['rel_res_x0'] for s in res['warm']]):.3f}")
    assert all(s["warm"] == 1 and s["fallback"] == 0 for s in res["warm"])
    assert it_w <= it_p + 8
