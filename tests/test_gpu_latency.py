"""Completion times of batched solves (`vie_stats.seconds`).

Each converged right-hand side reports the device wall-clock time from the
start of the call's device work to the FP64 true-residual check that first
found it converged (groups solved earlier in the same call included).  This
is a measurement, not a parity quantity, so the checks are consistency ones:
every converged right-hand side has 0 < seconds <= the call's host wall time,
the last one to finish comes close to that wall time, and a right-hand side
that is stopped before convergence reports 0.
"""

import time

import numpy as np
import pytest

from synth import Grid, sphere

pytestmark = pytest.mark.gpu
K0 = 2 * np.pi
CHANS = [((0.0, 0.0, 1.0), (1.0, 0.0, 0.0)), ((0.0, 0.6, 0.8), (1.0, 0.0, 0.0))]


@pytest.fixture(scope="module")
def V():
    import torch

    assert torch.cuda.is_available()
    from paper_2508_16471_amd import vie

    vie.lib()
    return vie


def _bodies():
    # two bodies on one grid (one batched group, different contrast) and one
    # on another grid (a second group, solved after the first)
    g16, g20 = Grid.centred(16, 1.0 / 16), Grid.centred(20, 1.0 / 16)
    return [(sphere(g16, 0.4, 2.25), g16.h, g16.origin), (sphere(g16, 0.4, 6.0), g16.h, g16.origin),
            (sphere(g20, 0.5, 3.0), g20.h, g20.origin)]


@pytest.mark.parametrize("solver", ["bicgstab", "fgmres"])
def test_completion_seconds(V, solver):
    ctx = V.vie_setup(_bodies(), V.make_options(K0, precision=V.VIE_MIXED, tol=1e-7,
                                                max_iter=5000))
    chans, nr = CHANS * 3, [2, 2, 2]

    def solve():
        if solver == "fgmres":
            return V.vie_solve_fgmres(ctx, chans, nr, V.fgmres_options(30, (2, 2), 4))
        return V.vie_solve(ctx, chans, nr)

    try:
        solve()  # tuning and graph capture
        t = time.perf_counter()
        rc, st = solve()
        wall = time.perf_counter() - t
    finally:
        V.vie_destroy(ctx)
    sec = np.array([s["seconds"] for s in st])
    print(solver, "wall", wall, "seconds", sec, "iters", [s["iters"] for s in st])
    assert rc == 0 and all(s["converged"] for s in st)
    assert np.all(sec > 0) and np.all(sec <= wall)
    assert sec.max() >= 0.5 * wall


def test_not_converged_reports_zero(V):
    ctx = V.vie_setup(_bodies()[:2], V.make_options(K0, precision=V.VIE_FP64, tol=1e-12,
                                                    max_iter=2))
    try:
        rc, st = V.vie_solve(ctx, CHANS * 2, [2, 2], allow_noconv=True)
    finally:
        V.vie_destroy(ctx)
    assert rc == V.VIE_ENOCONV
    assert all(not s["converged"] and s["seconds"] == 0.0 for s in st)
