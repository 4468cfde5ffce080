"""Oracle checks of full-size solves that no dense LU can reach: the 64^3
sphere (radius 1 lambda, eps 4, 137,376 body voxels; channels at +-30 deg,
the sphere study of Sec. III-A) on the FP64 and mixed paths, and one body
of the 128^3 benchmark family (PB fin metasurface, Sec. III-B) solved by the
benchmark's fast path (mixed block-Jacobi FGMRES on the z window).

For every solved current w the oracle computes, independently of the
library's FFT product:

* its direct O(N_b) operator rows (A w) on sampled body voxels; the library's
  FP64 product at w must equal them (rel. 1e-12), so the residual the library
  reports is that of the oracle's system;
* the sampled residual b - A w on those rows against b (rows are a sample,
  so the bound is a loose multiple of the solver's global tolerance);
* the far field of w by its direct sum on sampled directions (rel. 1e-12,
  the same current on both sides).

Mixed against FP64 (the error of the mixed path, stated per result): the far
field of the mixed solve is compared with that of an FP64 solve of the same
system to rel. residual 1e-10.  At the parity tolerance (mixed refinement to
1e-9) it must agree to the 1e-6 rel-L2 bar; at the benchmark tolerance
(1e-6) the error is printed and bounded by 1e-4.
"""

import numpy as np
import pytest

from oracle import vie_dense as vd
from synth import Grid, metasurface_family, random_planewave, sphere

pytestmark = pytest.mark.gpu
K0 = 2 * np.pi


@pytest.fixture(scope="module")
def V():
    import torch

    assert torch.cuda.is_available()
    from paper_2508_16471_amd import vie

    vie.lib()
    return vie


def _relerr(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def _oracle_checks(V, ctx, g, eps, chans, rows, th, ph, res_bar, tag):
    """Checks of every channel's current against the oracle; returns the far
    fields [nch][ndir][2]."""
    chi = (eps - 1.0).ravel()
    pos = vd.voxel_centres(g.n, g.h, g.origin)
    F = V.vie_farfield(ctx, 0, th, ph, len(chans))
    for q, (k, p) in enumerate(chans):
        w = V.vie_get_current(ctx, 0, q, g.n)
        y64 = V.vie_matvec(ctx, 0, w, V.VIE_FP64).reshape(3, -1)
        w = w.reshape(3, -1)
        aw = vd.matvec_rows(chi, pos, g.h, K0, w, rows)
        b = vd.rhs(chi, pos, K0, k, p)[:, rows]
        e_op = _relerr(y64[:, rows], aw)
        e_res = float(np.linalg.norm(b - aw) / np.linalg.norm(b))
        ft, fp = vd.farfield(w, pos, g.h, K0, th, ph)
        e_ff = _relerr(F[q], np.stack([ft, fp], -1))
        print(tag, q, "operator rows", e_op, "sampled residual", e_res, "far field", e_ff)
        assert e_op < 1e-12
        assert e_res < res_bar
        assert e_ff < 1e-12
    return F


def _rows(eps, rng, count=24):
    body = np.nonzero((eps != 1.0).ravel())[0]
    return np.unique(np.concatenate([rng.choice(body, count, replace=False), body[[0, -1]]]))


def _directions(rng, n=24):
    th = np.concatenate([[0.0, np.pi], rng.uniform(0, np.pi, n - 2)])
    ph = rng.uniform(0, 2 * np.pi, n)
    return th, ph


def test_c2_sphere_fp64_and_mixed_against_oracle(V):
    g = Grid.centred((64, 64, 64), 2.05 / 64)
    eps = sphere(g, 1.0, 4.0)
    a = np.deg2rad(30)
    chans = [((np.sin(a), 0, np.cos(a)), (0, 1.0, 0)), ((-np.sin(a), 0, np.cos(a)), (0, 1.0, 0))]
    rng = np.random.default_rng(642)
    rows = _rows(eps, rng)
    th, ph = _directions(rng)
    F = {}
    for name, prec, tol in (("fp64", V.VIE_FP64, 1e-10), ("mixed_parity", V.VIE_MIXED, 1e-9),
                            ("mixed_bench", V.VIE_MIXED, 1e-6)):
        ctx = V.vie_setup([(eps, g.h, g.origin)],
                          V.make_options(K0, precision=prec, tol=tol, max_iter=20000))
        try:
            rc, st = V.vie_solve(ctx, chans, [2])
            print(name, [s["iters"] for s in st], [s["rel_res"] for s in st])
            assert rc == 0 and all(s["converged"] and s["rel_res"] <= tol for s in st)
            F[name] = _oracle_checks(V, ctx, g, eps, chans, rows, th, ph, 1e3 * tol, name)
        finally:
            V.vie_destroy(ctx)
    for q in range(2):
        e_par = _relerr(F["mixed_parity"][q], F["fp64"][q])
        e_bench = _relerr(F["mixed_bench"][q], F["fp64"][q])
        print("C2 channel", q, "mixed vs FP64 far field: parity tol", e_par, "bench tol", e_bench)
        assert e_par < 1e-6
        assert e_bench < 1e-4


def test_w128_bench_body_fast_path_against_oracle(V):
    rng = np.random.default_rng(55)  # the benchmark's held-out seed: its first body
    g, eps = metasurface_family(rng, 128, 1.0 / 32)
    chans = [random_planewave(rng, cap_deg=20.0, elliptical=True) for _ in range(2)]
    rrng = np.random.default_rng(1280)
    rows = _rows(eps, rrng)
    th, ph = _directions(rrng)
    fo = V.fgmres_options(60, (2, 2), 8, V.VIE_MIXED)
    F = {}
    for name, prec, tol in (("fp64", V.VIE_FP64, 1e-10), ("mixed_parity", V.VIE_MIXED, 1e-9),
                            ("mixed_bench", V.VIE_MIXED, 1e-6)):
        opt = V.make_options(K0, precision=prec, tol=tol, max_iter=20000,
                             flags=V.VIE_FLAG_Z_WINDOW)
        ctx = V.vie_setup([(eps, g.h, g.origin)], opt)
        try:
            if name == "fp64":
                rc, st = V.vie_solve(ctx, chans, [2])
            else:
                rc, st = V.vie_solve_fgmres(ctx, chans, [2], fo)
            print(name, [s["iters"] for s in st], [s["rel_res"] for s in st])
            assert rc == 0 and all(s["converged"] and s["rel_res"] <= tol for s in st)
            F[name] = _oracle_checks(V, ctx, g, eps, chans, rows, th, ph, 1e3 * tol, name)
        finally:
            V.vie_destroy(ctx)
    for q in range(2):
        e_par = _relerr(F["mixed_parity"][q], F["fp64"][q])
        e_bench = _relerr(F["mixed_bench"][q], F["fp64"][q])
        print("W128 channel", q, "mixed vs FP64 far field: parity tol", e_par, "bench tol", e_bench)
        assert e_par < 1e-6
        assert e_bench < 1e-4
