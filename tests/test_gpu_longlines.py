"""GPU parity of FFT lines longer than 512 points (x and y axes up to 6144 =
3 * 2^11, the lengths a paper-scale metasurface of Sec. III-B needs: 2480 x
744 voxels laterally).  Long lines run one workgroup per line (x) or a few
columns per workgroup (y) and read their twiddles from the global table.

* The operator product on thin rods whose circulant lengths hit every long
  length (768 ... 6144 along x; 1536 and 6144 along y) equals the oracle's
  direct O(N_b) sums on sampled rows: FP64 rel. 1e-12, FP32 5e-6;
* a mixed-precision solve on a 2480-voxel rod (compressed-vector passes,
  FP32 inside FP64 refinement, tol 1e-8) satisfies the oracle's system on
  sampled rows (operator rows 1e-12, residual 1e-5) and its far field equals
  the oracle's direct sum of the same current (1e-12).
"""

import numpy as np
import pytest

from oracle import vie_dense as vd
from synth import Grid

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


def _rod(rng, n, h):
    eps = 1.0 + rng.uniform(0.5, 4.0, size=(n[2], n[1], n[0]))
    eps[rng.random(eps.shape) < 0.15] = 1.0  # holes: ragged lines
    return eps


@pytest.mark.parametrize("n,P", [((300, 3, 2), 768), ((450, 2, 2), 1024), ((700, 2, 3), 1536),
                                 ((1000, 2, 2), 2048), ((1400, 2, 2), 3072),
                                 ((2000, 2, 2), 4096), ((2480, 2, 2), 6144),
                                 ((3, 700, 2), 1536), ((2, 2480, 2), 6144)])
def test_long_line_product_matches_oracle(V, n, P):
    rng = np.random.default_rng(n[0] * 7 + n[1])
    h = 0.02
    g = Grid.centred(n, h)
    eps = _rod(rng, n, h)
    chi = (eps - 1).ravel()
    pos = vd.voxel_centres(g.n, g.h, g.origin)
    x = rng.standard_normal((3,) + n[::-1]) + 1j * rng.standard_normal((3,) + n[::-1])
    body = np.nonzero(chi)[0]
    rows = np.unique(np.concatenate([rng.choice(body, 40, replace=False), body[[0, -1]],
                                     [0, chi.size - 1]]))
    ref = vd.matvec_rows(chi, pos, h, K0, x.reshape(3, -1), rows)
    ctx = V.vie_setup([(eps, h, g.origin)], V.make_options(K0))
    try:
        _, fft, _ = V.vie_grid(ctx, 0)
        assert max(fft[0], fft[1]) == P
        y64 = V.vie_matvec(ctx, 0, x, V.VIE_FP64).reshape(3, -1)[:, rows]
        y32 = V.vie_matvec(ctx, 0, x, V.VIE_MIXED).reshape(3, -1)[:, rows]
    finally:
        V.vie_destroy(ctx)
    e64, e32 = _relerr(y64, ref), _relerr(y32, ref)
    print(n, P, "fp64", e64, "fp32", e32)
    assert e64 < 1e-12
    assert e32 < 5e-6


def test_long_rod_mixed_solve_against_oracle(V):
    rng = np.random.default_rng(2480)
    n, h = (2480, 2, 2), 0.02
    g = Grid.centred(n, h)
    eps = _rod(rng, n, h)
    chi = (eps - 1).ravel()
    pos = vd.voxel_centres(g.n, g.h, g.origin)
    chans = [((0.0, 0.6, 0.8), (1.0, 0.0, 0.0)), ((0.8, 0.0, 0.6), (0.0, 1.0, 0.0))]
    body = np.nonzero(chi)[0]
    rows = np.unique(np.concatenate([rng.choice(body, 32, replace=False), body[[0, -1]]]))
    th = np.deg2rad(np.array([0.0, 15.0, 60.0, 90.0, 120.0, 179.0]))
    ph = np.deg2rad(np.array([0.0, 40.0, 100.0, 200.0, 280.0, 350.0]))
    ctx = V.vie_setup([(eps, h, g.origin)],
                      V.make_options(K0, precision=V.VIE_MIXED, tol=1e-8, max_iter=20000))
    try:
        rc, st = V.vie_solve(ctx, chans, [2])
        print("iterations", [s["iters"] for s in st], "rel res", [s["rel_res"] for s in st])
        assert rc == 0 and all(s["converged"] for s in st)
        ws = [V.vie_get_current(ctx, 0, q, g.n) for q in range(2)]
        y64 = [V.vie_matvec(ctx, 0, w, V.VIE_FP64).reshape(3, -1) for w in ws]
        F = V.vie_farfield(ctx, 0, th, ph, 2)
    finally:
        V.vie_destroy(ctx)
    for q, (k, p) in enumerate(chans):
        w = ws[q].reshape(3, -1)
        aw = vd.matvec_rows(chi, pos, h, K0, w, rows)
        b = vd.rhs(chi, pos, K0, k, p)[:, rows]
        e_op = _relerr(y64[q][:, rows], aw)
        e_res = float(np.linalg.norm(b - aw) / np.linalg.norm(b))
        ft, fp = vd.farfield(w, pos, h, K0, th, ph)
        e_ff = _relerr(F[q], np.stack([ft, fp], -1))
        print(q, "operator rows", e_op, "sampled residual", e_res, "far field", e_ff)
        assert e_op < 1e-12 and e_res < 1e-5 and e_ff < 1e-12
