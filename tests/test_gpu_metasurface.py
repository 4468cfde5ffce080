"""The benchmark Pancharatnam-Berry metasurface at full size: 256 x 256 x 48
voxels of lambda/60 (FFT 512 x 512 x 96, 1.28 M body voxels), 8 x 8 fins of
eps 5.8 on an eps 2.1 slab.  Four channels (normal incidence and
(u, v) = (0.4, -0.3), each with both circular polarisations) are solved in
one batched call with the FP32 product inside FP64 refinement to rel.
residual 1e-6, then checked against the oracle on sampled rows:

* the library's FP64 product at the solved current equals the oracle's
  direct O(N_b) row sums (rel. 1e-12), so the residual the library reports
  is the residual of the oracle's system;
* the oracle's own sampled residual b - A w is small against b on those
  rows (a loose 1e-4 bound: the 1e-6 bound holds for the global norm, not
  row by row);
* the far field of every channel matches the oracle's direct sum on sampled
  directions (rel. 1e-12, the same current on both sides).
"""

import numpy as np
import pytest

from oracle import vie_dense as vd
from synth import circular_pol_basis, pb_metasurface, uv_directions

pytestmark = pytest.mark.gpu
K0 = 2 * np.pi


def _relerr(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def test_metasurface_256x256x48_batched_solve_matches_oracle_rows():
    import torch

    assert torch.cuda.is_available()
    from paper_2508_16471_amd import vie as V

    g, eps = pb_metasurface()
    chans = []
    for k in uv_directions()[[27, 7]]:
        _, _, L, R = circular_pol_basis(k)
        chans += [(k, L), (k, R)]
    chi = (eps - 1.0).ravel()
    body = np.nonzero(chi)[0]
    rng = np.random.default_rng(256)
    sel = np.concatenate([rng.choice(body, 20, replace=False), [0, len(chi) - 1, body[0], body[-1]]])
    pos = vd.voxel_centres(g.n, g.h, g.origin)
    ctx = V.vie_setup([(eps, g.h, g.origin)],
                      V.make_options(K0, precision=V.VIE_MIXED, tol=1e-6, max_iter=20000))
    try:
        rc, st = V.vie_solve(ctx, chans, [len(chans)])
        print("iterations", [s["iters"] for s in st], "rel res", [s["rel_res"] for s in st])
        assert rc == 0 and all(s["converged"] and s["rel_res"] <= 1e-6 for s in st)
        ws = [V.vie_get_current(ctx, 0, q, g.n) for q in range(len(chans))]
        y64 = [V.vie_matvec(ctx, 0, w, V.VIE_FP64).reshape(3, -1) for w in ws]
        th = np.deg2rad(np.array([0.0, 11.0, 37.0, 90.0, 143.0, 180.0]))
        ph = np.deg2rad(np.array([0.0, 90.0, 200.0, 45.0, 310.0, 0.0]))
        F = V.vie_farfield(ctx, 0, th, ph, len(chans))
    finally:
        V.vie_destroy(ctx)
    for q, (k, p) in enumerate(chans):
        w = ws[q].reshape(3, -1)
        aw = vd.matvec_rows(chi, pos, g.h, K0, w, sel)
        e_op = _relerr(y64[q][:, sel], aw)
        b = vd.rhs(chi, pos, K0, k, p)[:, sel]
        e_res = float(np.linalg.norm(b - aw) / np.linalg.norm(b))
        ft, fp = vd.farfield(w, pos, g.h, K0, th, ph)
        e_ff = _relerr(F[q], np.stack([ft, fp], -1))
        print(q, "operator rows", e_op, "sampled residual", e_res, "far field", e_ff)
        assert e_op < 1e-12
        assert e_res < 1e-4
        assert e_ff < 1e-12
