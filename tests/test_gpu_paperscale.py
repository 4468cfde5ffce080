"""The paper's full-wave metasurface (Sec. III-B) at its stated size on one
GPU: a 40 x 12 x 2 wavelength box at 62 cells per wavelength (2480 x 744 x
124 voxels), 91 x 27 silicon nanofins with the PB rotation of eq. 32 on a
glass substrate: 17.5 M body voxels, 52.5 M unknowns (the paper: 18.0 M
elements, 54.0 M unknowns).  The context computes on the z window that holds
the body (2480 x 744 x 35, FFT 6144 x 1536 x 96: x lines of 6144 = 3 * 2^11
points).  The operator product of a random body-supported vector, FP64 and
FP32 on the device, equals the oracle's direct O(N_b) sums on sampled rows
(rel. 1e-12 / 5e-6).  Setup time and device memory are printed.
"""

import time

import numpy as np
import pytest

from oracle import vie_dense as vd
from synth import paper_metasurface

pytestmark = pytest.mark.gpu
K0 = 2 * np.pi


def _relerr(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def test_paper_scale_metasurface_product_against_oracle():
    import torch

    assert torch.cuda.is_available()
    from paper_2508_16471_amd import vie as V

    V.lib()
    g, eps = paper_metasurface()
    chi = (eps - 1.0).ravel()
    body = np.nonzero(chi)[0]
    print("body voxels", body.size, "unknowns", 3 * body.size)
    rng = np.random.default_rng(2480744)
    xb = rng.standard_normal((3, body.size)) + 1j * rng.standard_normal((3, body.size))
    rows = np.unique(np.concatenate([rng.choice(body.size, 14, replace=False), [0, body.size - 1]]))
    free0 = torch.cuda.mem_get_info()[0]
    t0 = time.perf_counter()
    ctx = V.vie_setup([(eps, g.h, g.origin)], V.make_options(K0, flags=V.VIE_FLAG_Z_WINDOW))
    try:
        t_setup = time.perf_counter() - t0
        win, fft, _ = V.vie_grid(ctx, 0)
        assert fft[0] == 6144 and fft[1] == 1536
        bd = torch.from_numpy(body).cuda()
        x = torch.zeros((3, chi.size), dtype=torch.complex128, device="cuda")
        x[:, bd] = torch.from_numpy(xb).cuda()
        y = torch.empty_like(x)
        out = {}
        for prec in (V.VIE_FP64, V.VIE_MIXED):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            V.vie_matvec_dev(ctx, 0, x.data_ptr(), y.data_ptr(), 1, prec)
            torch.cuda.synchronize()
            out[prec] = (y[:, bd[rows]].cpu().numpy(), time.perf_counter() - t1)
        used = (free0 - torch.cuda.mem_get_info()[0]) / 2**30
        print("window", win, "fft", fft, "setup s", round(t_setup, 2), "device GiB", round(used, 1),
              "product s (fp64, fp32)", round(out[0][1], 3), round(out[1][1], 3))
    finally:
        V.vie_destroy(ctx)
    pos = vd.voxel_centres(g.n, g.h, g.origin)[body]
    ref = vd.matvec_rows(chi[body], pos, g.h, K0, xb, rows)
    e64, e32 = _relerr(out[0][0], ref), _relerr(out[1][0], ref)
    print("paper-scale product rows: fp64", e64, "fp32", e32)
    assert e64 < 1e-12
    assert e32 < 5e-6
