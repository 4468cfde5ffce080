"""The allocation-free operator product (vie_matvec_dev_static) against the
existing device-pointer product (vie_matvec_dev) and the oracle's dense
product, through the C ABI:

* two calls in a row, the second with a smaller input (a smaller grid and
  fewer vectors), each equal to vie_matvec_dev (FP64 rel. 1e-12, FP32 5e-6;
  bit for bit once both use the z-pass shape the context tuned) and to the
  oracle on every row;
* a body computed on its z window (box vectors pass through outside it);
* a request beyond the static scratch is refused with VIE_ENOTSUP and
  leaves the output untouched.
"""

import numpy as np
import pytest

from oracle import vie_dense as vd
from synth import Grid, random_ellipsoid_body

pytestmark = pytest.mark.gpu
K0 = 2 * np.pi


@pytest.fixture(scope="module")
def env():
    import torch

    assert torch.cuda.is_available()
    from paper_2508_16471_amd import vie

    vie.lib()
    return vie, torch


def _relerr(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.float64)).cuda()


def _host(t, shape):
    return t.cpu().numpy().view(np.complex128).reshape(shape)


def _products(V, torch, ctx, x, prec):
    """(static product, existing product, static product again) of x."""
    shape = x.shape
    xd = _dev(torch, x)
    ys, yd, ys2 = (torch.full_like(xd, np.nan) for _ in range(3))
    V.vie_matvec_dev_static(ctx, 0, xd.data_ptr(), ys.data_ptr(), shape[0], prec)
    V.vie_matvec_dev(ctx, 0, xd.data_ptr(), yd.data_ptr(), shape[0], prec)
    V.vie_matvec_dev_static(ctx, 0, xd.data_ptr(), ys2.data_ptr(), shape[0], prec)
    torch.cuda.synchronize()
    return _host(ys, shape), _host(yd, shape), _host(ys2, shape)


@pytest.mark.parametrize("prec,bar", [(0, 1e-12), (1, 5e-6)])
def test_static_product_two_calls_second_smaller(env, prec, bar):
    V, torch = env
    rng = np.random.default_rng(31 + prec)
    cases = [(Grid.centred((20, 17, 24), 0.06), 3), (Grid.centred((9, 8, 7), 0.09), 1)]
    for g, nvec in cases:  # the second call has the smaller input
        eps = random_ellipsoid_body(rng, g, kmax=3, axis_range=(0.2, 0.5))
        chi = (eps - 1).ravel()
        pos = vd.voxel_centres(g.n, g.h, g.origin)
        shape = (nvec, 3) + g.n[::-1]
        x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
        ctx = V.vie_setup([(eps, g.h, g.origin)], V.make_options(K0))
        try:
            ys, yd, ys2 = _products(V, torch, ctx, x, prec)
        finally:
            V.vie_destroy(ctx)
        for q in range(nvec):
            ref = vd.matvec(chi, pos, g.h, K0, x[q].reshape(3, -1)).reshape(x[q].shape)
            e_s, e_d = _relerr(ys[q], ref), _relerr(yd[q], ref)
            print(g.n, nvec, prec, q, "static vs oracle", e_s, "existing vs oracle", e_d)
            assert e_s < bar and e_d < bar
        assert _relerr(ys, yd) < bar
        assert np.array_equal(ys2, yd)  # same kernels and z shape: bit for bit


def test_static_product_on_z_window(env):
    V, torch = env
    rng = np.random.default_rng(33)
    n = (14, 12, 40)
    g = Grid.centred(n, 0.06)
    eps = np.ones(n[::-1])
    eps[15:21, 2:12, 1:13] = 2.2
    eps[21:23, 4:9, 3:10] = 4.5
    x = rng.standard_normal((2, 3) + n[::-1]) + 1j * rng.standard_normal((2, 3) + n[::-1])
    ctx = V.vie_setup([(eps, g.h, g.origin)], V.make_options(K0, flags=V.VIE_FLAG_Z_WINDOW))
    try:
        assert V.vie_grid(ctx, 0)[0][2] < n[2]
        ys, yd, ys2 = _products(V, torch, ctx, x, 0)
    finally:
        V.vie_destroy(ctx)
    assert _relerr(ys, yd) < 1e-12
    assert np.array_equal(ys2, yd)
    out = np.ones(n[2], bool)
    out[11:27] = False  # window layers: body layers 15..22 plus 4 on each side
    assert np.array_equal(ys[:, :, out], x[:, :, out])


def test_static_product_refuses_oversize(env):
    V, torch = env
    g = Grid.centred((64, 64, 64), 0.03)
    eps = np.ones(g.n[::-1])
    eps[20:40, 20:40, 20:40] = 2.0
    nvec = 8  # FP64 work arrays of 8 vectors on a 128^3 circulant: > 256 MiB
    x = torch.zeros((nvec, 3) + g.n[::-1] + (2,), dtype=torch.float64, device="cuda")
    y = torch.full_like(x, 7.0)
    ctx = V.vie_setup([(eps, g.h, g.origin)], V.make_options(K0))
    try:
        with pytest.raises(V.VieError) as e:
            V.vie_matvec_dev_static(ctx, 0, x.data_ptr(), y.data_ptr(), nvec, V.VIE_FP64)
        assert e.value.code == V.VIE_ENOTSUP
        torch.cuda.synchronize()
        assert bool((y == 7.0).all())
    finally:
        V.vie_destroy(ctx)
