"""Pins of the conv-net oracle: finite differences, a direct loop
definition of the convolution, and bf16 rounding properties."""

import numpy as np

from oracle import conv_ref as cr


def _net(rng, chans):
    return [(rng.standard_normal((27, co, ci)) * 0.3, rng.standard_normal(co) * 0.1)
            for ci, co in zip(chans[:-1], chans[1:])]


def test_conv3d_matches_direct_loops():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 4, 5, 2))
    W = rng.standard_normal((27, 3, 2))
    b = rng.standard_normal(3)
    y = cr.conv3d(x, W, b)
    Z, Y, X, _ = x.shape
    for (z, yy, xx) in [(0, 0, 0), (1, 2, 3), (2, 3, 4), (0, 3, 2)]:
        ref = b.copy()
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    t = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)
                    zz, y2, x2 = z + dz, yy + dy, xx + dx
                    if 0 <= zz < Z and 0 <= y2 < Y and 0 <= x2 < X:
                        ref += W[t] @ x[zz, y2, x2]
        assert np.allclose(y[z, yy, xx], ref, atol=1e-12)


def test_network_gradients_by_finite_differences():
    """2-layer, 4-channel net on 8^3: analytic gradients of the masked loss
    equal central differences (FP64, no rounding)."""
    rng = np.random.default_rng(1)
    params = _net(rng, [3, 4, 4])
    feat = rng.standard_normal((8, 8, 8, 3))
    target = rng.standard_normal((8, 8, 8, 4))
    mask = rng.random((8, 8, 8)) < 0.6

    def loss_of(p):
        out, _ = cr.forward(p, feat)
        return cr.masked_rel_l2(out, target, mask, 3)[0]

    out, acts = cr.forward(params, feat)
    loss, g = cr.masked_rel_l2(out, target, mask, 3)
    grads = cr.backward(params, acts, g)
    eps = 1e-6
    for li in range(2):
        W, b = params[li]
        for idx in [(0, 0, 0), (13, 1, 2), (26, 3, 1)]:
            if idx[2] >= W.shape[2] or idx[1] >= W.shape[1]:
                continue
            Wp, Wm = W.copy(), W.copy()
            Wp[idx] += eps
            Wm[idx] -= eps
            pp = [(Wp, b) if k == li else params[k] for k in range(2)]
            pm = [(Wm, b) if k == li else params[k] for k in range(2)]
            fd = (loss_of(pp) - loss_of(pm)) / (2 * eps)
            assert abs(fd - grads[li][0][idx]) < 1e-6 * max(1.0, abs(fd))
        bp, bm = b.copy(), b.copy()
        bp[1] += eps
        bm[1] -= eps
        fd = (loss_of([(W, bp) if k == li else params[k] for k in range(2)])
              - loss_of([(W, bm) if k == li else params[k] for k in range(2)])) / (2 * eps)
        assert abs(fd - grads[li][1][1]) < 1e-6 * max(1.0, abs(fd))


def test_bf16_rounding():
    v = np.array([1.0, 1.0 + 2**-8, 1.0 + 2**-7, 3.14159, -2.5e-3, 0.0])
    r = cr.bf16_round(v)
    assert r[0] == 1.0 and r[5] == 0.0
    assert r[1] == 1.0  # tie to even
    assert r[2] == 1.0 + 2**-7  # representable
    assert np.all(np.abs(r - v) <= np.abs(v) * 2**-8 + 1e-300)
