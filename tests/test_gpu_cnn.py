"""GPU parity of the learned warm start's network kernels (bf16 MFMA, fp32
accumulation) against the FP64 oracle on identical bf16-rounded tensors,
plus the warm-started solve."""

import numpy as np
import pytest

from oracle import conv_ref as cr
from oracle import vie_dense as vd
from synth import Grid, sphere

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


def _setup_net(V, rng):
    net = V.vie_cnn_create(7)
    p = V.vie_cnn_params(net).copy()
    p += rng.standard_normal(p.shape).astype(np.float32) * 0.02  # non-zero biases, dead channels
    V.vie_cnn_params(net, p)
    return net, p


def _oracle_params(V, p):
    return [(cr.bf16_round(W.astype(np.float64)), b.astype(np.float64)) for W, b in V.cnn_unpack(p)]


def _features(rng, d):
    f = np.zeros((d[2], d[1], d[0], 32))
    f[..., :25] = rng.standard_normal((d[2], d[1], d[0], 25))
    body = rng.random((d[2], d[1], d[0])) < 0.4
    f[..., 0] = np.where(body, rng.uniform(0.2, 1.5, body.shape), 0.0)
    return cr.bf16_round(f), body


@pytest.mark.parametrize("d", [(12, 10, 9), (8, 8, 4), (17, 5, 6)])
def test_network_forward_matches_oracle(env, d):
    V, torch = env
    rng = np.random.default_rng(sum(d))
    net, p = _setup_net(V, rng)
    try:
        feat, _ = _features(rng, d)
        ft = torch.tensor(feat, dtype=torch.float32).to(torch.bfloat16).cuda().contiguous()
        out = torch.zeros((d[2], d[1], d[0], 16), dtype=torch.float32, device="cuda")
        V.vie_cnn_infer_dev(net, d, ft.data_ptr(), out.data_ptr())
        torch.cuda.synchronize()
        ref, _ = cr.forward(_oracle_params(V, p), feat, round_bf16=True)
        err = _relerr(out.cpu().numpy(), ref)
        print(d, "forward rel err", err)
        assert err < 1e-3  # rel-L2 bar of the learned-part parity
    finally:
        V.vie_cnn_destroy(net)


def test_network_gradients_match_oracle(env):
    V, torch = env
    rng = np.random.default_rng(3)
    d = (12, 10, 9)
    net, p = _setup_net(V, rng)
    try:
        feat, body = _features(rng, d)
        tgt = rng.standard_normal((d[2], d[1], d[0], 6))
        ft = torch.tensor(feat, dtype=torch.float32).to(torch.bfloat16).cuda().contiguous()
        tt = torch.tensor(tgt, dtype=torch.float32).cuda().contiguous()
        loss, g = V.vie_cnn_grad_dev(net, d, ft.data_ptr(), tt.data_ptr())
        params = _oracle_params(V, p)
        out, acts = cr.forward(params, feat, round_bf16=True)
        rloss, gout = cr.masked_rel_l2(out, tgt, feat[..., 0] > 0, 6)
        grads = cr.backward(params, acts, gout, round_bf16=True)
        assert abs(loss - rloss) < 1e-3 * rloss
        for (gW, gb), (W_gpu, b_gpu) in zip(grads, V.cnn_unpack(g)):
            ew, eb = _relerr(W_gpu, gW), _relerr(b_gpu, gb)
            print("grad rel err W", ew, "b", eb)
            assert ew < 1e-3 and eb < 1e-3
    finally:
        V.vie_cnn_destroy(net)


def test_training_reduces_loss(env):
    V, torch = env
    rng = np.random.default_rng(4)
    d = (16, 16, 8)
    net, _ = _setup_net(V, rng)
    try:
        feat, _ = _features(rng, d)
        tgt = np.tanh(feat[..., 1:7]) * 0.5  # a learnable local map of the inputs
        ft = torch.tensor(feat, dtype=torch.float32).to(torch.bfloat16).cuda().contiguous()
        tt = torch.tensor(tgt, dtype=torch.float32).cuda().contiguous()
        losses = [V.vie_cnn_train_step_dev(net, d, ft.data_ptr(), tt.data_ptr(), 3e-3) for _ in range(60)]
        print("loss", losses[0], "->", losses[-1])
        assert losses[-1] < 0.5 * losses[0]
    finally:
        V.vie_cnn_destroy(net)


def test_sample_tensors_and_warm_started_solve(env):
    """Features / targets of a solved sphere equal their definitions; a
    warm-started solve (untrained network) still meets tol and matches LU."""
    V, torch = env
    g = Grid.centred(10, 0.06)
    eps = sphere(g, 0.25, 3.0)
    chans = [([0, 0, 1.0], [1, 0, 0]), ([0.6, 0, 0.8], [0, 1.0, 0])]
    ctx = V.vie_setup([(eps, g.h, g.origin)], V.make_options(K0, tol=1e-11, max_iter=3000))
    net = V.vie_cnn_create(11)
    try:
        V.vie_solve(ctx, chans, [2])
        w = V.vie_get_current(ctx, 0, 1, g.n)
        d = V.vie_cnn_sample_dev(ctx, 0, 1)
        ft = torch.zeros((d[2], d[1], d[0], 32), dtype=torch.bfloat16, device="cuda")
        tt = torch.zeros((d[2], d[1], d[0], 6), dtype=torch.float32, device="cuda")
        V.vie_cnn_sample_dev(ctx, 0, 1, ft.data_ptr(), tt.data_ptr())
        f = ft.float().cpu().numpy()
        t = tt.cpu().numpy()
        chi = eps - 1
        body = chi > 0
        zz, yy, xx = np.nonzero(body)
        lo = (xx.min() - 4 if xx.min() >= 4 else 0, yy.min() - 4 if yy.min() >= 4 else 0,
              zz.min() - 4 if zz.min() >= 4 else 0)
        pos = vd.voxel_centres(g.n, g.h, g.origin)
        b = vd.rhs(chi.ravel(), pos, K0, *chans[1]).reshape(3, *chi.shape)
        s = np.sqrt((np.abs(b) ** 2).sum() / body.sum())
        fb = f[zz - lo[2], yy - lo[1], xx - lo[0]]
        assert np.allclose(fb[:, 0], cr.bf16_round(chi[body] / 4), atol=1e-6)
        for c in range(3):
            assert np.allclose(fb[:, 1 + 2 * c], cr.bf16_round(b[c][body].real / s), atol=1e-2 * 4)
            tb = t[zz - lo[2], yy - lo[1], xx - lo[0]]
            assert np.allclose(tb[:, 2 * c] + 1j * tb[:, 2 * c + 1], w[c][body] / s, atol=1e-5)
        # warm-started solve
        V.vie_attach_cnn(ctx, net)
        V.vie_set_options(ctx, V.make_options(K0, tol=1e-11, max_iter=3000, warm_start=1))
        rc, st = V.vie_solve(ctx, chans, [2])
        for q, (k, p) in enumerate(chans):
            assert st[q]["warm"] == 1 and st[q]["converged"] == 1
            w_lu = vd.solve_lu(chi.ravel(), pos, g.h, K0, k, p)
            w_gpu = V.vie_get_current(ctx, 0, q, g.n).reshape(3, -1)
            assert _relerr(w_gpu, w_lu) < 1e-8
        print("warm stats", st)
    finally:
        V.vie_destroy(ctx)
        V.vie_cnn_destroy(net)


def test_checkpoint_resume_is_exact(env, tmp_path):
    """Training interrupted after 2 of 4 epochs and resumed from its checkpoint
    (parameters, Adam moments and step, shuffling state) ends bit for bit where
    the uninterrupted run does; the Adam state round-trips through the ABI."""
    V, torch = env
    from paper_2508_16471_amd.train_warmstart import train

    rng = np.random.default_rng(8)
    d = (16, 16, 8)
    samples = []
    for _ in range(3):
        feat, _ = _features(rng, d)
        tgt = np.tanh(feat[..., 1:7]) * 0.5
        samples.append((d, torch.tensor(feat, dtype=torch.float32).to(torch.bfloat16).cuda().contiguous(),
                        torch.tensor(tgt, dtype=torch.float32).cuda().contiguous()))
    nets = []
    try:
        a, ha, _ = train(V, torch, samples, 4, 3e-3, 3)
        nets.append(a)
        ck = str(tmp_path / "ck.npz")
        b0, _, _ = train(V, torch, samples, 4, 3e-3, 3, checkpoint=ck, stop_after=2)
        nets.append(b0)
        b, hb, _ = train(V, torch, samples, 4, 3e-3, 3, resume=ck)
        nets.append(b)
        assert np.array_equal(V.vie_cnn_params(a), V.vie_cnn_params(b))
        ma, va, sa = V.vie_cnn_adam_state(a)
        mb, vb, sb = V.vie_cnn_adam_state(b)
        assert sa == sb == 12 and np.array_equal(ma, mb) and np.array_equal(va, vb)
        assert ha == hb
        with pytest.raises(V.VieError):
            V.vie_cnn_adam_state(b, (ma, -np.abs(va) - 1, sa))
    finally:
        for n in nets:
            V.vie_cnn_destroy(n)
