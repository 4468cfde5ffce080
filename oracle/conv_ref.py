"""Plain FP64 3-D convolutional network (test infrastructure only).

Reference for the learned warm start of the Krylov solve: a stack of 3x3x3
"same" convolutions (zero padding) with bias and ReLU between layers, the
masked relative-L2 loss, and the exact backward pass, written as 27 shifted
tensor contractions.  Tensors are channels-last (D2, D1, D0, C); weights
are (27, Cout, Cin) with tap index t = (dz+1)*9 + (dy+1)*3 + (dx+1), so that
out[z,y,x,o] = b[o] + sum_t sum_i W[t,o,i] in[z+dz, y+dy, x+dx, i].

Optional rounding to bfloat16 (round to nearest even on the fp32 value) at
the points where the GPU path stores bf16 lets tests compare on identical
rounded tensors.
"""

from __future__ import annotations

import numpy as np

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def bf16_round(a):
    """Round float values to bfloat16 (nearest even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) >> 16 << 16
    return (u.astype(np.uint32)).view(np.float32).astype(np.float64)


def _shift(x, dz, dy, dx):
    """y[z,y,x] = x[z+dz, y+dy, x+dx] with zeros outside."""
    out = np.zeros_like(x)
    Z, Y, X = x.shape[:3]
    zs, ys, xs = slice(max(0, -dz), min(Z, Z - dz)), slice(max(0, -dy), min(Y, Y - dy)), slice(max(0, -dx), min(X, X - dx))
    zd, yd, xd = slice(max(0, dz), min(Z, Z + dz)), slice(max(0, dy), min(Y, Y + dy)), slice(max(0, dx), min(X, X + dx))
    out[zs, ys, xs] = x[zd, yd, xd]
    return out


def conv3d(x, W, b=None):
    """Same-padded 3x3x3 convolution, channels-last.  W: (27, Cout, Cin)."""
    out = np.zeros(x.shape[:3] + (W.shape[1],))
    for t, (dz, dy, dx) in enumerate(TAPS):
        out += _shift(x, dz, dy, dx) @ W[t].T
    if b is not None:
        out += b
    return out


def conv3d_backward(x, W, g):
    """Gradients of sum(g * conv3d(x, W, b)) w.r.t. x, W and b."""
    gx = np.zeros_like(x)
    gW = np.zeros_like(W)
    for t, (dz, dy, dx) in enumerate(TAPS):
        xs = _shift(x, dz, dy, dx)
        gW[t] = np.einsum("zyxo,zyxi->oi", g, xs)
        gx += _shift(g @ W[t], -dz, -dy, -dx)
    gb = g.sum(axis=(0, 1, 2))
    return gx, gW, gb


def forward(params, feat, round_bf16=False):
    """Network forward.  params: list of (W, b); ReLU after every layer but
    the last.  Returns (output, list of layer inputs)."""
    rb = bf16_round if round_bf16 else (lambda a: a)
    acts = [rb(feat)]
    h = acts[0]
    for li, (W, b) in enumerate(params):
        z = conv3d(h, rb(W), b)
        if li + 1 < len(params):
            h = rb(np.maximum(z, 0.0))
            acts.append(h)
        else:
            h = z
    return h, acts


def masked_rel_l2(out, target, mask, nout):
    """Loss sum_mask |out - t|^2 / sum_mask |t|^2 over the first nout channels,
    and its gradient w.r.t. out."""
    m = mask[..., None].astype(float)
    d = (out[..., :nout] - target[..., :nout]) * m
    den = float((target[..., :nout] ** 2 * m).sum())
    loss = float((d**2).sum()) / den
    g = np.zeros_like(out)
    g[..., :nout] = 2.0 * d / den
    return loss, g


def backward(params, acts, gout, round_bf16=False):
    """Gradients of the loss w.r.t. every (W, b), given dL/d(output)."""
    rb = bf16_round if round_bf16 else (lambda a: a)
    grads = [None] * len(params)
    g = gout
    for li in range(len(params) - 1, -1, -1):
        W, _ = params[li]
        gx, gW, gb = conv3d_backward(acts[li], rb(W), rb(g) if round_bf16 else g)
        grads[li] = (gW, gb)
        if li > 0:
            g = gx * (acts[li] > 0)
    return grads
