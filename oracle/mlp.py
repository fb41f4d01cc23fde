"""Oracle for the learned candidate ordering — TEST INFRASTRUCTURE.

Only the test suite may import this module.  Plain numpy in float64.

The paper has no learned component; the encoder is this project's addition on
top of the exact scan.  It only reorders candidates (the scan's results do not
depend on the order), so its training quality is measured, never pinned.

Model (the readings the GPU library follows):

* resample: a series of length L (L x d) goes to P = 32 points by linear
  interpolation at t_k = k (L - 1) / 31: x_k = s_i0 + f (s_i1 - s_i0) with
  i0 = floor(t_k), i1 = min(i0 + 1, L - 1), f = t_k - i0.  The input vector
  is [x_0, ..., x_31] flattened point-major (index k d + dim).
* encoder: widths (P d) -> H -> H -> E (96 -> 256 -> 256 -> 64 at d = 3);
  z = W r(h) + b with r(.) = round to bfloat16 and W = r(master weights);
  ReLU on the hidden layers, the output layer is linear.  Biases stay fp32.
* predicted distance of a pair: ||e_a - e_b||_2; loss: mean over the batch
  of (prediction - target)^2, the target being the pair's DK distance.
* backward: the rounding r(.) passes gradients unchanged; the operands of
  both backward products (dz with r(W) for the input gradient, dz with r(h)
  for the weight gradient) are rounded to bfloat16 as in the forward pass.
* Adam (beta1 0.9, beta2 0.999, eps 1e-8) on fp32 master weights.

``rounding=False`` drops every r(.) (a smooth fp64 network), which is what
the finite-difference check differentiates.
"""
from __future__ import annotations

import numpy as np

P = 32


def bf16_round(x):
    """Round to nearest bfloat16 (8 significant bits), ties to even, from
    the float64 value itself (frexp: x = m 2^e, 0.5 <= |m| < 1)."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)
    return np.ldexp(np.rint(m * 256.0) / 256.0, e)


def resample(vals, offsets, p=P):
    """[n, p * d] float64 inputs of the series vals[offsets[i]:offsets[i+1]]."""
    vals = np.asarray(vals, dtype=np.float64)
    n = len(offsets) - 1
    d = vals.shape[1]
    out = np.empty((n, p * d))
    for i in range(n):
        s = vals[offsets[i]:offsets[i + 1]]
        L = s.shape[0]
        for k in range(p):
            num = k * (L - 1)
            i0 = num // (p - 1)
            f = (num - i0 * (p - 1)) / (p - 1)
            i1 = min(i0 + 1, L - 1)
            out[i, k * d:(k + 1) * d] = s[i0] + f * (s[i1] - s[i0])
    return out


def param_shapes(d_in, hidden, d_out):
    return [(hidden, d_in), (hidden,), (hidden, hidden), (hidden,), (d_out, hidden), (d_out,)]


def forward(params, x, rounding=True):
    """Returns (embeddings, cache) for inputs x [n, d_in]."""
    r = bf16_round if rounding else (lambda v: v)
    W1, b1, W2, b2, W3, b3 = params
    h0 = r(x)
    z1 = h0 @ r(W1).T + b1
    a1 = np.maximum(z1, 0.0)
    h1 = r(a1)
    z2 = h1 @ r(W2).T + b2
    a2 = np.maximum(z2, 0.0)
    h2 = r(a2)
    e = h2 @ r(W3).T + b3
    return e, (h0, z1, h1, z2, h2)


def pair_loss(ea, eb, y):
    """Mean squared error of ||ea - eb|| against y, and its gradients with
    respect to ea and eb."""
    diff = ea - eb
    pred = np.sqrt(np.sum(diff * diff, axis=1))
    err = pred - y
    loss = np.mean(err * err)
    g = 2.0 * err / len(y)
    safe = np.where(pred > 0, pred, 1.0)
    dea = (g / safe)[:, None] * diff * (pred > 0)[:, None]
    return loss, pred, dea, -dea


def backward(params, cache, de, rounding=True):
    """Parameter gradients for the upstream gradient de [n, d_out]."""
    r = bf16_round if rounding else (lambda v: v)
    W1, b1, W2, b2, W3, b3 = params
    h0, z1, h1, z2, h2 = cache
    g3 = de
    dW3 = r(g3).T @ h2
    db3 = g3.sum(0)
    dh2 = r(g3) @ r(W3)
    g2 = dh2 * (z2 > 0)
    dW2 = r(g2).T @ h1
    db2 = g2.sum(0)
    dh1 = r(g2) @ r(W2)
    g1 = dh1 * (z1 > 0)
    dW1 = r(g1).T @ h0
    db1 = g1.sum(0)
    return [dW1, db1, dW2, db2, dW3, db3]


def batch_grads(params, xa, xb, y, rounding=True):
    """Loss and parameter gradients of one batch of pairs (both towers share
    the weights: the batch runs as one stacked pass of 2n rows)."""
    n = len(y)
    e, cache = forward(params, np.concatenate([xa, xb]), rounding)
    loss, pred, dea, deb = pair_loss(e[:n], e[n:], y)
    grads = backward(params, cache, np.concatenate([dea, deb]), rounding)
    return loss, grads


def adam_step(params, grads, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (step number t >= 1); returns new (params, m, v)."""
    out_p, out_m, out_v = [], [], []
    for p_, g, m_, v_ in zip(params, grads, m, v):
        m_ = b1 * m_ + (1 - b1) * g
        v_ = b2 * v_ + (1 - b2) * g * g
        mh = m_ / (1 - b1 ** t)
        vh = v_ / (1 - b2 ** t)
        out_p.append(p_ - lr * mh / (np.sqrt(vh) + eps))
        out_m.append(m_)
        out_v.append(v_)
    return out_p, out_m, out_v
