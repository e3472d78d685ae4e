"""Learned warm start for the pressure solve (oracle; project addition, not in
the paper). TEST INFRASTRUCTURE ONLY.

A 6-layer convolutional network maps three per-cell channels
(divergence right side, inverse density, previous pressure) to a correction
of the previous pressure; multigrid then starts from
    p0 = p_prev + s_p * y,
and alone decides the final answer.

Definition (2D; the 3D network is the same with 3x3x3 taps):
  * inputs, normalised per sample: x0 = b h^2 / s_b, x1 = (1/rho) / max(1/rho),
    x2 = p_prev / s_p, with s_b, s_p the root-mean-square values of b h^2 and
    p_prev (1 when zero);
  * layers: 3x3 convolutions with circular padding, channels 3 -> 32 -> 32 ->
    32 -> 32 -> 32 -> 1, bias, ReLU after every layer but the last;
  * target: t = (p - p_prev) / s_p; loss = mean over cells of (y - t)^2;
  * precision: weights, activations and the gradients entering each layer's
    products are bfloat16 at layer boundaries
    (round to nearest even from float32), sums accumulate in float32 on the
    GPU; this oracle accumulates in float64 and rounds the same quantities to
    bfloat16 when `bf16=True` (exact float64 arithmetic when False, used for the
    finite-difference gradient check).
  * optimiser: Adam (beta1 0.9, beta2 0.999, eps 1e-8) on float32 master
    weights.

Arrays: activations (C, H, W) or (C, D, H, W) with x fastest; weights
(Cout, Cin, 3, 3) or (Cout, Cin, 3, 3, 3) where tap (kz,) ky, kx multiplies the
input at ((z + kz - 1,) y + ky - 1, x + kx - 1).
"""
import itertools

import numpy as np

CHANNELS = (3, 32, 32, 32, 32, 32, 1)


def bf16(x):
    """Round float64 values to bfloat16 (through float32, nearest even)."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def taps(dim):
    """Tap index tuples (t_0, ..., t_{dim-1}) in {0, 1, 2}^dim, last axis fastest;
    tap t multiplies the input at offset t - 1 along each axis."""
    return list(itertools.product(range(3), repeat=dim))


def init_params(seed=0, dim=2):
    """He-normal weights (float32 master copy), zero biases; W has shape
    (Cout, Cin, 3[, 3], 3)."""
    rng = np.random.default_rng(seed)
    params = []
    for l in range(6):
        ci, co = CHANNELS[l], CHANNELS[l + 1]
        fan = ci * 3 ** dim
        std = np.sqrt(2.0 / fan) if l < 5 else 0.1 * np.sqrt(1.0 / fan)
        W = (rng.standard_normal((co, ci) + (3,) * dim) * std).astype(np.float32).astype(np.float64)
        params.append([W, np.zeros(co)])
    return params


def _shift(x, t, sign):
    """x moved so that out[..., i] = x[..., i + sign (t - 1)] (periodic) on the spatial axes."""
    for a, ta in enumerate(t):
        x = np.roll(x, -sign * (ta - 1), axis=x.ndim - len(t) + a)
    return x


def conv(x, W, b):
    """out[o, i] = b[o] + sum_{c, t} W[o, c, t] x[c, i + t - 1] (periodic), i a 2D or 3D index."""
    dim = x.ndim - 1
    out = np.zeros((W.shape[0],) + x.shape[1:])
    for t in taps(dim):
        out += np.einsum("oc,c...->o...", W[(slice(None), slice(None)) + t], _shift(x, t, 1))
    return out + b.reshape((-1,) + (1,) * dim)


def conv_grad_input(g, W):
    """Adjoint of conv in x."""
    dim = g.ndim - 1
    out = np.zeros((W.shape[1],) + g.shape[1:])
    for t in taps(dim):
        v = np.einsum("oc,o...->c...", W[(slice(None), slice(None)) + t], g)
        out += _shift(v, t, -1)
    return out


def conv_grad_weight(g, x):
    dim = x.ndim - 1
    dW = np.zeros((g.shape[0], x.shape[0]) + (3,) * dim)
    axes = tuple(range(1, dim + 1))
    for t in taps(dim):
        dW[(slice(None), slice(None)) + t] = np.tensordot(g, _shift(x, t, 1), axes=(axes, axes))
    return dW, g.sum(axis=axes)


def normalise(b, inv_rho, p_prev, h):
    bh = b * h * h
    sb = float(np.sqrt(np.mean(bh * bh))) or 1.0
    sp = float(np.sqrt(np.mean(p_prev * p_prev))) or 1.0
    sr = float(np.max(inv_rho)) or 1.0
    x = np.stack([bh / sb, inv_rho / sr, p_prev / sp])
    return x, sp


def forward(params, x, use_bf16=True):
    """Returns (y, cache) with y of the spatial shape of x."""
    q = bf16 if use_bf16 else (lambda a: a)
    acts = [q(x)]
    for l, (W, b) in enumerate(params):
        z = conv(acts[-1], q(W), b)
        if l < 5:
            acts.append(q(np.maximum(z, 0.0)))
        else:
            acts.append(z)
    return acts[-1][0], acts


def loss_and_grads(params, x, t, use_bf16=True):
    q = bf16 if use_bf16 else (lambda a: a)
    y, acts = forward(params, x, use_bf16)
    N = y.size
    loss = float(np.mean((y - t) ** 2))
    g = (2.0 / N) * (y - t)[None]
    grads = [None] * 6
    for l in range(5, -1, -1):
        W, b = params[l]
        # the gradient entering layer l's products is bfloat16, like its activations
        g = q(g * (acts[l + 1] > 0)) if l < 5 else q(g)
        dW, db = conv_grad_weight(g, acts[l])
        grads[l] = [dW, db]
        if l > 0:
            g = conv_grad_input(g, q(W))
    return loss, grads


def adam(params, grads, state, lr, step, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step on float32 master weights (state: list of (m, v) pairs)."""
    for l in range(6):
        for j in range(2):
            m, v = state[l][j]
            g = grads[l][j].astype(np.float32)
            m[...] = np.float32(b1) * m + np.float32(1 - b1) * g
            v[...] = np.float32(b2) * v + np.float32(1 - b2) * g * g
            mh = m / np.float32(1 - b1 ** step)
            vh = v / np.float32(1 - b2 ** step)
            p32 = params[l][j].astype(np.float32) - np.float32(lr) * mh / (np.sqrt(vh) + np.float32(eps))
            params[l][j] = p32.astype(np.float64)
    return params


def adam_state(params):
    return [[(np.zeros(W.shape, np.float32), np.zeros(W.shape, np.float32)),
             (np.zeros(b.shape, np.float32), np.zeros(b.shape, np.float32))] for W, b in params]
