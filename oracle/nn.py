"""Learned warm start for the pressure solve (oracle; project addition, not in
the paper). TEST INFRASTRUCTURE ONLY.

A 6-layer convolutional network maps three per-cell channels
(divergence right side, inverse density, previous pressure) to a correction
of the previous pressure; multigrid then starts from
    p0 = p_prev + s_p * y,
and remains the judge of the final answer.

Definition (2D):
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

Arrays: activations (C, H, W) with W = x fastest; weights (Cout, Cin, 3, 3)
where tap (ky, kx) multiplies the input at (y + ky - 1, x + kx - 1).
"""
import numpy as np

CHANNELS = (3, 32, 32, 32, 32, 32, 1)


def bf16(x):
    """Round float64 values to bfloat16 (through float32, nearest even)."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def init_params(seed=0):
    """He-normal weights (float32 master copy), zero biases."""
    rng = np.random.default_rng(seed)
    params = []
    for l in range(6):
        ci, co = CHANNELS[l], CHANNELS[l + 1]
        std = np.sqrt(2.0 / (ci * 9)) if l < 5 else 0.1 * np.sqrt(1.0 / (ci * 9))
        W = (rng.standard_normal((co, ci, 3, 3)) * std).astype(np.float32).astype(np.float64)
        params.append([W, np.zeros(co)])
    return params


def conv(x, W, b):
    """out[o, y, x] = b[o] + sum_{i, ky, kx} W[o, i, ky, kx] x[i, y+ky-1, x+kx-1] (periodic)."""
    C, H, Wd = x.shape
    out = np.zeros((W.shape[0], H, Wd))
    for ky in range(3):
        for kx in range(3):
            xs = np.roll(np.roll(x, -(ky - 1), axis=1), -(kx - 1), axis=2)
            out += np.einsum("oi,ihw->ohw", W[:, :, ky, kx], xs)
    return out + b[:, None, None]


def conv_grad_input(g, W):
    """Adjoint of conv in x."""
    out = np.zeros((W.shape[1],) + g.shape[1:])
    for ky in range(3):
        for kx in range(3):
            t = np.einsum("oi,ohw->ihw", W[:, :, ky, kx], g)
            out += np.roll(np.roll(t, ky - 1, axis=1), kx - 1, axis=2)
    return out


def conv_grad_weight(g, x):
    dW = np.zeros((g.shape[0], x.shape[0], 3, 3))
    for ky in range(3):
        for kx in range(3):
            xs = np.roll(np.roll(x, -(ky - 1), axis=1), -(kx - 1), axis=2)
            dW[:, :, ky, kx] = np.einsum("ohw,ihw->oi", g, xs)
    return dW, g.sum(axis=(1, 2))


def normalise(b, inv_rho, p_prev, h):
    bh = b * h * h
    sb = float(np.sqrt(np.mean(bh * bh))) or 1.0
    sp = float(np.sqrt(np.mean(p_prev * p_prev))) or 1.0
    sr = float(np.max(inv_rho)) or 1.0
    x = np.stack([bh / sb, inv_rho / sr, p_prev / sp])
    return x, sp


def forward(params, x, use_bf16=True):
    """Returns (y, cache) with y of shape (H, W)."""
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
