"""Oracle pins for the learned warm start's network (2D and 3D).

* bfloat16 rounding against bit patterns worked by hand (round to nearest,
  ties to even on the 16-bit truncation);
* the convolution against its definition summed cell by cell (brute force);
* the input gradient is the adjoint of the convolution (<conv x, g> = <x, conv^T g>);
* weight, bias and whole-network gradients against central finite
  differences of the exact-arithmetic network;
* one Adam step against its closed form for a scalar.
"""
import itertools

import numpy as np
import pytest

from oracle import nn


def test_bf16_rounding_bit_patterns():
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: even mantissa (1) wins
    assert nn.bf16(1.0 + 2.0 ** -8) == 1.0
    # 1 + 3 * 2^-8 is a tie between 1 + 2^-7 (odd) and 1 + 2^-6 (even)
    assert nn.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    # just above the tie rounds up
    assert nn.bf16(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7
    # exactly representable values stay, signs are symmetric
    for v in (0.0, 1.0, -2.5, 3.0 * 2.0 ** -20, 65280.0):
        assert nn.bf16(v) == v
        assert nn.bf16(-v) == -v
    # 8 significant bits: pi -> 3.140625
    assert nn.bf16(np.pi) == 3.140625


@pytest.mark.parametrize("shape", [(5, 6), (4, 3, 5)])
def test_conv_matches_definition(shape):
    dim = len(shape)
    rng = np.random.default_rng(1)
    x = rng.standard_normal((3,) + shape)
    W = rng.standard_normal((2, 3) + (3,) * dim)
    b = rng.standard_normal(2)
    out = nn.conv(x, W, b)
    for idx in itertools.product(*[range(s) for s in shape]):
        for o in range(2):
            ref = b[o]
            for t in itertools.product(range(3), repeat=dim):
                src = tuple((i + ti - 1) % s for i, ti, s in zip(idx, t, shape))
                for c in range(3):
                    ref += W[(o, c) + t] * x[(c,) + src]
            assert abs(out[(o,) + idx] - ref) <= 1e-12 * (1 + abs(ref))


@pytest.mark.parametrize("shape", [(6, 7), (4, 5, 3)])
def test_conv_input_gradient_is_adjoint(shape):
    dim = len(shape)
    rng = np.random.default_rng(2)
    x = rng.standard_normal((4,) + shape)
    g = rng.standard_normal((3,) + shape)
    W = rng.standard_normal((3, 4) + (3,) * dim)
    lhs = np.sum(nn.conv(x, W, np.zeros(3)) * g)
    rhs = np.sum(x * nn.conv_grad_input(g, W))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("dim", [2, 3])
def test_network_gradients_finite_differences(dim):
    shape = (5, 4) if dim == 2 else (4, 3, 4)
    rng = np.random.default_rng(3)
    params = nn.init_params(7, dim)
    for W, b in params:
        b += 0.05 * rng.standard_normal(b.shape)  # non-zero biases exercise db
    x = rng.standard_normal((3,) + shape)
    t = rng.standard_normal(shape)
    loss, grads = nn.loss_and_grads(params, x, t, use_bf16=False)
    eps = 1e-6
    for l in (0, 2, 5):
        for j in (0, 1):
            arr = params[l][j]
            for _ in range(3):
                k = tuple(int(rng.integers(0, s)) for s in arr.shape)
                old = arr[k]
                arr[k] = old + eps
                lp, _ = nn.loss_and_grads(params, x, t, use_bf16=False)
                arr[k] = old - eps
                lm, _ = nn.loss_and_grads(params, x, t, use_bf16=False)
                arr[k] = old
                fd = (lp - lm) / (2 * eps)
                assert abs(grads[l][j][k] - fd) <= 1e-6 * max(1.0, abs(fd)), (l, j, k)


def test_adam_closed_form_scalar():
    params = [[np.array([[0.5]]), np.array([0.0])]] + [[np.zeros((1, 1)), np.zeros(1)] for _ in range(5)]
    grads = [[np.array([[2.0]]), np.array([0.0])]] + [[np.zeros((1, 1)), np.zeros(1)] for _ in range(5)]
    state = nn.adam_state(params)
    nn.adam(params, grads, state, lr=0.1, step=1)
    # first step: m = 0.1 g, v = 0.001 g^2, mhat = g, vhat = g^2 -> w -= lr g / (|g| + eps)
    expect = np.float32(0.5) - np.float32(0.1) * np.float32(2.0) / (np.float32(2.0) + np.float32(1e-8))
    assert params[0][0][0, 0] == np.float64(np.float32(expect))


def test_forward_of_a_13_cube_patch_gives_the_centre_value():
    """Six 3x3x3 layers reach 6 cells: the oracle forward on the 13^3 periodic
    patch around a voxel gives that voxel's output of the full-grid forward
    (the sampled 256^3 parity test relies on it). 20^3 grid, voxels inside
    and on the faces (their patches wrap around the box)."""
    rng = np.random.default_rng(31)
    n = 20
    params = nn.init_params(9, dim=3)
    params[5][0] *= 10.0
    x = rng.standard_normal((3, n, n, n))
    y, _ = nn.forward(params, x, use_bf16=True)
    for k, j, i in [(10, 10, 10), (0, 5, 19), (19, 0, 7), (3, 17, 0), (6, 13, 2)]:
        idx = [np.arange(c - 6, c + 7) % n for c in (k, j, i)]
        patch = x[:, idx[0][:, None, None], idx[1][None, :, None], idx[2][None, None, :]]
        yp, _ = nn.forward(params, patch, use_bf16=True)
        assert abs(yp[6, 6, 6] - y[k, j, i]) <= 1e-12 * np.abs(y).max()
