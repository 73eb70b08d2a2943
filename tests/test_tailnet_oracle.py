"""Pins of the FP64 tail-network reference: a brute-force convolution with
explicit loops, central finite differences of the loss for every parameter
tensor, and Adam's first step in closed form."""

import numpy as np
import pytest

from oracle import tailnet as tn


def brute_conv(x, W, b, d):
    N, C, T = x.shape
    O, _, K = W.shape
    y = np.zeros((N, O, T))
    for n in range(N):
        for o in range(O):
            for t in range(T):
                acc = b[o]
                for c in range(C):
                    for j in range(K):
                        u = t + d * (j - K // 2)
                        if 0 <= u < T:
                            acc += W[o, c, j] * x[n, c, u]
                y[n, o, t] = acc
    return y


@pytest.mark.parametrize("d", [1, 3, 7])
def test_conv_matches_loops(d):
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 3, 11))
    W = rng.standard_normal((4, 3, 5))
    b = rng.standard_normal(4)
    np.testing.assert_allclose(tn.conv(x, W, b, d), brute_conv(x, W, b, d), atol=1e-12)


def test_identity_kernel_passes_input_through():
    x = np.random.default_rng(1).standard_normal((1, 2, 9))
    W = np.zeros((2, 2, 5))
    W[0, 0, 2] = W[1, 1, 2] = 1.0
    np.testing.assert_array_equal(tn.conv(x, W, np.zeros(2), 4), x)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(2)
    P = tn.init_params(rng, k=3, hidden=5, taps=3)
    for k in P:                     # make biases non-trivial so ReLU kinks are exercised
        P[k] = P[k] + 0.05 * rng.standard_normal(P[k].shape)
    dil = (1, 2, 3)
    x = rng.standard_normal((2, 3, 13))
    tgt = rng.standard_normal((2, 2, 13))
    mask = (rng.random((2, 13)) < 0.8).astype(float)
    loss, g = tn.loss_and_grad(P, x, tgt, mask, dil)
    h = 1e-6
    for key in P:
        flat = P[key].reshape(-1)
        for i in range(0, flat.size, max(1, flat.size // 7)):
            old = flat[i]
            flat[i] = old + h
            lp, _ = tn.loss_and_grad(P, x, tgt, mask, dil)
            flat[i] = old - h
            lm, _ = tn.loss_and_grad(P, x, tgt, mask, dil)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[key].reshape(-1)[i]) <= 1e-6 * max(1.0, abs(fd)), (key, i, fd)


def test_adam_first_step_is_lr_times_sign():
    P = {"w": np.array([1.0, -2.0, 3.0])}
    G = {"w": np.array([0.5, -0.25, 0.0])}
    M = {"w": np.zeros(3)}
    V = {"w": np.zeros(3)}
    tn.adam_step(P, G, M, V, step=1, lr=0.01, eps=0.0 + 1e-30)
    # after bias correction, the first step moves each weight by lr * sign(g)
    np.testing.assert_allclose(P["w"], [1.0 - 0.01, -2.0 + 0.01, 3.0], atol=1e-12)
