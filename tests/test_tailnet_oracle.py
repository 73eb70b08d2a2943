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


# ---------------------------------------------------------------------------
# the inference form with half-precision activations
# ---------------------------------------------------------------------------


def test_half_rounding_hand_values():
    u = 2.0 ** -10                      # spacing of halves in [1, 2)
    cases = [(1 + u / 2, 1.0), (1 + 1.5 * u, 1 + 2 * u), (1 + u / 4, 1.0), (1 + 0.75 * u, 1 + u),
             (70000.0, 65504.0), (-1e6, -65504.0), (2.0 ** -25, 0.0), (3 * 2.0 ** -26, 2.0 ** -24),
             (-(1 + 1.5 * u), -(1 + 2 * u))]
    for v, want in cases:
        assert tn.to_f16(np.array([v]))[0] == want, v


def _unit_net(w1=1.0, w2=1.0):
    """k = 1, hidden 1: centre taps only, so y = (c0, c1) * w2 * w1 * x."""
    def centre(o, c, v):
        W = np.zeros((o, c, 5))
        W[:, :, 2] = v
        return W
    W3 = np.zeros((2, 1, 5))
    W3[0, 0, 2], W3[1, 0, 2] = 1.0, 2.0
    return {"W1": centre(1, 1, w1), "b1": np.zeros(1), "W2": centre(1, 1, w2), "b2": np.zeros(1),
            "W3": W3, "b3": np.zeros(2)}


def test_half_form_rounds_input_and_both_activations():
    e = 2.0 ** -12                       # below half a half-ulp at 1: rounds away
    x = np.full((1, 1, 8), 1.0)
    for P, xin in ((_unit_net(), x * (1 + e)),          # the input is stored as a half
                   (_unit_net(w1=1 + e), x),            # so is the first activation
                   (_unit_net(w2=1 + e), x)):           # and the second
        y, _ = tn.forward(P, xin)
        assert not np.allclose(y[0, 0], 1.0, rtol=0, atol=1e-6)
        y16 = tn.forward_f16(P, xin)
        np.testing.assert_array_equal(y16[0, 0], np.ones(8))
        np.testing.assert_array_equal(y16[0, 1], np.full(8, 2.0))


def test_half_form_equals_plain_form_on_exact_values():
    """Integer weights, inputs and biases small enough that every activation
    is an integer below 2048: both forms agree exactly."""
    rng = np.random.default_rng(7)
    P = {"W1": rng.integers(-1, 2, (6, 3, 5)).astype(float), "b1": rng.integers(-2, 3, 6).astype(float),
         "W2": rng.integers(-1, 2, (6, 6, 5)).astype(float), "b2": rng.integers(-2, 3, 6).astype(float),
         "W3": rng.integers(-1, 2, (2, 6, 5)).astype(float), "b3": rng.integers(-2, 3, 2).astype(float)}
    x = rng.integers(-3, 4, (2, 3, 40)).astype(float)
    y, (_, a1, _, a2, _) = tn.forward(P, x)
    assert np.abs(a1).max() < 2048 and np.abs(a2).max() < 2048
    np.testing.assert_array_equal(tn.forward_f16(P, x), y)


def test_adam_two_steps_closed_form():
    """Two steps with b1 = 1/2, b2 = 3/4 (so that the bias corrections of step 2,
    1 - b1^2 = 3/4 and 1 - b2^2 = 7/16, differ from those of step 1), lr = 1,
    gradients 1 then 3, worked by hand:
      step 1: m = 1/2, v = 1/4, m^ = 1, v^ = 1, w -= 1;
      step 2: m = 7/4, v = 39/16, m^ = 7/3, v^ = 39/7, w -= (7/3) / sqrt(39/7)."""
    P = {"w": np.array([5.0, -1.0])}
    M = {"w": np.zeros(2)}
    V = {"w": np.zeros(2)}
    tn.adam_step(P, {"w": np.array([1.0, -1.0])}, M, V, step=1, lr=1.0, b1=0.5, b2=0.75, eps=0.0)
    np.testing.assert_allclose(P["w"], [4.0, 0.0], rtol=0, atol=1e-15)
    tn.adam_step(P, {"w": np.array([3.0, -3.0])}, M, V, step=2, lr=1.0, b1=0.5, b2=0.75, eps=0.0)
    d = (7.0 / 3.0) / np.sqrt(39.0 / 7.0)
    np.testing.assert_allclose(P["w"], [4.0 - d, d], rtol=0, atol=1e-14)
    np.testing.assert_allclose(M["w"], [1.75, -1.75], rtol=0, atol=1e-15)
    np.testing.assert_allclose(V["w"], [39.0 / 16.0, 39.0 / 16.0], rtol=0, atol=1e-15)
