"""FP64 reference of the series-tail network (test infrastructure only).

The network maps the first k Neumann iterates of one trace (k input
channels over a window of T samples centred on t = 0) to two channels: the
even-pass and odd-pass sums of the remaining series terms.  Layers:

    conv(k -> H, K taps, dilation d1), ReLU,
    conv(H -> H, K taps, dilation d2), ReLU,
    conv(H -> 2, K taps, dilation d3)

Each conv is y[o][t] = b[o] + sum_c sum_j W[o][c][j] x[c][t + d (j - K//2)]
with zeros outside [0, T) ("same" padding).  Loss: mean squared error over
the samples where the mask is 1.

Everything here is plain numpy in float64 with explicit loops over taps; the
gradients are written out by hand and pinned by finite differences in
tests/test_tailnet_oracle.py.  The HIP kernels share no code with it.
"""

from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np

ARCH = dict(k=4, hidden=64, taps=5, dil=(1, 4, 16), out=2)


def init_params(rng: np.random.Generator, k: int = 4, hidden: int = 64, taps: int = 5,
                out: int = 2) -> Dict[str, np.ndarray]:
    """He-style initialisation; last layer small so the net starts near zero."""
    def w(o, c, scale):
        return rng.standard_normal((o, c, taps)) * scale
    return {
        "W1": w(hidden, k, np.sqrt(2.0 / (k * taps))), "b1": np.zeros(hidden),
        "W2": w(hidden, hidden, np.sqrt(2.0 / (hidden * taps))), "b2": np.zeros(hidden),
        "W3": w(out, hidden, 0.1 * np.sqrt(1.0 / (hidden * taps))), "b3": np.zeros(out),
    }


def shift(x: np.ndarray, s: int) -> np.ndarray:
    """xs[..., t] = x[..., t + s], zero outside the window."""
    T = x.shape[-1]
    out = np.zeros_like(x)
    if s >= 0:
        if s < T:
            out[..., :T - s] = x[..., s:]
    else:
        if -s < T:
            out[..., -s:] = x[..., :T + s]
    return out


def conv(x: np.ndarray, W: np.ndarray, b: np.ndarray, d: int) -> np.ndarray:
    """x [N][C][T], W [O][C][K], b [O] -> [N][O][T]."""
    K = W.shape[2]
    y = np.broadcast_to(b[None, :, None], (x.shape[0], W.shape[0], x.shape[2])).astype(np.float64).copy()
    for j in range(K):
        y += np.einsum("oc,nct->not", W[:, :, j], shift(x, d * (j - K // 2)))
    return y


def conv_backward(x: np.ndarray, W: np.ndarray, d: int, gy: np.ndarray) -> Tuple[np.ndarray, ...]:
    """Gradients of sum(gy * conv(x, W, b, d)) with respect to x, W and b."""
    K = W.shape[2]
    gx = np.zeros_like(x, dtype=np.float64)
    gW = np.zeros_like(W, dtype=np.float64)
    for j in range(K):
        s = d * (j - K // 2)
        gW[:, :, j] = np.einsum("not,nct->oc", gy, shift(x, s))
        # y[t] depends on x[t + s]: x[u] receives gy[u - s]
        gx += np.einsum("oc,not->nct", W[:, :, j], shift(gy, -s))
    gb = gy.sum(axis=(0, 2))
    return gx, gW, gb


def forward(P: Dict[str, np.ndarray], x: np.ndarray, dil=ARCH["dil"]) -> Tuple[np.ndarray, List]:
    a1 = conv(x, P["W1"], P["b1"], dil[0])
    h1 = np.maximum(a1, 0.0)
    a2 = conv(h1, P["W2"], P["b2"], dil[1])
    h2 = np.maximum(a2, 0.0)
    y = conv(h2, P["W3"], P["b3"], dil[2])
    return y, [x, a1, h1, a2, h2]


FP16_MAX = 65504.0


def to_f16(v: np.ndarray) -> np.ndarray:
    """Round to the nearest IEEE half (ties to even), saturating at +-65504,
    back in float64: the storage step of the inference form below."""
    return np.clip(np.asarray(v, dtype=np.float64), -FP16_MAX, FP16_MAX).astype(np.float16).astype(np.float64)


def forward_f16(P: Dict[str, np.ndarray], x: np.ndarray, dil=ARCH["dil"]) -> np.ndarray:
    """The inference form of the tail network with half-precision activations:
    the input and both hidden activations (after the ReLU) are stored as
    halves, every product and sum is exact arithmetic on those values (float64
    here; float32 accumulation on the GPU), the weights are used as given."""
    h0 = to_f16(x)
    h1 = to_f16(np.maximum(conv(h0, P["W1"], P["b1"], dil[0]), 0.0))
    h2 = to_f16(np.maximum(conv(h1, P["W2"], P["b2"], dil[1]), 0.0))
    return conv(h2, P["W3"], P["b3"], dil[2])


def loss_and_grad(P: Dict[str, np.ndarray], x: np.ndarray, target: np.ndarray, mask: np.ndarray,
                  dil=ARCH["dil"]) -> Tuple[float, Dict[str, np.ndarray]]:
    """Masked mean squared error and its gradient with respect to every parameter."""
    y, (x0, a1, h1, a2, h2) = forward(P, x, dil)
    cnt = max(1.0, float(mask.sum()) * y.shape[1])
    r = (y - target) * mask[:, None, :]
    loss = float((r * r).sum() / cnt)
    gy = 2.0 * r / cnt
    g = {}
    gh2, g["W3"], g["b3"] = conv_backward(h2, P["W3"], dil[2], gy)
    ga2 = gh2 * (a2 > 0)
    gh1, g["W2"], g["b2"] = conv_backward(h1, P["W2"], dil[1], ga2)
    ga1 = gh1 * (a1 > 0)
    _, g["W1"], g["b1"] = conv_backward(x0, P["W1"], dil[0], ga1)
    return loss, g


def adam_step(P, G, M, V, step: int, lr: float = 1e-3, b1: float = 0.9, b2: float = 0.999,
              eps: float = 1e-8) -> None:
    """One Adam update (Kingma and Ba 2015), in place, with bias correction."""
    for k in P:
        M[k] = b1 * M[k] + (1 - b1) * G[k]
        V[k] = b2 * V[k] + (1 - b2) * G[k] * G[k]
        mh = M[k] / (1 - b1 ** step)
        vh = V[k] / (1 - b2 ** step)
        P[k] = P[k] - lr * mh / (np.sqrt(vh) + eps)
