"""The tail network's HIP kernels against the FP64 network reference
(oracle/tailnet.py, itself pinned by finite differences)."""

import numpy as np
import pytest

from gpu_common import require_gpu, say
from oracle import tailnet as tn

pytestmark = pytest.mark.gpu


def _flat(P, k):
    return np.concatenate([P["W1"].ravel(), P["b1"], P["W2"].ravel(), P["b2"], P["W3"].ravel(), P["b3"]])


def _unflat(v, k, H):
    out, o = {}, 0
    for name, shape in (("W1", (H, k, 5)), ("b1", (H,)), ("W2", (H, H, 5)), ("b2", (H,)),
                        ("W3", (2, H, 5)), ("b3", (2,))):
        n = int(np.prod(shape))
        out[name] = v[o:o + n].reshape(shape)
        o += n
    return out


@pytest.mark.parametrize("N,k,T,H", [(3, 4, 70, 64), (5, 2, 200, 64), (1, 4, 64, 64), (4, 4, 130, 16),
                                     (2, 3, 90, 8), (3, 4, 70, 5)])
def test_forward_loss_backward_match_reference(N, k, T, H):
    mk = require_gpu()
    import torch

    say(f"tailnet N={N} k={k} T={T} H={H}")
    rng = np.random.default_rng(N * 100 + T)
    P = tn.init_params(rng, k=k, hidden=H)
    for key in P:
        P[key] = (P[key] + 0.05 * rng.standard_normal(P[key].shape)).astype(np.float32).astype(np.float64)
    x = rng.standard_normal((N, k, T)).astype(np.float32)
    tgt = (0.1 * rng.standard_normal((N, 2, T))).astype(np.float32)
    mask = (rng.random((N, T)) < 0.7).astype(np.float32)
    count = float(mask.sum() * 2)
    loss_ref, g_ref = tn.loss_and_grad(P, x.astype(np.float64), tgt.astype(np.float64),
                                       mask.astype(np.float64))
    y_ref, _ = tn.forward(P, x.astype(np.float64))
    assert mk.mk_net_param_count(k, H) == _flat(P, k).size
    assert mk.net_hidden(_flat(P, k).size, k) == H
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    params = d(_flat(P, k).astype(np.float32))
    xd, td, md = d(x), d(tgt), d(mask)
    work = torch.zeros(2 * N * H * T, device="cuda")
    work2 = torch.zeros(2 * N * H * T + H * H * 5, device="cuda")
    y = torch.zeros((N, 2, T), device="cuda")
    gy = torch.zeros_like(y)
    grads = torch.zeros_like(params)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    part = torch.zeros(64, dtype=torch.float64, device="cuda")
    mk.mk_net_forward(params, xd, work, y)
    mk.mk_net_loss(y, td, md, count, gy, loss, part)
    mk.mk_net_backward(params, xd, work, gy, grads, work2)
    torch.cuda.synchronize()
    np.testing.assert_allclose(y.cpu().numpy(), y_ref, rtol=1e-4, atol=1e-5 * np.abs(y_ref).max())
    assert abs(loss.item() - loss_ref) <= 1e-4 * loss_ref
    G = _unflat(grads.cpu().numpy().astype(np.float64), k, H)
    for key in g_ref:
        scale = np.abs(g_ref[key]).max() + 1e-30
        err = np.abs(G[key] - g_ref[key]).max() / scale
        say(f"  grad {key}: max rel err {err:.2e}")
        assert err <= 2e-4, key


def test_adam_and_bf16_rounding_match_reference():
    mk = require_gpu()
    import torch

    rng = np.random.default_rng(9)
    n = 1000
    w = rng.standard_normal(n).astype(np.float32)
    g = rng.standard_normal(n).astype(np.float32)
    P = {"w": w.astype(np.float64)}
    M = {"w": np.zeros(n)}
    V = {"w": np.zeros(n)}
    wd, gd = torch.from_numpy(w.copy()).cuda(), torch.from_numpy(g).cuda()
    md, vd, wq = torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")
    for step in (1, 2, 3):
        tn.adam_step(P, {"w": g.astype(np.float64)}, M, V, step, lr=1e-2)
        mk.mk_net_adam(wd, wq, gd, md, vd, step, lr=1e-2)
    torch.cuda.synchronize()
    np.testing.assert_allclose(wd.cpu().numpy(), P["w"], rtol=1e-5, atol=1e-6)
    # bf16 rounding: nearest, ties to even, of the updated weights
    u = wd.cpu().numpy().view(np.uint32).astype(np.uint64)
    want = (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16).astype(np.uint32).view(np.float32)
    assert np.array_equal(wq.cpu().numpy(), want)
