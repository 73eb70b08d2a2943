"""mk_net_loss_noalloc (the loss without a caller scratch buffer) against
mk_net_loss through the C ABI: two calls in a row, the second with a smaller
input, each bit for bit equal to mk_net_loss with its own scratch buffer and
the same number of partial sums; and the size limit is refused."""

import numpy as np
import pytest

from gpu_common import require_gpu, say

pytestmark = pytest.mark.gpu


def _case(rng, N, T):
    y = rng.standard_normal((N, 2, T)).astype(np.float32)
    tgt = (0.3 * rng.standard_normal((N, 2, T))).astype(np.float32)
    mask = (rng.random((N, T)) < 0.6).astype(np.float32)
    return y, tgt, mask, float(mask.sum() * 2)


def _both(mk, torch, y, tgt, mask, count, nparts):
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    yd, td, md = d(y), d(tgt), d(mask)
    gy_a, gy_b = torch.full_like(yd, np.nan), torch.full_like(yd, np.nan)
    loss_a = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
    loss_b = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
    part = torch.full((nparts,), np.nan, dtype=torch.float64, device="cuda")
    mk.mk_net_loss(yd, td, md, count, gy_a, loss_a, part)
    mk.mk_net_loss_noalloc(yd, td, md, count, gy_b, loss_b, nparts)
    torch.cuda.synchronize()
    return (loss_a.item(), gy_a.cpu().numpy()), (loss_b.item(), gy_b.cpu().numpy())


def test_noalloc_loss_matches_the_allocating_entry_point():
    mk = require_gpu()
    import torch

    rng = np.random.default_rng(77)
    for N, T, nparts in ((96, 1024, 1024), (5, 301, 37)):
        say(f"no-alloc loss N={N} T={T} nparts={nparts}")
        y, tgt, mask, count = _case(rng, N, T)
        (la, ga), (lb, gb) = _both(mk, torch, y, tgt, mask, count, nparts)
        # the same definition in numpy: the FP32 residual, squared and summed in FP64
        r = ((y - tgt) * mask[:, None, :]).astype(np.float64)
        want = float((r * r).sum() / count)
        say(f"  loss {lb:.12e} (allocating {la:.12e}, numpy {want:.12e})")
        assert lb == la
        assert np.array_equal(gb, ga)
        assert abs(lb - want) <= 1e-12 * want


def test_noalloc_loss_refuses_sizes_beyond_its_array():
    mk = require_gpu()
    import torch

    y = torch.zeros((2, 2, 8), device="cuda")
    mask = torch.ones((2, 8), device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    for bad in (0, 1025):
        with pytest.raises(mk.MKError) as ei:
            mk.mk_net_loss_noalloc(y, y, mask, 1.0, torch.zeros_like(y), loss, bad)
        assert ei.value.status == mk.MK_ERR_ARG
