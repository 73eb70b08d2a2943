"""R streamed from pinned host memory (a device cap below the size of R):
the pipelined batches of Algorithm 2 for reflection data larger than the
GPU's memory.  A plan with a cap holds R on the host and copies slabs of
frequency bins into two device buffers on every synthesis; each slab's
contraction is the resident plan's kernel on those bins, so every output is
the resident plan's, bit for bit, and matches the FP64 oracle at the FP32
bar.  Cases: the streaming GEMV (complex64 and FP16 R), the tiled batch on
the matrix cores (FP32 and FP16, with per-focal bands), the series tail and
restart, the auxiliary fields, and the full-size workload with six slabs."""

import numpy as np
import pytest

from gpu_common import FIELD_NAMES, TOL_FP32, require_gpu, say
from mkgen.layered import make_config, small_problem
from oracle import SynthesisOperator, marchenko, rel_l2

pytestmark = pytest.mark.gpu


def _r_bytes(p, rprec, nf_max):
    """Bytes of R in the plan's storage (row-major, or tiled for nf_max > 4)."""
    nr, B = p.Rhat.shape[0], p.Rhat.shape[1]
    ns_pad = (nr + 31) // 32 * 32
    e = 8 if rprec == 0 else 4
    if nf_max > 4:
        ng = (nr + 15) // 16
        return B * ng * 16 * ns_pad * e
    return B * nr * ns_pad * e


def _solve(mk, p, cap, rprec=0, nf_max=None, fbands=None, niter=None, flags=0, tail=None, aux=False):
    nr, nt = p.Rhat.shape[0], p.geom.nt
    nf_max = nf_max or p.nf
    plan = mk.mk_plan(nr, nr, nt, p.geom.dt, p.geom.dx, band=p.band, nf_max=nf_max, rprec=rprec, flags=flags,
                      r_dev_bytes=cap)
    mk.mk_load_R(plan, p.Rhat)
    if tail is not None:
        mk.mk_tail_record(plan, 4, 64)
    mk.mk_set_focal(plan, p.Gd, p.itd, p.shift, fbands)
    if tail is not None:
        mk.mk_iterate(plan, 4)
        mk.mk_tail_apply(plan, tail)
    norms = mk.mk_iterate(plan, p.niter if niter is None else niter)
    names = FIELD_NAMES + (("f2plus", "pminus") if aux else ())
    out = {k: mk.mk_get(plan, k, np.zeros(p.Gd.shape, np.float32)) for k in names}
    out["norms"] = norms
    out["image"] = mk.mk_image(plan)
    mk.mk_destroy(plan)
    return out


def _same_bits(a, b, label):
    for k in a:
        assert np.array_equal(a[k], b[k]), (label, k)


@pytest.mark.parametrize("rprec,nf,bands", [(0, 1, False), (1, 2, False), (0, 8, False), (1, 8, True),
                                            (2, 8, True)])
def test_streamed_equals_resident_and_oracle(rprec, nf, bands):
    mk = require_gpu()
    p = small_problem(seed=81, n=40, nt=128, nf=nf, niter=8)
    fb = None
    if bands:
        rng = np.random.default_rng(5)
        fb = np.stack([np.zeros(nf, np.int32), rng.integers(10, 65, nf).astype(np.int32)], axis=1)
    total = _r_bytes(p, rprec, nf)
    cap = total // 3               # two slab buffers of a sixth of R each: six or seven slabs
    say(f"streamed R: rprec {rprec}, nf {nf}, bands {bands}, R {total} bytes, cap {cap}")
    res = _solve(mk, p, 0, rprec, fbands=fb, aux=True)
    st = _solve(mk, p, cap, rprec, fbands=fb, aux=True)
    _same_bits(st, res, f"rprec{rprec}-nf{nf}")
    if rprec == 0:
        S = SynthesisOperator(p.Rhat, p.band, p.c, p.geom.nt)
        ref = marchenko(S, p.Gd, p.itd, p.shift, p.niter, fbands=fb)
        for k in FIELD_NAMES:
            e = max(rel_l2(st[k][f], ref[k][f]) for f in range(nf))
            say(f"  {k}: {e:.2e}")
            assert e <= TOL_FP32, (k, e)


@pytest.mark.parametrize("mode", [1, 2])
def test_streamed_tail_and_restart(mode):
    mk = require_gpu()
    p = small_problem(seed=82, n=32, nt=128, nf=3, niter=4)
    cap = _r_bytes(p, 0, 3) // 4
    res = _solve(mk, p, 0, tail=mode)
    st = _solve(mk, p, cap, tail=mode)
    _same_bits(st, res, f"tail{mode}")


def test_cap_exactly_at_R_keeps_it_resident_and_small_caps_are_refused():
    mk = require_gpu()
    p = small_problem(seed=83, n=24, nt=64, nf=1, niter=4)
    total = _r_bytes(p, 0, 1)
    a = _solve(mk, p, total)
    b = _solve(mk, p, 0)
    _same_bits(a, b, "cap=R")
    bin_bytes = total // p.Rhat.shape[1]
    nr, nt = p.Rhat.shape[0], p.geom.nt
    with pytest.raises(mk.MKError) as ei:
        mk.mk_plan(nr, nr, nt, p.geom.dt, p.geom.dx, band=p.band, r_dev_bytes=2 * bin_bytes - 1)
    assert ei.value.status == mk.MK_ERR_ARG
    # two bins fit: one-bin slabs, every bin its own copy
    c = _solve(mk, p, 2 * bin_bytes)
    _same_bits(c, b, "one-bin slabs")


def test_streamed_full_size_solve():
    """601 x 601, nt 2048, complex64 R of 2.96 GB under a 1 GB cap (six
    slabs): the whole 32-pass solve and the G assembly, against the oracle."""
    mk = require_gpu()
    import time

    import torch

    p = make_config("medium", nf=1)
    cap = 1 << 30
    say("medium nf=1 with R streamed under a 1 GiB device cap")
    nr, nt = p.Rhat.shape[0], p.geom.nt
    plan = mk.mk_plan(nr, nr, nt, p.geom.dt, p.geom.dx, band=p.band, r_dev_bytes=cap)
    mk.mk_load_R(plan, p.Rhat)
    Gd, itd = torch.from_numpy(p.Gd).cuda(), torch.from_numpy(p.itd).cuda()
    mk.mk_set_focal(plan, Gd, itd, p.shift)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    norms = mk.mk_iterate(plan, 32)
    t1 = time.perf_counter()
    got = {k: mk.mk_get(plan, k, np.zeros(p.Gd.shape, np.float32)) for k in FIELD_NAMES}
    mk.mk_destroy(plan)
    gbs = 32 * p.Rhat.nbytes / (t1 - t0) / 1e9
    say(f"  32 passes in {t1 - t0:.2f} s: R crosses PCIe at {gbs:.1f} GB/s")
    S = SynthesisOperator(p.Rhat, p.band, p.c, nt)
    ref = marchenko(S, p.Gd, p.itd, p.shift, 32)
    for k in FIELD_NAMES:
        e = rel_l2(got[k][0], ref[k][0])
        say(f"  {k}: {e:.2e}")
        assert e <= TOL_FP32, (k, e)
    ref_n = ref["norms"][:, 0]
    err = np.abs(norms[:, 0] - ref_n) / np.maximum(ref_n, 1e-3 * ref_n[0])
    assert err.max() <= 1e-5
