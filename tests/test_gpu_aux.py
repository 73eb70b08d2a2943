"""The auxiliary fields of Algorithm 1's second loop, f2+ and p-, against the
FP64 oracle (relative L2 per focal point: 1e-5 for the FP32 paths, 1e-3 for
FP16 R), including the empty series, continuation after the request, and the
refusal after a series tail."""

import numpy as np
import pytest

from gpu_common import FIELD_NAMES, require_gpu, say
from mkgen.layered import small_problem
from oracle import SynthesisOperator, marchenko, rel_l2

pytestmark = pytest.mark.gpu


def _plan(p, rprec=0, flags=0):
    mk = require_gpu()
    nr, nt = p.Rhat.shape[0], p.geom.nt
    plan = mk.mk_plan(nr, nr, nt, p.geom.dt, p.geom.dx, band=p.band, nf_max=p.nf, rprec=rprec, flags=flags)
    mk.mk_load_R(plan, p.Rhat)
    mk.mk_set_focal(plan, p.Gd, p.itd, p.shift)
    return mk, plan


def _get(mk, plan, p, name):
    return mk.mk_get(plan, name, np.zeros((p.nf, p.Rhat.shape[0], p.geom.nt), np.float32))


def _ref(p, niter):
    return marchenko(SynthesisOperator(p.Rhat, p.band, p.c, p.geom.nt), p.Gd, p.itd, p.shift, niter)


def _check(got, want, tol, label):
    e = max(rel_l2(got[f], want[f]) for f in range(want.shape[0]))
    say(f"  {label}: {e:.2e}")
    assert e <= tol, (label, e)


@pytest.mark.parametrize("niter", [7, 8])
def test_aux_fields_fp32(niter):
    say(f"aux fields, GEMV path, {niter} passes")
    p = small_problem(seed=95, n=24, nt=128, nf=3, niter=niter)
    mk, plan = _plan(p)
    mk.mk_iterate(plan, niter)
    got = {k: _get(mk, plan, p, k) for k in ("f2plus", "pminus")}
    # the request must not disturb the series: continue and compare
    mk.mk_iterate(plan, 2)
    cont = {k: _get(mk, plan, p, k) for k in FIELD_NAMES}
    mk.mk_destroy(plan)
    ref = _ref(p, niter)
    _check(got["f2plus"], ref["f2p"], 1e-5, "f2+")
    _check(got["pminus"], ref["pmin"], 1e-5, "p-")
    ref2 = _ref(p, niter + 2)
    for k in FIELD_NAMES:
        _check(cont[k], ref2[k], 1e-5, f"continued {k}")


@pytest.mark.parametrize("rprec,tol", [(0, 1e-5), (1, 1e-3)])
def test_aux_fields_batched(rprec, tol):
    say(f"aux fields, matrix cores, rprec {rprec}")
    p = small_problem(seed=96, n=48, nt=256, nf=12, niter=6)
    mk, plan = _plan(p, rprec=rprec)
    mk.mk_iterate(plan, 6)
    got = {k: _get(mk, plan, p, k) for k in ("f2plus", "pminus")}
    mk.mk_destroy(plan)
    ref = _ref(p, 6)
    _check(got["f2plus"], ref["f2p"], tol, f"f2+ r{rprec}")
    _check(got["pminus"], ref["pmin"], tol, f"p- r{rprec}")


def test_aux_fields_before_any_pass_and_after_a_tail():
    say("aux fields: empty series, and refused after a tail")
    p = small_problem(seed=97, n=16, nt=128, nf=2, niter=4)
    mk, plan = _plan(p)
    f2 = _get(mk, plan, p, "f2plus")
    pm = _get(mk, plan, p, "pminus")
    ref1 = _ref(p, 1)                      # p- after one pass is RN_0 = S N_-1: the scale of the check
    np.testing.assert_array_equal(f2, p.Gd[..., (-np.arange(p.geom.nt)) % p.geom.nt])
    for f in range(p.nf):
        assert np.linalg.norm(pm[f]) <= 1e-5 * np.linalg.norm(ref1["pmin"][f])
    mk.mk_tail_record(plan, 4, 32)
    mk.mk_set_focal(plan, p.Gd, p.itd, p.shift)
    mk.mk_iterate(plan, 4)
    mk.mk_tail_apply(plan, mk.TAIL_GEOMETRIC)
    for name in ("f2plus", "pminus"):
        with pytest.raises(mk.MKError) as ei:
            _get(mk, plan, p, name)
        assert ei.value.status == mk.MK_ERR_STATE
    mk.mk_destroy(plan)
