"""The library's own stopping rule (mk_iterate_tol) against the FP64 oracle.

The rule reads the FP64 norms of the series' last terms to estimate what the
terms not yet added still carry, relative to the smallest focusing function,
and keeps running passes until that estimate is within tol.  The oracle's
converged series (many more terms than any run here) is the truth: every
field of every focal point must be within tol of it when the rule stops,
for the plain series, after a geometric tail and restart, and for R = 0."""

import numpy as np
import pytest

from gpu_common import FIELD_NAMES, require_gpu, say
from mkgen.layered import small_problem
from oracle import SynthesisOperator, marchenko, rel_l2

pytestmark = pytest.mark.gpu


def _plan(mk, p, nf_max=None):
    nr, nt = p.Rhat.shape[0], p.geom.nt
    plan = mk.mk_plan(nr, nr, nt, p.geom.dt, p.geom.dx, band=p.band, nf_max=nf_max or p.nf)
    mk.mk_load_R(plan, p.Rhat)
    return plan


def _fields(mk, plan, p):
    return {k: mk.mk_get(plan, k, np.zeros(p.Gd.shape, np.float32)) for k in FIELD_NAMES}


def _worst(got, ref):
    return {k: max(rel_l2(got[k][f], ref[k][f]) for f in range(ref[k].shape[0])) for k in FIELD_NAMES}


@pytest.fixture(scope="module")
def problem():
    return small_problem(seed=61, n=40, nt=128, nf=6, niter=8, rho_target=0.7)


@pytest.fixture(scope="module")
def converged(problem):
    p = problem
    return marchenko(SynthesisOperator(p.Rhat, p.band, p.c, p.geom.nt), p.Gd, p.itd, p.shift, 80)


@pytest.mark.parametrize("tol", [1e-2, 1e-3, 1e-4])
def test_plain_series_stops_within_tol(problem, converged, tol):
    mk = require_gpu()
    p = problem
    plan = _plan(mk, p)
    mk.mk_set_focal(plan, p.Gd, p.itd, p.shift)
    n, est = mk.mk_iterate_tol(plan, tol, 60)
    got = _fields(mk, plan, p)
    assert mk.mk_passes(plan) == n
    # a second call finds nothing left to do
    n2, _ = mk.mk_iterate_tol(plan, tol, 60)
    mk.mk_destroy(plan)
    worst = _worst(got, converged)
    say(f"tol {tol:.0e}: {n} passes, estimate max {est.max():.2e}; " +
        ", ".join(f"{k}={v:.2e}" for k, v in worst.items()))
    assert n2 == 0
    assert np.all(est <= tol)
    for k, e in worst.items():
        assert e <= tol, (k, e)
    # and the rule does not run far past what the truth needs
    S = SynthesisOperator(p.Rhat, p.band, p.c, p.geom.nt)
    need = next(m for m in range(1, 61)
                if max(_worst(marchenko(S, p.Gd, p.itd, p.shift, m), converged).values()) <= tol)
    say(f"  the oracle's series reaches tol after {need} terms")
    assert n <= need + 4


@pytest.mark.parametrize("tol", [1e-3, 1e-4])
def test_after_geometric_tail_and_restart(problem, converged, tol):
    mk = require_gpu()
    p = problem
    plan = _plan(mk, p)
    mk.mk_tail_record(plan, 4, 64)
    mk.mk_set_focal(plan, p.Gd, p.itd, p.shift)
    mk.mk_iterate(plan, 4, want_norms=False)
    mk.mk_tail_apply(plan, mk.TAIL_GEOMETRIC)
    n, est = mk.mk_iterate_tol(plan, tol, 60)
    got = _fields(mk, plan, p)
    mk.mk_destroy(plan)
    worst = _worst(got, converged)
    say(f"tail, tol {tol:.0e}: {n} more passes, estimate max {est.max():.2e}; " +
        ", ".join(f"{k}={v:.2e}" for k, v in worst.items()))
    assert np.all(est <= tol)
    for k, e in worst.items():
        assert e <= tol, (k, e)


def test_zero_reflectivity_stops_after_two_passes(problem):
    mk = require_gpu()
    p = problem
    plan = mk.mk_plan(p.Rhat.shape[0], p.Rhat.shape[0], p.geom.nt, p.geom.dt, p.geom.dx, band=p.band,
                      nf_max=p.nf)
    mk.mk_load_R(plan, np.zeros_like(p.Rhat))
    mk.mk_set_focal(plan, p.Gd, p.itd, p.shift)
    n, est = mk.mk_iterate_tol(plan, 1e-6, 10)
    mk.mk_destroy(plan)
    assert n == 2 and not est.any()


def test_budget_and_arguments(problem):
    mk = require_gpu()
    p = problem
    plan = _plan(mk, p)
    mk.mk_set_focal(plan, p.Gd, p.itd, p.shift)
    n, est = mk.mk_iterate_tol(plan, 1e-12, 3)            # the budget runs out first
    assert n == 3 and est.max() > 1e-12
    for bad in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(mk.MKError) as ei:
            mk.mk_iterate_tol(plan, bad, 3)
        assert ei.value.status == mk.MK_ERR_ARG
    with pytest.raises(mk.MKError):
        mk.mk_iterate_tol(plan, 1e-3, -1)
    mk.mk_destroy(plan)


@pytest.mark.parametrize("tail", [None, "geometric"])
def test_fields_outside_the_mute_window_keep_their_start(problem, tail):
    """The rule reads only the mute windows of f1+ and f1- and adds the
    sums of squares of N_-1 outside them: that holds if nothing writes
    there.  Outside every trace's window f1+ must still be N_-1 = G_d(-t)
    and f1- zero, to the bit, after passes, a tail and its restart."""
    mk = require_gpu()
    p = problem
    plan = _plan(mk, p)
    mk.mk_tail_record(plan, 4, 64)
    mk.mk_set_focal(plan, p.Gd, p.itd, p.shift)
    mk.mk_iterate(plan, 4, want_norms=False)
    if tail is not None:
        mk.mk_tail_apply(plan, mk.TAIL_GEOMETRIC)
    mk.mk_iterate_tol(plan, 1e-5, 20)
    got = _fields(mk, plan, p)
    mk.mk_destroy(plan)
    nt = p.geom.nt
    k = np.arange(nt)
    L = np.minimum(p.itd.astype(np.int64) - p.shift, nt // 2)[..., None]
    outside = ~((k < L) | (k > nt - L))
    n_start = p.Gd[..., (-k) % nt]
    say(f"outside-window samples: {int(outside.sum())} of {outside.size}, tail {tail}")
    assert outside.any()
    assert np.array_equal(got["f1plus"][outside], n_start[outside])
    assert not got["f1minus"][outside].any()
