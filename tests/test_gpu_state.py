"""Checkpoint and resume of a running series (mk_get_state / mk_set_state),
and the total Green's function (MK_GTOTAL).

Resume: a series saved after some passes and restored into a fresh plan
continues with the same bits as the uninterrupted plan -- fields, norms and
the passes the stopping rule picks -- on the streaming GEMV (complex64), the
FP16 matrix-core batch with per-focal bands and one X plane, and a series
after a geometric tail and its restart (with iterates recorded).  Blobs of
another shape or a truncated blob are refused.

Total G: the Theory section reads G from the auxiliary fields f2+ and p-;
the oracle forms exactly that, p-(t) + S[N_last](t) + f2+(-t), and the
library returns G+ + G- (equal by Algorithm 1's signs, a pinned identity of
the oracle); both are compared at the FP32 bar.
"""

import numpy as np
import pytest

from gpu_common import FIELD_NAMES, TOL_FP32, require_gpu, say
from mkgen.layered import small_problem
from oracle import SynthesisOperator, marchenko, rel_l2

pytestmark = pytest.mark.gpu


def _plan(mk, p, rprec=0, flags=0, nf_max=None, record=False):
    nr, nt = p.Rhat.shape[0], p.geom.nt
    plan = mk.mk_plan(nr, nr, nt, p.geom.dt, p.geom.dx, band=p.band, nf_max=nf_max or p.nf, rprec=rprec,
                      flags=flags)
    mk.mk_load_R(plan, p.Rhat)
    if record:
        mk.mk_tail_record(plan, 4, 64)
    return plan


def _fields(mk, plan, p):
    return {k: mk.mk_get(plan, k, np.zeros(p.Gd.shape, np.float32)) for k in FIELD_NAMES}


def _start(mk, plan, p, fb, first, tail):
    mk.mk_set_focal(plan, p.Gd, p.itd, p.shift, fb)
    if tail:
        mk.mk_iterate(plan, 4)
        mk.mk_tail_apply(plan, mk.TAIL_GEOMETRIC)
    mk.mk_iterate(plan, first)


CASES = [  # (rprec, flags, nf, bands, tail)
    (0, 0, 2, False, False),
    (1, 0x8, 8, True, False),
    (0, 0, 3, False, True),
]


@pytest.mark.parametrize("rprec,flags,nf,bands,tail", CASES)
def test_resume_continues_bit_for_bit(rprec, flags, nf, bands, tail):
    mk = require_gpu()
    p = small_problem(seed=91, n=36, nt=128, nf=nf, niter=8)
    fb = None
    if bands:
        rng = np.random.default_rng(4)
        fb = np.stack([np.zeros(nf, np.int32), rng.integers(12, 65, nf).astype(np.int32)], axis=1)
    say(f"resume: rprec {rprec}, flags {flags:#x}, nf {nf}, bands {bands}, tail {tail}")
    a = _plan(mk, p, rprec, flags, record=tail)
    _start(mk, a, p, fb, 3, tail)
    blob = mk.mk_get_state(a)
    want_norms = mk.mk_iterate(a, 5)
    want = _fields(mk, a, p)
    want_n, _ = mk.mk_iterate_tol(a, 1e-4, 30)
    want_tol = _fields(mk, a, p)
    mk.mk_destroy(a)

    # a fresh plan with a wider batch limit that keeps the same layout of R
    b = _plan(mk, p, rprec, flags, nf_max=nf + 3 if nf > 4 else 4, record=tail)
    mk.mk_set_state(b, blob)
    assert mk.mk_passes(b) == 3 + (6 if tail else 0)
    got_norms = mk.mk_iterate(b, 5)
    got = _fields(mk, b, p)
    got_n, _ = mk.mk_iterate_tol(b, 1e-4, 30)
    got_tol = _fields(mk, b, p)
    mk.mk_destroy(b)
    assert np.array_equal(got_norms, want_norms)
    for k in FIELD_NAMES:
        assert np.array_equal(got[k], want[k]), k
        assert np.array_equal(got_tol[k], want_tol[k]), k
    assert got_n == want_n
    say(f"  identical after 5 more passes and {got_n} judged ones")


def test_resume_matches_the_oracle_series():
    mk = require_gpu()
    p = small_problem(seed=92, n=30, nt=128, nf=2, niter=8)
    a = _plan(mk, p)
    mk.mk_set_focal(a, p.Gd, p.itd, p.shift)
    mk.mk_iterate(a, 4)
    blob = mk.mk_get_state(a)
    mk.mk_destroy(a)
    b = _plan(mk, p)
    mk.mk_set_state(b, blob)
    mk.mk_iterate(b, 4)
    got = _fields(mk, b, p)
    mk.mk_destroy(b)
    ref = marchenko(SynthesisOperator(p.Rhat, p.band, p.c, p.geom.nt), p.Gd, p.itd, p.shift, 8)
    for k in FIELD_NAMES:
        e = max(rel_l2(got[k][f], ref[k][f]) for f in range(p.nf))
        assert e <= TOL_FP32, (k, e)


def test_foreign_or_truncated_blobs_are_refused():
    mk = require_gpu()
    p = small_problem(seed=93, n=24, nt=64, nf=2, niter=4)
    a = _plan(mk, p)
    mk.mk_set_focal(a, p.Gd, p.itd, p.shift)
    mk.mk_iterate(a, 2)
    blob = mk.mk_get_state(a)
    for bad in (blob[:len(blob) - 8], b"XXXXXXXX" + blob[8:]):
        with pytest.raises(mk.MKError) as ei:
            mk.mk_set_state(a, bad)
        assert ei.value.status == mk.MK_ERR_ARG
    mk.mk_destroy(a)
    q = small_problem(seed=93, n=24, nt=128, nf=2, niter=4)     # another nt
    c = _plan(mk, q)
    with pytest.raises(mk.MKError) as ei:
        mk.mk_set_state(c, blob)
    assert ei.value.status == mk.MK_ERR_ARG
    d = _plan(mk, p, nf_max=1)                                     # nf above nf_max
    with pytest.raises(mk.MKError) as ei:
        mk.mk_set_state(d, blob)
    assert ei.value.status == mk.MK_ERR_ARG
    mk.mk_destroy(c)
    mk.mk_destroy(d)


@pytest.mark.parametrize("nf", [1, 6])
def test_total_G_against_the_oracle(nf):
    mk = require_gpu()
    p = small_problem(seed=94, n=28, nt=128, nf=nf, niter=8)
    plan = _plan(mk, p)
    mk.mk_set_focal(plan, p.Gd, p.itd, p.shift)
    mk.mk_iterate(plan, p.niter)
    g = mk.mk_get(plan, "Gtotal", np.zeros(p.Gd.shape, np.float32))
    f = _fields(mk, plan, p)
    mk.mk_destroy(plan)
    ref = marchenko(SynthesisOperator(p.Rhat, p.band, p.c, p.geom.nt), p.Gd, p.itd, p.shift, p.niter)
    e = max(rel_l2(g[j], ref["Gtotal"][j]) for j in range(nf))
    say(f"total G (nf {nf}): {e:.2e} against the oracle's p- + S N_last + f2+(-t)")
    assert e <= TOL_FP32
    assert np.array_equal(g, f["Gplus"] + f["Gminus"])
