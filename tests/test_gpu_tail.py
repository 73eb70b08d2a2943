"""The series-tail path on the GPU against the FP64 reference: recorded
iterates, the restart on the fixed-point residual, geometric and network
tails (bar 1e-5 relative L2, complex64 R)."""

import numpy as np
import pytest

from gpu_common import FIELD_NAMES, require_gpu, say
from mkgen.layered import small_problem
from oracle import SynthesisOperator, marchenko, rel_l2
from oracle import tail as ot
from oracle import tailnet as tn

pytestmark = pytest.mark.gpu
K, T = 4, 64


def _gpu(p, mode, m, params=None, tune=None, rprec=0, k=K, T=T):
    mk = require_gpu()
    nr, nt = p.Rhat.shape[0], p.geom.nt
    plan = mk.mk_plan(nr, nr, nt, p.geom.dt, p.geom.dx, band=p.band, nf_max=p.nf, rprec=rprec)
    mk.mk_load_R(plan, p.Rhat)
    if tune is not None:
        mk.mk_tune(plan, tune)
    mk.mk_tail_record(plan, k, T)
    if params is not None:
        mk.mk_tail_load(plan, params)
    mk.mk_set_focal(plan, p.Gd, p.itd, p.shift)
    mk.mk_iterate(plan, k)
    hist = mk.mk_tail_history(plan)
    res = mk.mk_tail_apply(plan, mode)
    norms = mk.mk_iterate(plan, m) if m else None
    out = {k: mk.mk_get(plan, k, np.zeros(p.Gd.shape, np.float32)) for k in FIELD_NAMES}
    out.update(hist=hist, res=res, norms=norms, passes=mk.mk_passes(plan))
    mk.mk_destroy(plan)
    return out


def _ref(p, mode, m, P=None, k=K, T=T, f16=False):
    S = SynthesisOperator(p.Rhat, p.band, p.c, p.geom.nt)
    a = marchenko(S, p.Gd, p.itd, p.shift, k, keep_iterates=True)
    hist = ot.history(a["iterates"], k, T)
    f1p, f1m = a["f1plus"], a["f1minus"]
    if mode == 1:
        te, to = ot.geometric_tails(hist)
        f1p, f1m = ot.apply_tails(f1p, f1m, te, to, p.itd, p.shift)
    elif mode == 0:
        te, to = ot.net_tails(hist, P, f16=f16)
        f1p, f1m = ot.apply_tails(f1p, f1m, te, to, p.itd, p.shift)
    f1p, f1m, rho, norms = ot.restart(S, p.Gd, p.itd, p.shift, f1p, niter=m)
    gp, gm = ot.g_fields(S, f1p, f1m)
    res = np.linalg.norm(rho.reshape(p.nf, -1), axis=1) / np.linalg.norm(p.Gd.reshape(p.nf, -1), axis=1)
    return dict(f1plus=f1p, f1minus=f1m, Gplus=gp, Gminus=gm, hist=hist, res=res, norms=norms)


def _compare(g, r, label, tol=1e-5):
    for key in FIELD_NAMES:
        e = max(rel_l2(g[key][f], r[key][f]) for f in range(r[key].shape[0]))
        say(f"  {label} {key}: {e:.2e}")
        assert e <= tol, (label, key, e)
    e = rel_l2(g["hist"], r["hist"])
    assert e <= tol, ("hist", e)
    np.testing.assert_allclose(g["res"], r["res"], rtol=1e-4, atol=1e-9)


@pytest.mark.parametrize("mode", [2, 1])
def test_restart_and_geometric_tail(mode):
    say(f"tail mode {mode}")
    p = small_problem(seed=71, n=24, nt=128, nf=2, niter=8)
    g = _gpu(p, mode, 3)
    _compare(g, _ref(p, mode, 3), f"mode{mode}")
    assert g["passes"] == K + 2 + 3


def test_no_tail_restart_equals_plain_passes():
    mk = require_gpu()
    say("restart == plain")
    p = small_problem(seed=72, n=24, nt=128, nf=2, niter=8)
    g = _gpu(p, 2, 3)
    from gpu_common import run_gpu

    plain = run_gpu(p, niter=K + 2 + 3)
    for key in FIELD_NAMES:
        assert rel_l2(g[key], plain[key]) <= 2e-6, key
    # the residual is N'' - (N_1 + N_3) formed by cancellation in FP32, so the
    # continued terms carry about u / rho^k relative error (rounding only)
    np.testing.assert_allclose(g["norms"], plain["norms"][K + 2:], rtol=1e-3)


def _bf16_net(rng, k, hidden):
    """Random network weights (FP32 vector) and their BF16-rounded FP64 copy."""
    P = tn.init_params(rng, k=k, hidden=hidden)
    P["W3"] *= 5.0
    P["b3"] = 0.01 * rng.standard_normal(2)
    flat = np.concatenate([P["W1"].ravel(), P["b1"], P["W2"].ravel(), P["b2"], P["W3"].ravel(), P["b3"]])
    flat = flat.astype(np.float32)
    u = flat.view(np.uint32).astype(np.uint64)
    rounded = (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16).astype(np.uint32).view(np.float32)
    Pr, o = {}, 0
    for key in ("W1", "b1", "W2", "b2", "W3", "b3"):
        n = P[key].size
        Pr[key] = rounded[o:o + n].astype(np.float64).reshape(P[key].shape)
        o += n
    return flat, Pr


@pytest.mark.parametrize("tune,hidden", [(None, 64), (1, 64), (None, 12), (None, 16)])
def test_network_tail_matches_reference(tune, hidden):
    """Hidden width 16 takes the one-kernel form (half-precision activations on
    the matrix cores, the tail applied in the same kernel; the oracle's
    half-precision inference form), the others go layer by layer in FP32."""
    say(f"network tail, contraction {tune}, hidden {hidden}")
    flat, Pr = _bf16_net(np.random.default_rng(5), K, hidden)
    p = small_problem(seed=73, n=20, nt=128, nf=3, niter=8)
    g = _gpu(p, 0, 2, params=flat, tune=tune)
    _compare(g, _ref(p, 0, 2, Pr, f16=hidden == 16), "net", tol=2e-5)


@pytest.mark.parametrize("k,T,nt,n,nf", [(6, 128, 128, 20, 3), (13, 32, 256, 16, 2), (4, 600, 2048, 24, 8),
                                         (8, 1024, 2048, 16, 4), (3, 64, 64, 12, 2)])
def test_fused_network_tail_shapes(k, T, nt, n, nf):
    """The one-kernel network tail (hidden 16) over input widths that pad to
    4, 8 and 16 channels, windows of one to four 256-sample tiles with a
    ragged last tile, and mute windows that leave some tiles out."""
    say(f"fused network tail k {k} T {T} nt {nt} n {n} nf {nf}")
    flat, Pr = _bf16_net(np.random.default_rng(9 + k), k, 16)
    p = small_problem(seed=80 + k, n=n, nt=nt, nf=nf, niter=k + 4)
    g = _gpu(p, 0, 2, params=flat, k=k, T=T)
    _compare(g, _ref(p, 0, 2, Pr, k=k, T=T, f16=True), f"fused k{k}", tol=2e-5)


@pytest.mark.parametrize("mode,nt", [(1, 2048), (2, 2048), (1, 4096)])
def test_tail_one_wave_per_trace(mode, nt):
    """2048 traces at nt 2048 and 4096: the restart kernels in their
    one-wave-per-trace (fused) form, geometric tail and restart alone."""
    say(f"tail one wave per trace, mode {mode}, nt {nt}")
    p = small_problem(seed=77, n=32, nt=nt, nf=64, niter=8)
    g = _gpu(p, mode, 2)
    _compare(g, _ref(p, mode, 2), f"wave-per-trace mode {mode}", tol=2e-5)


def test_tail_state_errors():
    mk = require_gpu()
    p = small_problem(seed=74, n=8, nt=64, nf=1)
    plan = mk.mk_plan(8, 8, 64, p.geom.dt, p.geom.dx)
    mk.mk_load_R(plan, p.Rhat)
    with pytest.raises(mk.MKError) as ei:
        mk.mk_tail_load(plan, np.zeros(mk.mk_net_param_count(4, 64), np.float32))
    assert ei.value.status == mk.MK_ERR_STATE
    mk.mk_tail_record(plan, 4, 32)
    with pytest.raises(mk.MKError):
        mk.mk_tail_load(plan, np.zeros(7, np.float32))
    mk.mk_set_focal(plan, p.Gd, p.itd, p.shift)
    mk.mk_iterate(plan, 3)
    with pytest.raises(mk.MKError) as ei:
        mk.mk_tail_apply(plan, 2)                      # only 3 of 4 passes
    assert ei.value.status == mk.MK_ERR_STATE
    mk.mk_iterate(plan, 1)
    with pytest.raises(mk.MKError) as ei:
        mk.mk_tail_apply(plan, 0)                      # no network loaded
    assert ei.value.status == mk.MK_ERR_STATE
    mk.mk_tail_apply(plan, 2)
    with pytest.raises(mk.MKError) as ei:
        mk.mk_tail_apply(plan, 2)                      # once per series
    assert ei.value.status == mk.MK_ERR_STATE
    mk.mk_destroy(plan)


@pytest.mark.parametrize("rprec", [1, 2])
def test_restart_then_G_with_16bit_R(rprec):
    """16-bit R: after the restart the series' X scale is the (small) residual
    norm; the G assembly must keep f1+ and f1- on the scale of G_d, or its
    16-bit spectra overflow.  Three focal points put G (six columns) on the
    matrix cores with 16-bit X."""
    say(f"restart + G, rprec {rprec}")
    p = small_problem(seed=75, n=24, nt=128, nf=3, niter=8)
    g = _gpu(p, 1, 2, rprec=rprec)
    r = _ref(p, 1, 2)
    tol = {1: 2e-3, 2: 2e-2}[rprec]
    for key in FIELD_NAMES:
        assert np.all(np.isfinite(g[key])), key
        e = max(rel_l2(g[key][f], r[key][f]) for f in range(p.nf))
        say(f"  {key}: {e:.2e}")
        assert e <= tol, (key, e)
