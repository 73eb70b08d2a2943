"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bar: relative L2 <= 1e-5 for each of f1+, f1-, G+, G- and each focal point
(the FP32 tolerance of the plain path), the series norms to the same
relative accuracy, and bitwise reproducibility run to run.
"""

import json
import os

import numpy as np
import pytest

from gpu_common import FIELD_NAMES, TOL_FP32, assert_parity, require_gpu, run_gpu, run_oracle, say
from mkgen.layered import make_config, small_problem

pytestmark = pytest.mark.gpu


def _norm_check(g, r, tol=TOL_FP32):
    scale = np.maximum(r.max(axis=0, keepdims=True), 1e-30)
    err = np.abs(g - r) / scale
    assert err.max() <= tol, f"norms off by {err.max():.3e}"


@pytest.mark.parametrize("seed,n,nt,nf", [(0, 8, 64, 1), (1, 12, 128, 3), (2, 5, 32, 2), (3, 33, 256, 2)])
def test_small_problems(seed, n, nt, nf):
    say(f"small problem seed={seed} n={n} nt={nt} nf={nf}")
    p = small_problem(seed=seed, n=n, nt=nt, nf=nf, niter=8, rho_target=0.6)
    g = run_gpu(p)
    r = run_oracle(p)
    assert_parity(g, r, label=f"small{seed}")
    _norm_check(g["norms"], r["norms"])
    assert g["passes"] == 8


@pytest.mark.parametrize("nt", [128, 256, 1024, 2048, 4096])
def test_one_wave_per_trace(nt):
    """2048 traces: the one-wave-per-trace epilogue at every transform length
    (the fused pass at nt 2048 and 4096), with the G assembly."""
    say(f"one wave per trace nt={nt}")
    p = small_problem(seed=40 + nt % 97, n=32, nt=nt, nf=64, niter=5, rho_target=0.6)
    g = run_gpu(p)
    r = run_oracle(p)
    assert_parity(g, r, label=f"wave-per-trace nt{nt}")
    _norm_check(g["norms"], r["norms"])


def test_hand_derived_spike_cases(golden_dir):
    """The closed-form worked examples of tests/golden, run on the GPU."""
    import cmath
    import math

    from mkgen.layered import Geometry, LayerModel, Problem

    for name, spikes_of in (("single_interface.json", lambda c: [(c["k1"], c["r"])]),
                            ("two_interfaces.json", lambda c: [(c["k1"], c["r1"]), (c["k2"], c["r2"])])):
        case = json.load(open(os.path.join(golden_dir, name)))
        nt = case["nt"]
        say(f"spike case {name}")
        Rhat = np.array([sum(a * cmath.exp(-2j * math.pi * w * k / nt) for k, a in spikes_of(case))
                         for w in range(nt // 2 + 1)], dtype=np.complex64).reshape(1, -1, 1)
        Gd = np.zeros((1, 1, nt), dtype=np.float32)
        Gd[0, 0, case["kd"]] = 1.0
        geom = Geometry(n=1, dx=1.0, nt=nt, dt=1.0)
        p = Problem(name=name, geom=geom, model=LayerModel(np.zeros(0), np.ones(1), np.zeros(0)),
                    Rhat=Rhat, band=(0, nt // 2), Gd=Gd, itd=np.array([[case["kd"]]], np.int32),
                    shift=case["shift"], niter=case["niter"])
        g = run_gpu(p)
        for key in ("f1plus", "f1minus", "Gplus", "Gminus"):
            want = np.zeros(nt)
            for k, a in case["expected"][key].items():
                want[int(k) % nt] += a
            np.testing.assert_allclose(g[key][0, 0], want, atol=2e-6, err_msg=f"{name} {key}")
        np.testing.assert_allclose(g["norms"][:, 0], case["expected"]["norms"], atol=2e-6)


def test_tiny_config_full_solve():
    """101 x 101, nt 512, 3 flat layers, one focal point, 16 passes."""
    say("tiny config")
    p = make_config("tiny")
    g = run_gpu(p)
    r = run_oracle(p)
    assert_parity(g, r, label="tiny")
    _norm_check(g["norms"], r["norms"])


def test_per_focal_bands_and_device_inputs():
    say("per-focal bands")
    p = small_problem(seed=5, n=16, nt=128, nf=3, niter=6)
    fb = np.array([[0, 20], [5, 64], [10, 40]], dtype=np.int32)
    g = run_gpu(p, fbands=fb)
    r = run_oracle(p, fbands=fb)
    assert_parity(g, r, label="bands")
    gd = run_gpu(p, fbands=fb, on_device=True)
    for k in FIELD_NAMES:
        assert np.array_equal(g[k], gd[k]), k


def test_sub_band_plan():
    say("sub-band plan")
    p = small_problem(seed=6, n=10, nt=64, nf=2, niter=6, band=(3, 25))
    assert p.Rhat.shape[1] == 23
    assert_parity(run_gpu(p), run_oracle(p), label="subband")


def test_continuation_and_determinism():
    say("continuation")
    p = small_problem(seed=7, n=16, nt=128, nf=2, niter=8)
    a = run_gpu(p, chunks=[8])
    b = run_gpu(p, chunks=[3, 0, 5])
    c = run_gpu(p, chunks=[8])
    d = run_gpu(p, chunks=[2, "G", 3, "G", 3])
    assert b["passes"] == 8
    for k in FIELD_NAMES:
        assert np.array_equal(a[k], b[k]), k
        assert np.array_equal(a[k], c[k]), k
        assert np.array_equal(a[k], d[k]), k
    assert np.array_equal(a["norms"], b["norms"])
    assert np.array_equal(a["norms"], d["norms"])


def test_zero_passes_and_zero_R():
    say("zero passes / zero R")
    p = small_problem(seed=8, n=8, nt=64, nf=1)
    g = run_gpu(p, niter=0)
    r = run_oracle(p, niter=0)
    assert_parity(g, r, label="zero-passes")
    z = run_gpu(p, R=np.zeros_like(p.Rhat), niter=4)
    Gd = p.Gd.astype(np.float32)
    assert np.array_equal(z["Gplus"], Gd)
    assert not z["f1minus"].any() and not z["Gminus"].any() and not z["norms"].any()


def test_error_paths():
    mk = require_gpu()
    say("error paths")
    p = small_problem(seed=9, n=8, nt=64)
    plan = mk.mk_plan(8, 8, 64, p.geom.dt, p.geom.dx, nf_max=2)
    with pytest.raises(mk.MKError) as ei:
        mk.mk_set_focal(plan, p.Gd, p.itd, p.shift)
    assert ei.value.status == mk.MK_ERR_STATE
    bad = p.Rhat.copy()
    bad[0, 3, 2] = np.nan
    with pytest.raises(mk.MKError) as ei:
        mk.mk_load_R(plan, bad)
    assert ei.value.status == mk.MK_ERR_ARG
    mk.mk_load_R(plan, p.Rhat)
    with pytest.raises(mk.MKError) as ei:
        mk.mk_iterate(plan, 1)
    assert ei.value.status == mk.MK_ERR_STATE
    g = p.Gd.copy()
    g[0, 1, 1] = np.inf
    with pytest.raises(mk.MKError) as ei:
        mk.mk_set_focal(plan, g, p.itd, p.shift)
    assert ei.value.status == mk.MK_ERR_ARG
    with pytest.raises(ValueError):            # the binding checks nf against nf_max first
        mk.mk_set_focal(plan, np.zeros((3, 8, 64), np.float32), np.zeros((3, 8), np.int32), 1)
    g3, i3 = np.zeros((3, 8, 64), np.float32), np.zeros((3, 8), np.int32)
    st = mk.load_library().mk_set_focal(plan.handle, 3, g3.ctypes.data, i3.ctypes.data, 1, None, 0)
    assert st == mk.MK_ERR_ARG                 # and so does the library
    with pytest.raises(mk.MKError) as ei:
        mk.mk_set_focal(plan, p.Gd, p.itd, p.shift, np.array([[0, 40]], np.int32))
    assert ei.value.status == mk.MK_ERR_ARG
    mk.mk_destroy(plan)


def test_device_inputs_and_outputs():
    """Device G_d / itd / bands and device outputs: the same values as the host
    path; a non-finite device G_d is refused and leaves no focal points set."""
    mk = require_gpu()
    import torch

    say("device inputs and outputs")
    p = small_problem(seed=12, n=24, nt=128, nf=5, niter=4)
    band = np.array([[2, 60], [0, 64], [5, 40], [1, 64], [3, 50]], np.int32)
    plan = mk.mk_plan(24, 24, 128, p.geom.dt, p.geom.dx, band=p.band, nf_max=5)
    mk.mk_load_R(plan, p.Rhat)
    mk.mk_set_focal(plan, p.Gd, p.itd, p.shift, band)
    mk.mk_iterate(plan, 4)
    host = {k: mk.mk_get(plan, k, np.zeros(p.Gd.shape, np.float32)) for k in ("f1plus", "Gminus")}
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()      # noqa: E731
    mk.mk_set_focal(plan, d(p.Gd), d(p.itd), p.shift, d(band))
    mk.mk_iterate(plan, 4)
    for k in ("f1plus", "Gminus"):
        out = torch.empty(p.Gd.shape, dtype=torch.float32, device="cuda")
        mk.mk_get(plan, k, out)
        assert np.array_equal(out.cpu().numpy(), host[k]), k
    for bad in (np.inf, np.nan):
        g = p.Gd.copy()
        g[3, 7, 11] = bad
        with pytest.raises(mk.MKError) as ei:
            mk.mk_set_focal(plan, d(g), d(p.itd), p.shift, d(band))
        assert ei.value.status == mk.MK_ERR_ARG
        with pytest.raises(mk.MKError) as ei:
            mk.mk_iterate(plan, 1)
        assert ei.value.status == mk.MK_ERR_STATE
    mk.mk_set_focal(plan, d(p.Gd), d(p.itd), p.shift, d(band))
    mk.mk_iterate(plan, 4)
    assert np.array_equal(mk.mk_get(plan, "f1plus", np.zeros(p.Gd.shape, np.float32)), host["f1plus"])
    mk.mk_destroy(plan)


def test_divergence_is_reported():
    mk = require_gpu()
    say("divergence")
    p = small_problem(seed=10, n=8, nt=64, rho_target=None)
    # scale R so the Neumann operator is far from a contraction
    R = p.Rhat * np.float32(8.0 / max(p.rho * p.rscale, 1e-30) if p.rho else 1.0)
    plan = mk.mk_plan(8, 8, 64, p.geom.dt, p.geom.dx, nf_max=1, div_factor=10.0)
    mk.mk_load_R(plan, R)
    mk.mk_set_focal(plan, p.Gd, p.itd, p.shift)
    with pytest.raises(mk.MKError) as ei:
        mk.mk_iterate(plan, 40)
    assert ei.value.status == mk.MK_ERR_DIVERGED
    # the stopping rule's passes: the judge applies the same check
    mk.mk_set_focal(plan, p.Gd, p.itd, p.shift)
    with pytest.raises(mk.MKError) as ei:
        mk.mk_iterate_tol(plan, 1e-9, 40)
    assert ei.value.status == mk.MK_ERR_DIVERGED
    mk.mk_destroy(plan)
