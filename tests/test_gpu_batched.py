"""Batched focal points on the matrix cores, reduced-precision R, per-focal
bands and the contraction autotuner, each against the FP64 oracle.

Bars: 1e-5 relative L2 for complex64 R (every contraction variant the
autotuner may pick), 1e-3 for FP16 R, 1e-2 for BF16 R.  BF16's unit
roundoff is 3.9e-3, and G- nearly cancels (it is S f1+ - f1- of two much
larger fields), so its relative error reaches a few 1e-3; the measured
errors are printed.
"""

import numpy as np
import pytest

from gpu_common import TOL_FP32, assert_parity, require_gpu, run_gpu, run_oracle, say
from mkgen.layered import make_config, small_problem

pytestmark = pytest.mark.gpu

TOL = {0: TOL_FP32, 1: 1e-3, 2: 1e-2}


def _flags(variant, tiled):
    """Row-major R for the variants that read only that layout (plans with nf > 4 tile R by default)."""
    mk = require_gpu()
    return 0 if tiled else mk.MK_FLAG_ROW_R


@pytest.mark.parametrize("variant,tiled", [(v, False) for v in range(9)] + [(v, True) for v in (6, 7, 8)])
@pytest.mark.parametrize("n,nt,nf", [(70, 64, 6), (37, 128, 40), (300, 32, 20), (250, 64, 20)])
def test_every_contraction_variant_fp32(variant, tiled, n, nt, nf):
    """Every variant against the oracle.  The LDS-staged tiles with two waves
    per SIMD (variants 7, 8) run blocks of two waves (128 receivers) where
    that pads fewer receiver rows (70, 37, 300 receivers) and of four
    otherwise (250 receivers, and the 128-row tiles of variant 6)."""
    say(f"variant {variant} tiled {tiled} n={n} nt={nt} nf={nf}")
    p = small_problem(seed=20 + nf, n=n, nt=nt, nf=nf, niter=6)
    g = run_gpu(p, tune=variant, flags=_flags(variant, tiled))
    assert g["variant"] == variant
    assert_parity(g, run_oracle(p), label=f"v{variant}{'t' if tiled else ''}")


def test_row_major_variant_refused_on_tiled_plan():
    mk = require_gpu()
    plan = mk.mk_plan(16, 16, 64, 0.004, 10.0, nf_max=8)
    with pytest.raises(mk.MKError):
        mk.mk_tune(plan, 1)
    mk.mk_tune(plan, 7)
    mk.mk_destroy(plan)


@pytest.mark.parametrize("rprec", [1, 2])
@pytest.mark.parametrize("variant,tiled", [(0, False), (1, False), (4, False), (7, False), (6, True), (7, True),
                                           (8, True)])
def test_reduced_precision_R(rprec, variant, tiled):
    say(f"rprec {rprec} variant {variant} tiled {tiled}")
    p = small_problem(seed=31, n=48, nt=128, nf=20, niter=8)
    g = run_gpu(p, rprec=rprec, tune=variant, flags=_flags(variant, tiled))
    assert_parity(g, run_oracle(p), tol=TOL[rprec], label=f"prec{rprec}-v{variant}")


@pytest.mark.parametrize("rprec", [1, 2])
@pytest.mark.parametrize("nf", [1, 2, 3, 5])
def test_reduced_precision_gemv_few_columns(rprec, nf):
    """16-bit R through the streaming contraction with one to five focal
    columns: the one-, two- and four-column run shapes alone and together in
    one pass (the G assembly doubles the columns), on a row count (37
    receivers x 65 bins) that no run length divides."""
    mk = require_gpu()
    say(f"gemv rprec {rprec} nf {nf}")
    p = small_problem(seed=60 + nf, n=37, nt=128, nf=nf, niter=6)
    g = run_gpu(p, rprec=rprec, tune=0, flags=mk.MK_FLAG_ROW_R)
    assert g["variant"] == 0
    assert_parity(g, run_oracle(p), tol=TOL[rprec], label=f"gemv{rprec}-nf{nf}")


@pytest.mark.parametrize("rprec", [1, 2])
@pytest.mark.parametrize("variant", [1, 6])
def test_single_plane_16bit_X(rprec, variant):
    """MK_FLAG_FAST_X: one 16-bit plane of X (half the products, about twice the error)."""
    mk = require_gpu()
    say(f"fast X rprec {rprec} variant {variant}")
    p = small_problem(seed=31, n=48, nt=128, nf=20, niter=8)
    g = run_gpu(p, rprec=rprec, tune=variant, flags=mk.MK_FLAG_FAST_X | _flags(variant, variant >= 6))
    assert_parity(g, run_oracle(p), tol=2 * TOL[rprec], label=f"fastx{rprec}-v{variant}")


@pytest.mark.parametrize("rprec,variant", [(0, 1), (0, 0), (1, 1), (2, 5), (0, 6), (1, 6), (2, 8)])
def test_per_focal_bands_batched(rprec, variant):
    say(f"bands rprec {rprec} variant {variant}")
    p = small_problem(seed=41, n=50, nt=128, nf=24, niter=6)
    rng = np.random.default_rng(3)
    hi = rng.integers(10, 65, size=p.nf)
    lo = np.where(rng.random(p.nf) < 0.3, rng.integers(0, 8, size=p.nf), 0)
    fb = np.stack([lo, hi], axis=1).astype(np.int32)
    g = run_gpu(p, fbands=fb, rprec=rprec, tune=variant, flags=_flags(variant, variant >= 6))
    assert_parity(g, run_oracle(p, fbands=fb), tol=TOL[rprec], label=f"bands{rprec}-{variant}")


def test_autotuner_choice_passes_parity(tmp_path, monkeypatch):
    mk = require_gpu()
    say("autotune")
    monkeypatch.setenv("MK_TUNE_CACHE", str(tmp_path / "tune.txt"))
    p = small_problem(seed=51, n=64, nt=128, nf=12, niter=5)
    g = run_gpu(p, flags=mk.MK_FLAG_AUTOTUNE)
    assert 0 <= g["variant"] <= 8
    assert_parity(g, run_oracle(p), label="autotune")
    text = (tmp_path / "tune.txt").read_text()
    assert "ncols=12" in text and "ncols=24" in text
    g2 = run_gpu(p, flags=mk.MK_FLAG_AUTOTUNE)        # choices now come from the cache file
    assert g2["variant"] == g["variant"]
    for k in ("f1plus", "Gplus"):
        assert np.array_equal(g[k], g2[k])


@pytest.mark.parametrize("rprec", [0, 1])
def test_autotuner_with_bands(tmp_path, monkeypatch, rprec):
    """Bands make the LDS-staged contraction walk its active tiles by default;
    with the autotuner timing the variants on first use, whichever variant
    it picks (walking or not) must keep parity."""
    mk = require_gpu()
    say(f"autotune with bands, rprec {rprec}")
    monkeypatch.setenv("MK_TUNE_CACHE", str(tmp_path / "tune.txt"))
    p = small_problem(seed=52, n=48, nt=128, nf=20, niter=5)
    rng = np.random.default_rng(9)
    fb = np.stack([np.zeros(p.nf, np.int32), rng.integers(10, 65, p.nf).astype(np.int32)], axis=1)
    g = run_gpu(p, fbands=fb, rprec=rprec, flags=mk.MK_FLAG_AUTOTUNE)
    assert_parity(g, run_oracle(p, fbands=fb), tol=TOL[rprec], label=f"autotune-bands{rprec}")


def test_medium_focal_line_batched():
    """601 x 601, nt 2048, 64 focal points: FP32 and FP16 batched, first 2 passes."""
    say("medium nf=64 batched")
    p = make_config("medium", nf=64)
    r = run_oracle(p, niter=2)
    g = run_gpu(p, niter=2)
    assert g["variant"] != 0
    assert_parity(g, r, label="medium64-fp32")
    g16 = run_gpu(p, niter=2, rprec=1)
    assert_parity(g16, r, tol=1e-3, label="medium64-fp16")
    for v, tiled in ((6, True), (7, True), (7, False), (1, False)):   # both kernel families, both layouts
        gv = run_gpu(p, niter=2, rprec=1, tune=v, flags=_flags(v, tiled))
        assert gv["variant"] == v
        assert_parity(gv, r, tol=1e-3, label=f"medium64-fp16-v{v}{'t' if tiled else ''}")
    g32 = run_gpu(p, niter=2, tune=8)
    assert_parity(g32, r, label="medium64-fp32-v8t")


@pytest.mark.parametrize("rprec,variant,bands", [(0, 7, True), (1, 6, True), (1, 7, False), (2, 8, True),
                                                 (1, 7, True)])
def test_tile_walk_equals_grid_launch(rprec, variant, bands):
    """The persistent kernel walks the list of active tiles (MK_FLAG_WALK, and
    by default with bands); each tile is the grid form's computation
    (MK_FLAG_GRID), so every output is the same bits, and the oracle agrees."""
    mk = require_gpu()
    p = small_problem(seed=44, n=60, nt=128, nf=40, niter=5)
    fb = None
    if bands:
        rng = np.random.default_rng(8)
        fb = np.stack([np.zeros(p.nf, np.int32), rng.integers(8, 65, p.nf).astype(np.int32)], axis=1)
    say(f"tile walk rprec {rprec} variant {variant} bands {bands}")
    grid = run_gpu(p, fbands=fb, rprec=rprec, tune=variant, flags=mk.MK_FLAG_GRID)
    walk = run_gpu(p, fbands=fb, rprec=rprec, tune=variant, flags=mk.MK_FLAG_WALK)
    for k in ("f1plus", "f1minus", "Gplus", "Gminus", "norms"):
        assert np.array_equal(walk[k], grid[k]), k
    if bands:      # the default form of a banded plan is the walk
        dflt = run_gpu(p, fbands=fb, rprec=rprec, tune=variant)
        for k in ("f1plus", "f1minus", "Gplus", "Gminus", "norms"):
            assert np.array_equal(dflt[k], walk[k]), k
    assert_parity(walk, run_oracle(p, fbands=fb), tol=TOL[rprec], label=f"walk{rprec}-v{variant}")


def test_tile_walk_under_graph_replay_with_new_bands():
    """Graph replays keep the tile list's address and read its length from
    device memory: a new focal set with other bands replays the same graph
    and must match the eager passes bit for bit."""
    mk = require_gpu()
    p = small_problem(seed=45, n=48, nt=128, nf=24, niter=4)
    nr, nt = p.Rhat.shape[0], p.geom.nt
    outs = {}
    for flags in (mk.MK_FLAG_WALK, mk.MK_FLAG_WALK | mk.MK_FLAG_GRAPH):
        plan = mk.mk_plan(nr, nr, nt, p.geom.dt, p.geom.dx, band=p.band, nf_max=p.nf, rprec=1, flags=flags)
        mk.mk_load_R(plan, p.Rhat)
        res = []
        for trial in range(3):
            rng_t = np.random.default_rng(100 + trial)
            fb = np.stack([np.zeros(p.nf, np.int32), rng_t.integers(6, 65, p.nf).astype(np.int32)], axis=1)
            mk.mk_set_focal(plan, p.Gd, p.itd, p.shift, fb)
            n = mk.mk_iterate(plan, 4)
            res.append((n, mk.mk_get(plan, "Gminus", np.zeros(p.Gd.shape, np.float32))))
        mk.mk_destroy(plan)
        outs[flags] = res
    for (n0, g0), (n1, g1) in zip(outs[mk.MK_FLAG_WALK], outs[mk.MK_FLAG_WALK | mk.MK_FLAG_GRAPH]):
        assert np.array_equal(n0, n1) and np.array_equal(g0, g1)
