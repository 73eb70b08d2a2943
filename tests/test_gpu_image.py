"""The double-focusing image (mk_image) against the FP64 oracle.

Per focal point, the image of the GPU solve against the oracle image of the
oracle solve on the same inputs.  The image is a bilinear form of G- and f1+,
so (Cauchy-Schwarz) relative errors e_G and e_f of the two fields move it by
at most c (e_G + e_f + e_G e_f) ||G-|| ||f1+||: the bar is that bound with
e_G = e_f = the fields' own bar (1e-5 for the FP32 paths, 1e-3 for FP16 R).
"""

import numpy as np
import pytest

from gpu_common import require_gpu, say
from mkgen.layered import small_problem
from oracle import SynthesisOperator, image, marchenko

pytestmark = pytest.mark.gpu


def _solve_and_image(p, fbands=None, rprec=0, flags=0, nf_max=None):
    mk = require_gpu()
    nr, nt = p.Rhat.shape[0], p.geom.nt
    plan = mk.mk_plan(nr, nr, nt, p.geom.dt, p.geom.dx, band=p.band, nf_max=nf_max or p.nf, rprec=rprec,
                      flags=flags)
    mk.mk_load_R(plan, p.Rhat)
    mk.mk_set_focal(plan, p.Gd, p.itd, p.shift, fbands)
    mk.mk_iterate(plan, p.niter, want_norms=False)
    img = mk.mk_image(plan)
    # again after G- was fetched (cached G assembly): the same bits
    mk.mk_get(plan, "Gminus", np.zeros((p.nf, nr, nt), np.float32))
    img2 = mk.mk_image(plan)
    mk.mk_destroy(plan)
    assert np.array_equal(img, img2)
    return img


def _check(p, img, tol, fbands=None, label=""):
    S = SynthesisOperator(p.Rhat, p.band, p.c, p.geom.nt)
    ref = marchenko(S, p.Gd, p.itd, p.shift, p.niter, fbands=fbands)
    want = image(ref["Gminus"], ref["f1plus"], p.c)
    for f in range(p.nf):
        bound = p.c * np.linalg.norm(ref["Gminus"][f]) * np.linalg.norm(ref["f1plus"][f])
        err = abs(img[f] - want[f])
        say(f"  {label} focal {f}: image {img[f]:.6e} oracle {want[f]:.6e} |diff| {err:.2e} "
            f"(bar {tol * (2 + tol) * bound:.2e})")
        assert err <= tol * (2 + tol) * bound, (label, f, err)


def test_image_fp32_with_focal_bands():
    """GEMV path (three focal points), per-focal bands: the plan reorders the
    focal points by band end and mk_image returns them in the caller's order."""
    say("image: FP32, per-focal bands")
    p = small_problem(seed=91, n=24, nt=128, nf=3, niter=8)
    fb = np.array([[0, 30], [2, 64], [0, 12]], dtype=np.int32)
    img = _solve_and_image(p, fbands=fb)
    _check(p, img, 1e-5, fbands=fb, label="fp32 bands")


@pytest.mark.parametrize("rprec,tol", [(0, 1e-5), (1, 1e-3)])
def test_image_batched(rprec, tol):
    """Matrix-core contraction over a batch of 12 focal points, complex64 and FP16 R."""
    say(f"image: batched, rprec {rprec}")
    p = small_problem(seed=92, n=48, nt=256, nf=12, niter=6)
    img = _solve_and_image(p, rprec=rprec)
    _check(p, img, tol, label=f"batched r{rprec}")


def test_image_long_traces():
    """nt 2048: several groups of eight loads per lane, and 16 traces per block row."""
    say("image: nt 2048")
    p = small_problem(seed=93, n=16, nt=2048, nf=4, niter=4)
    img = _solve_and_image(p)
    _check(p, img, 1e-5, label="nt2048")
