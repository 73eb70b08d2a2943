"""Solves through the checked build of the library (device-side bounds checks).

Run as a child process of tests/test_gpu_device_checks.py with MK_LIBRARY
pointing at libmk_checked.so, so that the test runner's own process keeps the
normal library.  Each case runs a solve, then asks mk_device_checks() which
kernel files saw a range end past its allocation; it prints one line per case
("case <name> checks <mask>") and, for the first case, the worst error
against the FP64 oracle.  Exit status 0 when every case ran.

    python tests/device_checks_run.py [--one]     # --one: only the first case
"""

import os
import sys

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)

from gpu_common import FIELD_NAMES, assert_parity, run_gpu, run_oracle  # noqa: E402
from mkgen.layered import small_problem  # noqa: E402
from paper_2106_04649_amd import mk  # noqa: E402


def report(name):
    print(f"case {name} checks {mk.mk_device_checks()}", flush=True)


def main(one=False):
    torch.cuda.set_device(0)
    mk.load_library()
    assert os.path.basename(mk.LIB_PATH) == "libmk_checked.so", mk.LIB_PATH
    mk.mk_device_checks()                          # start from clear words

    # one focal point: the streaming contraction and the per-trace kernels
    p = small_problem(seed=3, n=40, nt=128, nf=1, niter=6)
    g = run_gpu(p)
    assert_parity(g, run_oracle(p), label="checked-gemv")
    report("gemv")
    if one:
        return

    # focal batches on the matrix cores: direct tiles, LDS-staged tiles (tiled
    # R), 16-bit R with two planes of X, bands (the tile walk), one plane
    p = small_problem(seed=5, n=48, nt=128, nf=20, niter=5)
    rng = np.random.default_rng(2)
    fb = np.stack([np.zeros(p.nf, np.int32), rng.integers(10, 65, p.nf).astype(np.int32)], axis=1)
    for name, kw in (("mfma-direct", dict(tune=1, flags=mk.MK_FLAG_ROW_R)),
                     ("lds-fp32", dict(tune=7)),
                     ("lds-fp16-2x", dict(tune=6, rprec=1)),
                     ("walk-fp16-bands", dict(tune=7, rprec=1, fbands=fb)),
                     ("lds-bf16-1x", dict(tune=8, rprec=2, flags=mk.MK_FLAG_FAST_X)),
                     ("gemv-fp16", dict(tune=0, rprec=1, flags=mk.MK_FLAG_ROW_R))):
        run_gpu(p, **kw)
        report(name)

    # the series tail (geometric and a random network), the restart, the
    # stopping rule, the auxiliary fields, the image and a state round trip
    nr, nt = p.Rhat.shape[0], p.geom.nt
    plan = mk.mk_plan(nr, nr, nt, p.geom.dt, p.geom.dx, band=p.band, nf_max=p.nf, rprec=1)
    mk.mk_load_R(plan, p.Rhat)
    mk.mk_tail_record(plan, 4, 64)
    mk.mk_tail_load(plan, (np.random.default_rng(7).standard_normal(mk.mk_net_param_count(4, 16)) * 0.05)
                    .astype(np.float32))
    for mode in (mk.TAIL_GEOMETRIC, mk.TAIL_NET):
        mk.mk_set_focal(plan, p.Gd, p.itd, p.shift, fb)
        mk.mk_iterate(plan, 4, want_norms=False)
        mk.mk_tail_apply(plan, mode)
        mk.mk_iterate_tol(plan, 1e-4, 10)
        for k in FIELD_NAMES + ("Gtotal",):
            mk.mk_get(plan, k, np.zeros(p.Gd.shape, np.float32))
        mk.mk_image(plan)
        report(f"tail-{mode}")
    blob = mk.mk_get_state(plan)
    mk.mk_set_state(plan, blob)
    mk.mk_iterate(plan, 2)
    report("state")
    mk.mk_destroy(plan)

    # a plain series' auxiliary fields, and R streamed from host memory
    plan = mk.mk_plan(nr, nr, nt, p.geom.dt, p.geom.dx, band=p.band, nf_max=p.nf, r_dev_bytes=1 << 18)
    mk.mk_load_R(plan, p.Rhat)
    mk.mk_set_focal(plan, p.Gd, p.itd, p.shift)
    mk.mk_iterate(plan, 4)
    for k in ("f2plus", "pminus"):
        mk.mk_get(plan, k, np.zeros(p.Gd.shape, np.float32))
    mk.mk_destroy(plan)
    report("aux-streamed")


if __name__ == "__main__":
    main(one="--one" in sys.argv[1:])
