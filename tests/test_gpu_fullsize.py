"""Parity at the benchmark's full size: 601 x 601 receivers/shots, nt 2048,
complex64 R of 2.96 GB, in the launch configuration the benchmark times.

The oracle finishes a few passes of this size in seconds, so the first
passes and the G assembly are compared element by element.
"""

import numpy as np
import pytest

from gpu_common import assert_parity, run_gpu, run_oracle, say
from mkgen.layered import make_config

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def medium():
    say("generating the 601 x 601, nt 2048 workload")
    return make_config("medium", nf=1)


def test_medium_single_focal_first_passes(medium):
    for niter in (1, 2):
        say(f"medium nf=1 niter={niter}")
        g = run_gpu(medium, niter=niter)
        r = run_oracle(medium, niter=niter)
        assert_parity(g, r, label=f"medium-nf1-{niter}")


def test_medium_focal_line_subset():
    say("medium nf=4 on the 500 m line")
    p = make_config("medium", nf=4)
    g = run_gpu(p, niter=2)
    r = run_oracle(p, niter=2)
    assert_parity(g, r, label="medium-nf4")
