"""Pins of the double-focusing image oracle: explicit-loop convolution on
tiny inputs, and hand-derived spike cases run through the oracle's series
(tests/golden/imaging.json)."""

import json
import os

import numpy as np
import pytest

from oracle import SynthesisOperator, double_focused, image, marchenko
from test_oracle import spike_rhat, spikes_to_trace


def _brute(Gm, f1p, c):
    """c * sum_x sum_t' G-(x, t - t') f1+(x, t') with explicit loops."""
    nf, nx, nt = Gm.shape
    out = np.zeros((nf, nt))
    for f in range(nf):
        for t in range(nt):
            acc = 0.0
            for x in range(nx):
                for tp in range(nt):
                    acc += Gm[f, x, (t - tp) % nt] * f1p[f, x, tp]
            out[f, t] = c * acc
    return out


@pytest.mark.parametrize("nt", [8, 9, 16])
def test_double_focused_matches_loops(nt):
    rng = np.random.default_rng(nt)
    Gm = rng.standard_normal((2, 3, nt))
    f1p = rng.standard_normal((2, 3, nt))
    want = _brute(Gm, f1p, 0.37)
    np.testing.assert_allclose(double_focused(Gm, f1p, 0.37), want, atol=1e-12)
    np.testing.assert_allclose(image(Gm, f1p, 0.37), want[:, 0], atol=1e-12)


def test_image_is_the_zero_lag_of_a_shifted_pair():
    # G- = delta at t = a, f1+ = delta at t = b: G^{-,+} = delta at a + b, image 1 iff a + b = 0 (mod nt)
    nt = 16
    for a in range(nt):
        for b in range(nt):
            Gm = np.zeros((1, 1, nt))
            f1p = np.zeros((1, 1, nt))
            Gm[0, 0, a] = 1.0
            f1p[0, 0, b] = 1.0
            assert image(Gm, f1p, 1.0)[0] == (1.0 if (a + b) % nt == 0 else 0.0)


def test_spike_cases(golden_dir):
    with open(os.path.join(golden_dir, "imaging.json")) as fh:
        cases = json.load(fh)["cases"]
    for case in cases:
        nt = case["nt"]
        Rhat = spike_rhat(nt, [tuple(s) for s in case["spikes"]]).reshape(1, -1, 1).astype(np.complex64)
        Gd = np.zeros((1, 1, nt), dtype=np.float32)
        Gd[0, 0, case["kd"]] = 1.0
        itd = np.array([[case["kd"]]], dtype=np.int32)
        S = SynthesisOperator(Rhat, (0, nt // 2), 1.0, nt)
        out = marchenko(S, Gd, itd, case["shift"], case["niter"])
        gmp = double_focused(out["Gminus"], out["f1plus"], 1.0)[0]
        np.testing.assert_allclose(gmp, spikes_to_trace(case["Gmp"], nt), atol=2e-7, err_msg=case["name"])
        assert abs(image(out["Gminus"], out["f1plus"], 1.0)[0] - case["image"]) <= 2e-7, case["name"]
