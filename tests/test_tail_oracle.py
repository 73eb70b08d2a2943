"""Pins of the series-tail reference (oracle/tail.py) against the plain
series of Algorithm 1 and closed forms."""

import numpy as np
import pytest

from mkgen.layered import small_problem
from oracle import SynthesisOperator, marchenko
from oracle import tail as ot


def test_window_round_trip():
    x = np.random.default_rng(0).standard_normal((2, 3, 32))
    w = ot.window(x, 32)
    np.testing.assert_array_equal(ot.unwindow(w, 32), x)
    w8 = ot.window(x, 8)
    assert w8[0, 0, 4] == x[0, 0, 0] and w8[0, 0, 0] == x[0, 0, 28] and w8[0, 0, 7] == x[0, 0, 3]


def test_restart_without_tail_is_two_more_passes_of_the_series():
    p = small_problem(seed=3, n=10, nt=64, nf=2, niter=4)
    S = SynthesisOperator(p.Rhat, p.band, p.c, p.geom.nt)
    k, m = 4, 5
    a = marchenko(S, p.Gd, p.itd, p.shift, k)
    b = marchenko(S, p.Gd, p.itd, p.shift, k + 2 + m)
    f1p, f1m, rho, norms = ot.restart(S, p.Gd, p.itd, p.shift, a["f1plus"], niter=m)
    np.testing.assert_allclose(f1p, b["f1plus"], atol=1e-12)
    np.testing.assert_allclose(f1m, b["f1minus"], atol=1e-12)
    # the residual is the next odd term of the series, and the continued norms are its norms
    c = marchenko(S, p.Gd, p.itd, p.shift, k + 2 + m, keep_iterates=True)
    np.testing.assert_allclose(rho, c["iterates"][k + 1], atol=1e-12)
    np.testing.assert_allclose(norms, c["norms"][k + 2:], rtol=1e-10)
    gp, gm = ot.g_fields(S, f1p, f1m)
    np.testing.assert_allclose(gp, b["Gplus"], atol=1e-12)
    np.testing.assert_allclose(gm, b["Gminus"], atol=1e-12)


def test_geometric_tails_exact_on_a_geometric_series():
    rng = np.random.default_rng(1)
    a, b = rng.standard_normal((2, 3, 16)), rng.standard_normal((2, 3, 16))
    qe, qo = 0.3, 0.5
    hist = np.stack([a, b, qe * a, qo * b], axis=2)          # N0, N1, N2, N3
    te, to = ot.geometric_tails(hist)
    # sum_{m>=2} qe^m a and sum_{m>=2} qo^m b
    np.testing.assert_allclose(te, qe ** 2 / (1 - qe) * a, atol=1e-12)
    np.testing.assert_allclose(to, qo ** 2 / (1 - qo) * b, atol=1e-12)


def test_exact_tail_makes_the_residual_vanish():
    """Adding the true remaining terms leaves only the truncation of the long run."""
    p = small_problem(seed=5, n=8, nt=64, nf=1, niter=4)
    S = SynthesisOperator(p.Rhat, p.band, p.c, p.geom.nt)
    k, K = 4, 60
    full = marchenko(S, p.Gd, p.itd, p.shift, K, keep_iterates=True)
    a = marchenko(S, p.Gd, p.itd, p.shift, k)
    N = full["iterates"]
    te = ot.window(sum(N[i] for i in range(k, K, 2)), 64)
    to = ot.window(sum(N[i] for i in range(k + 1, K, 2)), 64)
    f1p, f1m = ot.apply_tails(a["f1plus"], a["f1minus"], te, to, p.itd, p.shift)
    np.testing.assert_allclose(f1p, full["f1plus"], atol=1e-12)
    np.testing.assert_allclose(f1m, full["f1minus"], atol=1e-12)
    _, _, rho, _ = ot.restart(S, p.Gd, p.itd, p.shift, f1p)
    assert np.linalg.norm(rho) <= 1e-10 * np.linalg.norm(p.Gd)


# ---------------------------------------------------------------------------
# the network's tails: normalisation by the RMS of N_0 and the output rescale
# ---------------------------------------------------------------------------


def _golden_net(golden_dir):
    import json
    import os

    with open(os.path.join(golden_dir, "tail_network.json")) as fh:
        case = json.load(fh)
    P = {k: np.array(case[k], dtype=np.float64) for k in ("W1", "b1", "W2", "b2", "W3", "b3")}
    hist = np.array(case["hist"], dtype=np.float64)[None]          # [nf=1][nr=2][k][T]
    return case, P, hist


@pytest.mark.parametrize("f16", [False, True])
def test_net_tails_hand_derived(golden_dir, f16):
    case, P, hist = _golden_net(golden_dir)
    te, to = ot.net_tails(hist, P, f16=f16)
    np.testing.assert_array_equal(te[0], np.array(case["expected_even"]))
    np.testing.assert_array_equal(to[0], np.array(case["expected_odd"]))


@pytest.mark.parametrize("f16", [False, True])
@pytest.mark.parametrize("alpha", [2.0 ** -3, 2.0 ** 5])
def test_net_tails_scale_with_the_iterates(alpha, f16):
    """The series is linear in G_d, so the tails of alpha * (N_0 .. N_{k-1})
    are alpha times the tails: the input is divided by the RMS of N_0 and the
    output multiplied by it.  Powers of two keep every rounding identical."""
    from oracle import tailnet as tn

    rng = np.random.default_rng(4)
    P = tn.init_params(rng, k=4, hidden=6)
    for key in P:
        P[key] = P[key] + 0.1 * rng.standard_normal(P[key].shape)     # non-zero biases everywhere
    hist = rng.standard_normal((2, 3, 4, 48))
    hist[1, 2, 0] = 0.0                                                  # a trace with N_0 = 0
    te, to = ot.net_tails(hist, P, f16=f16)
    te_a, to_a = ot.net_tails(alpha * hist, P, f16=f16)
    np.testing.assert_array_equal(te_a, alpha * te)
    np.testing.assert_array_equal(to_a, alpha * to)
    assert not te[1, 2].any() and not to[1, 2].any()
    assert np.abs(te).max() > 0 and np.abs(to).max() > 0
