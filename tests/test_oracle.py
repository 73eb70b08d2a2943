"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these checks re-types the oracle's own formula: each compares the
oracle with something independent of it -- hand-derived worked examples
(tests/golden), time-domain brute force written with explicit loops, a dense
direct solve built by index arithmetic, singular values from LAPACK, and
structural identities of Eq. (1) and Algorithm 1.
"""

import cmath
import json
import math
import os

import numpy as np
import pytest

from mkgen.layered import make_config, small_problem
from oracle import SynthesisOperator, marchenko, mute_window, rel_l2, rev


# ---------------------------------------------------------------------------
# independent helpers (explicit loops / index arithmetic, no FFT)
# ---------------------------------------------------------------------------


def spike_rhat(nt, spikes):
    """rfft-convention spectrum of sum_j a_j * delta[t - k_j], written out."""
    out = np.zeros(nt // 2 + 1, dtype=np.complex128)
    for w in range(nt // 2 + 1):
        out[w] = sum(a * cmath.exp(-2j * math.pi * w * k / nt) for k, a in spikes)
    return out


def time_domain_from_band(Rhat_rws, lo, hi, nt):
    """Inverse DFT (Hermitian completion, DC/Nyquist real) by explicit sums."""
    nr, B, ns = Rhat_rws.shape
    Rt = np.zeros((nr, ns, nt))
    for r in range(nr):
        for s in range(ns):
            for k in range(nt):
                acc = 0.0
                for w in range(lo, hi + 1):
                    z = Rhat_rws[r, w - lo, s]
                    if w == 0 or w == nt // 2:
                        acc += z.real * math.cos(2 * math.pi * w * k / nt)
                    else:
                        e = cmath.exp(2j * math.pi * w * k / nt)
                        acc += 2.0 * (z * e).real
                Rt[r, s, k] = acc / nt
    return Rt


def brute_synthesis(Rt, x, c):
    """c * sum_s sum_j R(r, s, k - j) x(s, j): circular time convolution + space sum."""
    nr, ns, nt = Rt.shape
    nf = x.shape[0]
    y = np.zeros((nf, nr, nt))
    for f in range(nf):
        for r in range(nr):
            for k in range(nt):
                acc = 0.0
                for s in range(ns):
                    for j in range(nt):
                        acc += Rt[r, s, (k - j) % nt] * x[f, s, j]
                y[f, r, k] = c * acc
    return y


def load(golden_dir, name):
    with open(os.path.join(golden_dir, name)) as fh:
        return json.load(fh)


def spikes_to_trace(d, nt):
    out = np.zeros(nt)
    for k, a in d.items():
        out[int(k) % nt] += a
    return out


# ---------------------------------------------------------------------------
# mute window and time reversal
# ---------------------------------------------------------------------------


def test_mute_masks_match_hand_lists(golden_dir):
    for case in load(golden_dir, "mute_masks.json")["cases"]:
        m = mute_window(np.array([case["itd"]]), case["shift"], case["nt"])[0]
        assert sorted(np.nonzero(m)[0].tolist()) == case["kept"], case


def test_mute_is_symmetric_in_time():
    itd = np.array([[3, 17, 40, 1000]])
    m = mute_window(itd, 5, 64)
    assert np.array_equal(m, rev(m))


def test_reversal_and_rfft_conjugate():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((3, 32))
    r = rev(x)
    assert r[0, 0] == x[0, 0] and r[0, 1] == x[0, 31] and r[0, 16] == x[0, 16]
    assert np.array_equal(rev(r), x)
    np.testing.assert_allclose(np.fft.rfft(r), np.conj(np.fft.rfft(x)), atol=1e-12)


# ---------------------------------------------------------------------------
# synthesis = circular time convolution + space integral (Eq. (1))
# ---------------------------------------------------------------------------


@pytest.mark.parametrize("band", [(0, 8), (2, 6), (0, 3), (8, 8)])
def test_synthesis_matches_time_domain_brute_force(band):
    rng = np.random.default_rng(11)
    nr, ns, nt = 3, 4, 16          # nr != ns and random complex R catch a transposed operand
    lo, hi = band
    B = hi - lo + 1
    Rhat = (rng.standard_normal((nr, B, ns)) + 1j * rng.standard_normal((nr, B, ns)))
    x = rng.standard_normal((2, ns, nt))
    c = 0.37
    S = SynthesisOperator(Rhat.astype(np.complex64), (lo, hi), c, nt)
    Rt = time_domain_from_band(Rhat.astype(np.complex64).astype(np.complex128), lo, hi, nt)
    y_brute = brute_synthesis(Rt, x, c)
    np.testing.assert_allclose(S(x), y_brute, rtol=0, atol=1e-11 * max(1.0, np.abs(y_brute).max()))


def test_per_focal_bands_match_brute_force():
    rng = np.random.default_rng(12)
    nr = ns = 3
    nt = 16
    Rhat = rng.standard_normal((nr, 9, ns)) + 1j * rng.standard_normal((nr, 9, ns))
    x = rng.standard_normal((2, ns, nt))
    fb = np.array([[0, 3], [2, 7]], dtype=np.int32)
    S = SynthesisOperator(Rhat.astype(np.complex64), (0, 8), 1.0, nt)
    y = S(x, fb)
    R64 = Rhat.astype(np.complex64).astype(np.complex128)
    for f in range(2):
        lo, hi = fb[f]
        Rt = time_domain_from_band(R64[:, lo:hi + 1, :], lo, hi, nt)
        np.testing.assert_allclose(y[f], brute_synthesis(Rt, x[f:f + 1], 1.0)[0], atol=1e-11)


# ---------------------------------------------------------------------------
# hand-derived worked examples (Eq. (1) + Algorithm 1)
# ---------------------------------------------------------------------------


def _run_spike_case(case, spikes):
    nt = case["nt"]
    Rhat = spike_rhat(nt, spikes).reshape(1, -1, 1).astype(np.complex64)
    Gd = np.zeros((1, 1, nt), dtype=np.float32)
    Gd[0, 0, case["kd"]] = 1.0
    itd = np.array([[case["kd"]]], dtype=np.int32)
    S = SynthesisOperator(Rhat, (0, nt // 2), 1.0, nt)
    return marchenko(S, Gd, itd, case["shift"], case["niter"])


def test_single_interface_closed_form(golden_dir):
    case = load(golden_dir, "single_interface.json")
    out = _run_spike_case(case, [(case["k1"], case["r"])])
    nt = case["nt"]
    for key in ["f1plus", "f1minus", "Gminus", "Gplus", "f2p", "pmin", "Gtotal"]:
        want = spikes_to_trace(case["expected"][key], nt)
        np.testing.assert_allclose(out[key][0, 0], want, atol=2e-7, err_msg=key)
    np.testing.assert_allclose(out["norms"][:, 0], case["expected"]["norms"], atol=2e-7)


def test_two_interfaces_hand_derived_terms(golden_dir):
    case = load(golden_dir, "two_interfaces.json")
    out = _run_spike_case(case, [(case["k1"], case["r1"]), (case["k2"], case["r2"])])
    nt = case["nt"]
    for key in ["f1plus", "f1minus", "Gminus", "Gplus", "Gtotal"]:
        want = spikes_to_trace(case["expected"][key], nt)
        np.testing.assert_allclose(out[key][0, 0], want, atol=2e-7, err_msg=key)
    np.testing.assert_allclose(out["norms"][:, 0], case["expected"]["norms"], atol=2e-7)


# ---------------------------------------------------------------------------
# special cases and structure
# ---------------------------------------------------------------------------


def test_zero_reflectivity_leaves_the_initial_field():
    p = small_problem(seed=1)
    S = SynthesisOperator(np.zeros_like(p.Rhat), p.band, p.c, p.geom.nt)
    out = marchenko(S, p.Gd, p.itd, p.shift, 6)
    Gd = p.Gd.astype(np.float64)
    assert np.array_equal(out["f1plus"], rev(Gd))
    assert np.array_equal(out["Gplus"], Gd)
    assert np.array_equal(out["Gtotal"], Gd)
    assert not out["f1minus"].any() and not out["Gminus"].any() and not out["norms"].any()


def test_homogeneity_in_R_and_linearity_in_Gd():
    p = small_problem(seed=2, nf=2)
    nt = p.geom.nt
    alpha = 0.625                       # applied in FP64, where it costs one rounding
    S1 = SynthesisOperator(p.Rhat, p.band, p.c, nt)
    S2 = SynthesisOperator(p.Rhat.astype(np.complex128) * alpha, p.band, p.c, nt)
    o1 = marchenko(S1, p.Gd, p.itd, p.shift, 6, keep_iterates=True)
    o2 = marchenko(S2, p.Gd, p.itd, p.shift, 6, keep_iterates=True)
    for i in range(6):
        np.testing.assert_allclose(o2["iterates"][i], alpha ** (i + 1) * o1["iterates"][i],
                                   rtol=0, atol=1e-12 * np.abs(o1["iterates"][i]).max() + 1e-300)
    rng = np.random.default_rng(5)
    g1 = rng.standard_normal(p.Gd.shape)
    g2 = rng.standard_normal(p.Gd.shape)
    oa = marchenko(S1, g1, p.itd, p.shift, 6)
    ob = marchenko(S1, g2, p.itd, p.shift, 6)
    oc = marchenko(S1, 2.0 * g1 - 3.0 * g2, p.itd, p.shift, 6)
    for key in ["f1plus", "f1minus", "Gplus", "Gminus"]:
        np.testing.assert_allclose(oc[key], 2.0 * oa[key] - 3.0 * ob[key], atol=1e-10)


def test_contraction_bound_and_monotone_decrease():
    p = small_problem(seed=4, rho_target=0.2, nf=2)
    nt = p.geom.nt
    rho = p.c * max(np.linalg.svd(p.Rhat[:, w, :].astype(np.complex128), compute_uv=False)[0]
                    for w in range(p.Rhat.shape[1]))
    assert abs(rho - 0.2) < 1e-6
    S = SynthesisOperator(p.Rhat, p.band, p.c, nt)
    out = marchenko(S, p.Gd, p.itd, p.shift, 10)
    n = out["norms"]
    g = np.sqrt((p.Gd.astype(np.float64) ** 2).sum(axis=(1, 2)))
    assert (n[0] <= rho * g * (1 + 1e-12)).all()
    assert (n[1:] <= rho * n[:-1] * (1 + 1e-12) + 1e-300).all()
    assert (n[0] > 0).all()
    live = n[:-1] > 0
    assert (n[1:][live] < n[:-1][live]).all()


def _dense_operator(p):
    """A = theta * Rev * S as an explicit matrix, by index arithmetic."""
    nr, nt = p.Rhat.shape[0], p.geom.nt
    lo, hi = p.band
    Rt = time_domain_from_band(p.Rhat.astype(np.complex128), lo, hi, nt)
    k = np.arange(nt)
    conv = Rt[:, :, (k[:, None] - k[None, :]) % nt]          # [r][s][k][j]
    Smat = p.c * conv.transpose(0, 2, 1, 3).reshape(nr * nt, nr * nt)
    P = np.zeros((nr * nt, nr * nt))
    for r in range(nr):
        for kk in range(nt):
            P[r * nt + kk, r * nt + (-kk) % nt] = 1.0
    keep = np.zeros(nr * nt)
    for r in range(nr):
        lim = int(p.itd[0, r]) - p.shift
        for kk in range(nt):
            t = kk if kk < nt // 2 else kk - nt
            keep[r * nt + kk] = 1.0 if (abs(t) < lim and kk != nt // 2) else 0.0
    return Smat, P, np.diag(keep)


def test_dense_direct_solve_of_the_converged_series():
    p = small_problem(seed=6, rho_target=0.5, n=6, nt=32)
    nr, nt = p.Rhat.shape[0], p.geom.nt
    Smat, P, T = _dense_operator(p)
    A = T @ P @ Smat
    g = p.Gd[0].astype(np.float64).reshape(-1)
    rhs = P @ g
    f1p = np.linalg.solve(np.eye(nr * nt) - A @ A, rhs)       # f1+ = (I - A^2)^-1 Rev Gd
    f1m = T @ Smat @ f1p                                      # f1- = theta S f1+
    Gm = Smat @ f1p - f1m
    Gp = P @ f1p - Smat @ (P @ f1m)
    S = SynthesisOperator(p.Rhat, p.band, p.c, nt)
    normA = np.linalg.norm(A, 2)
    assert normA <= 0.5 + 1e-9
    for niter in (4, 8, 60):
        out = marchenko(S, p.Gd, p.itd, p.shift, niter)
        M = niter // 2
        bound = normA ** (2 * M + 2) / (1 - normA ** 2) * np.linalg.norm(g)
        err = np.linalg.norm(out["f1plus"][0].reshape(-1) - f1p)
        assert err <= bound * (1 + 1e-9) + 1e-12
    for key, ref in (("f1plus", f1p), ("f1minus", f1m), ("Gminus", Gm), ("Gplus", Gp)):
        np.testing.assert_allclose(out[key][0].reshape(-1), ref, atol=1e-12, err_msg=key)


def test_G_identities_through_series_terms():
    """G+ = Rev f1+ + sum_{even i} RN_{i+1}; G- = RN_0 + sum_{odd i} RN_{i+1} - f1-."""
    p = small_problem(seed=8, nf=2)
    S = SynthesisOperator(p.Rhat, p.band, p.c, p.geom.nt)
    niter = 6
    out = marchenko(S, p.Gd, p.itd, p.shift, niter)
    more = marchenko(S, p.Gd, p.itd, p.shift, niter + 1, keep_iterates=True)
    RN = more["synth"]
    gp = rev(out["f1plus"]) + sum(RN[i + 1] for i in range(0, niter, 2))
    gm = RN[0] + sum(RN[i + 1] for i in range(1, niter, 2)) - out["f1minus"]
    np.testing.assert_allclose(out["Gplus"], gp, atol=1e-12)
    np.testing.assert_allclose(out["Gminus"], gm, atol=1e-12)


@pytest.mark.parametrize("niter", [1, 4, 7])
def test_total_G_from_auxiliary_fields_equals_Gplus_plus_Gminus(niter):
    """The total G read from p- and f2+ (one synthesis of the last term) and
    the sum of G+ and G- (two syntheses of the focusing functions) are two
    routes to the same field; a dipping model and two focal points with
    different windows."""
    p = small_problem(seed=13, nf=2, ndips=1)
    S = SynthesisOperator(p.Rhat, p.band, p.c, p.geom.nt)
    out = marchenko(S, p.Gd, p.itd, p.shift, niter)
    total = out["Gplus"] + out["Gminus"]
    np.testing.assert_allclose(out["Gtotal"], total, atol=1e-12 * np.abs(total).max())
    assert np.abs(out["Gtotal"]).max() > 0


def test_rel_l2():
    assert rel_l2(np.ones(4), np.ones(4)) == 0.0
    assert abs(rel_l2(np.array([1.0, 0.0]), np.array([2.0, 0.0])) - 0.5) < 1e-15


# ---------------------------------------------------------------------------
# generated inputs
# ---------------------------------------------------------------------------


def test_generated_R_is_reciprocal_and_deterministic():
    p = small_problem(seed=9, ndips=2)
    assert np.array_equal(p.Rhat, p.Rhat.transpose(2, 1, 0))
    q = small_problem(seed=9, ndips=2)
    assert np.array_equal(p.Rhat, q.Rhat) and np.array_equal(p.Gd, q.Gd)
    t = make_config("tiny")
    assert np.array_equal(t.Rhat, t.Rhat.transpose(2, 1, 0))
    assert t.Rhat.shape == (101, 257, 101) and t.Gd.shape == (1, 101, 512)
    assert t.shift == 10 and (t.itd > t.shift).all()
    assert np.isfinite(t.Rhat).all() and np.isfinite(t.Gd).all()


def test_tiny_config_series_converges():
    p = make_config("tiny")
    S = SynthesisOperator(p.Rhat, p.band, p.c, p.geom.nt)
    out = marchenko(S, p.Gd, p.itd, p.shift, p.niter)
    n = out["norms"][:, 0]
    assert n[0] > 0 and n[-1] < 1e-2 * n[0]
    assert np.isfinite(out["Gplus"]).all() and np.isfinite(out["Gminus"]).all()
