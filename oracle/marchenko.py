"""Plain FP64 oracle of the iterative (Neumann-series) Marchenko scheme.

TEST INFRASTRUCTURE.  Imported only by ``tests/``, the smoke check and the
benchmark's CPU-baseline leg.  It is slow on purpose: every step is written as
the paper states it, with numpy's FFT and matrix product as the only library
primitives, so that it can be checked against the paper by eye.

What it follows (arXiv 2106.04649):

* Eq. (1), Theory section: one synthesis is a time convolution of the
  reflection response R with the current field followed by an integral over
  the surface positions x; the time convolution is done in the frequency
  domain, so each synthesis is rfft -> per-frequency contraction over x ->
  irfft.  The double integral is a Riemann sum with weight ``c = dx * dt``.
* Theory section: the focusing functions are sums of the terms ``N_i`` of a
  Neumann series, each term the muted synthesis of the previous one, started
  from the time-reversed first arrival; the Green's functions follow from
  the focusing functions by extra syntheses (Marchenko relations of the cited
  Wapenaar et al. 2014 work), the total Green's function from the auxiliary
  fields f2+ and p- (the cited Wapenaar et al. 2013 route).
* Algorithm 1 fixes the sign convention (the synthesis output is reversed
  in time and negated before the mute), the number of terms and which
  terms each output accumulates.

Readings of the paper where it is silent or ambiguous:

* the time axis is periodic with ``nt`` samples (circular convolution, FFT
  length ``nt``); time reversal maps sample ``k`` to ``(nt - k) mod nt``;
* the mute ``theta_t`` keeps samples with ``|t_k| < itd - shift`` (strict) and
  zeroes all others, ``t_k = k`` for ``k < nt/2`` and ``k - nt`` above; the
  sample ``k = nt/2`` is always zeroed;
* "padding" before the inverse FFT is zero-filling of the bins outside the
  band; DC and Nyquist are taken as real (numpy's ``irfft`` convention);
* ``niter`` iterations are ``niter`` terms ``N_0 .. N_{niter-1}``.

Parity pins (tests/test_oracle.py): brute-force time-domain convolution,
a closed-form single-interface example, R = 0, homogeneity in R and
linearity in G_d, a dense direct solve of the converged series, the norm
contraction bound, the G^+/G^- identities through the series terms, the
total G against G^+ + G^- and the closed form, and hand-written mute
masks.
"""

from __future__ import annotations

from typing import Dict, Optional, Tuple

import numpy as np


# ---------------------------------------------------------------------------
# time-axis helpers
# ---------------------------------------------------------------------------


def signed_time(nt: int) -> np.ndarray:
    """Sample times in samples on the periodic axis: k for k < nt/2, k - nt above."""
    k = np.arange(nt)
    return np.where(k < nt // 2, k, k - nt)


def rev(x: np.ndarray) -> np.ndarray:
    """Time reversal x(t) -> x(-t) on the periodic axis (last axis)."""
    nt = x.shape[-1]
    idx = (-np.arange(nt)) % nt
    return x[..., idx]


def mute_window(itd: np.ndarray, shift: int, nt: int) -> np.ndarray:
    """theta_t of Eq. (1): True where a sample is kept.

    Kept: ``|t_k| < itd - shift``; the sample ``nt/2`` (both +nt/2 and -nt/2)
    is never kept.  ``itd`` has any leading shape; the result adds a time axis.
    """
    t = np.abs(signed_time(nt))
    keep = t[None, :] < (np.asarray(itd, dtype=np.int64).reshape(-1, 1) - int(shift))
    keep[:, nt // 2] = False
    return keep.reshape(np.shape(itd) + (nt,))


def apply_mute(x: np.ndarray, itd: np.ndarray, shift: int) -> np.ndarray:
    """theta_t of Eq. (1) applied to a field (zero outside the window)."""
    return np.where(mute_window(itd, shift, x.shape[-1]), x, 0.0)


def rel_l2(a: np.ndarray, b: np.ndarray) -> float:
    """||a - b||_2 / ||b||_2 (0 when both vanish)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    na = np.linalg.norm(a - b)
    if nb == 0.0:
        return 0.0 if na == 0.0 else float("inf")
    return float(na / nb)


# ---------------------------------------------------------------------------
# synthesis: Eq. (1) without the mute
# ---------------------------------------------------------------------------


class SynthesisOperator:
    """S(x) = irfft(c * sum_s Rhat[r][w][s] * rfft(x)[s][w]) over the band.

    ``Rhat`` is complex64 receivers x frequencies x shots (the layout the
    Introduction and Implementation sections give for the reflection data),
    upcast once to complex128.  ``band = (lo, hi)`` is the inclusive rfft-bin
    range stored in ``Rhat``; bins outside it are zero ("padding" before the
    inverse transform, Implementation section).  ``fbands[f] = (lo_f, hi_f)``
    optionally narrows the band per focal point.
    """

    def __init__(self, Rhat: np.ndarray, band: Tuple[int, int], c: float, nt: int):
        lo, hi = int(band[0]), int(band[1])
        nr, B, ns = Rhat.shape
        if B != hi - lo + 1:
            raise ValueError("Rhat frequency axis does not match the band")
        if not (0 <= lo <= hi <= nt // 2):
            raise ValueError("band outside [0, nt/2]")
        self.nr, self.ns, self.nt = nr, ns, nt
        self.lo, self.hi, self.c = lo, hi, float(c)
        # frequency-major copy for one batched matrix product per frequency
        self.Rw = np.ascontiguousarray(Rhat.astype(np.complex128).transpose(1, 0, 2))

    def __call__(self, x: np.ndarray, fbands: Optional[np.ndarray] = None) -> np.ndarray:
        """x: [nf][ns][nt] real -> [nf][nr][nt] real (float64)."""
        x = np.asarray(x, dtype=np.float64)
        nf, ns, nt = x.shape
        if ns != self.ns or nt != self.nt:
            raise ValueError("field shape does not match the operator")
        X = np.fft.rfft(x, axis=-1)                        # forward transform over t
        Xb = X[:, :, self.lo:self.hi + 1]                  # [nf][ns][B]
        if fbands is not None:
            w = np.arange(self.lo, self.hi + 1)
            inb = (w[None, :] >= fbands[:, 0:1]) & (w[None, :] <= fbands[:, 1:2])
            Xb = Xb * inb[:, None, :]
        # per frequency: Y_w[r][f] = c * sum_s R_w[r][s] X_w[s][f]
        Yw = self.c * np.matmul(self.Rw, Xb.transpose(2, 1, 0))   # [B][nr][nf]
        Y = np.zeros((nf, self.nr, nt // 2 + 1), dtype=np.complex128)
        Y[:, :, self.lo:self.hi + 1] = Yw.transpose(2, 1, 0)
        return np.fft.irfft(Y, nt, axis=-1)                # inverse transform over t


# ---------------------------------------------------------------------------
# the Neumann series of the Theory section
# ---------------------------------------------------------------------------


def marchenko(S: SynthesisOperator, Gd: np.ndarray, itd: np.ndarray, shift: int,
              niter: int, fbands: Optional[np.ndarray] = None,
              keep_iterates: bool = False) -> Dict[str, np.ndarray]:
    """The Neumann series of the Theory section in FP64, ``niter`` terms.

    Returns f1plus, f1minus, Gplus, Gminus, f2p, pmin, Gtotal and norms.
    ``Gd`` [nf][nr][nt], ``itd`` [nf][nr] (samples), ``shift`` (samples).

    The series starts from the time-reversed first arrival,
    ``N_{-1}(t) = G_d(-t)``.  Term ``i`` is Eq. (1) applied to term
    ``i - 1``: the synthesis ``S N_{i-1}`` is evaluated at negative time,
    negated (the sign of Algorithm 1, which Eq. (1) leaves out) and
    windowed by ``theta_t``.  Terms of odd index build the downgoing
    focusing function, terms of even index the upgoing one, stored at
    positive time with the opposite sign:

        f1+ = N_{-1} + sum_{i odd} N_i,      f1-(t) = -sum_{i even} N_i(-t).

    Every term also enters the auxiliary field f2+ (all of them, from
    ``N_{-1}`` on) and every synthesis the field p-.  ``norms[i][f]`` is
    ``||N_i||_2``.  The Green's functions follow from the focusing
    functions by two more syntheses (Theory section, after Wapenaar et al.
    2014): ``G-(t) = S[f1+](t) - f1-(t)`` and
    ``G+(t) = f1+(-t) - S[f1-(-.)](t)``; their sum, the total G, is read from
    the auxiliary fields (the route the Theory section attributes to
    Wapenaar et al. 2013): ``G(t) = p-(t) + S[N_last](t) + f2+(-t)``, p-
    completed by the synthesis of the last term.
    """
    Gd = np.asarray(Gd, dtype=np.float64)
    nf = Gd.shape[0]
    keep = mute_window(itd, shift, Gd.shape[-1])

    start = rev(Gd)                            # N_{-1}
    down = start.copy()                        # f1+
    up = np.zeros_like(start)                  # f1-
    f2 = start.copy()                          # f2+
    psum = np.zeros_like(start)                # p-
    norms = np.zeros((niter, nf))
    terms, syntheses = [], []

    term = start
    for i in range(niter):
        s_prev = S(term, fbands)                           # S N_{i-1}
        term = np.where(keep, -rev(s_prev), 0.0)           # N_i = theta(-(S N_{i-1})(-t))
        psum = psum + s_prev
        f2 = f2 + term
        if i % 2 == 1:
            down = down + term
        else:
            up = up - rev(term)
        norms[i] = np.sqrt(np.sum(term * term, axis=(1, 2)))
        if keep_iterates:
            terms.append(term)
            syntheses.append(s_prev)

    Gminus = S(down, fbands) - up
    Gplus = rev(down) - S(rev(up), fbands)
    Gtotal = psum + S(term, fbands) + rev(f2)

    out = dict(f1plus=down, f1minus=up, Gplus=Gplus, Gminus=Gminus,
               f2p=f2, pmin=psum, Gtotal=Gtotal, norms=norms)
    if keep_iterates:
        shape = (0,) + Gd.shape
        out["iterates"] = np.stack(terms) if terms else np.zeros(shape)
        out["synth"] = np.stack(syntheses) if syntheses else np.zeros(shape)
    return out
