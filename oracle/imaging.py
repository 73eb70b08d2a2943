"""FP64 oracle of the double-focusing image (test infrastructure only).

TEST INFRASTRUCTURE.  Imported only by ``tests/``, the smoke check and the
benchmark's CPU-baseline leg.

What it follows (arXiv 2106.04649, Theory section, imaging paragraph, and the
last step of Algorithm 1): after the iterations, ``G^-`` and ``f1plus`` of one
focal point are convolved in time and integrated over the surface positions,
which gives ``G^{-,+}(x_F, x_F, t)``; its zero-time sample is the local
reflectivity at ``x_F``, the image.

Readings where the paper is silent:

* the integral over x and t is the Riemann sum with weight ``c = dx * dt``,
  the same discretisation as the synthesis of Eq. (1);
* the time axis is periodic with ``nt`` samples (circular convolution), so
  the zero-time sample is ``c * sum_x sum_t G^-(x, t) f1plus(x, (-t) mod nt)``.

Parity pins (tests/test_imaging_oracle.py): explicit-loop convolution on tiny
inputs, and hand-derived one-receiver spike cases (tests/golden/imaging.json)
run through the oracle's own series: a reflector at the focal depth images to
its reflection coefficient, one below images at its two-way delay, none at
zero time when the focal point lies below every reflector.
"""

from __future__ import annotations

import numpy as np


def double_focused(Gminus: np.ndarray, f1plus: np.ndarray, c: float) -> np.ndarray:
    """``G^{-,+}[f][t] = c * sum_x sum_t' G^-[f][x][(t - t') mod nt] f1plus[f][x][t']``.

    Gminus, f1plus: [nf][nx][nt] real.  The circular time convolution is a
    product of rffts (numpy's FFT as the library primitive), then the sum over x.
    """
    g = np.asarray(Gminus, dtype=np.float64)
    f = np.asarray(f1plus, dtype=np.float64)
    nt = g.shape[-1]
    conv = np.fft.irfft(np.fft.rfft(g, axis=-1) * np.fft.rfft(f, axis=-1), n=nt, axis=-1)
    return c * conv.sum(axis=-2)


def image(Gminus: np.ndarray, f1plus: np.ndarray, c: float) -> np.ndarray:
    """Zero-time sample of ``G^{-,+}`` per focal point, written out as the sum
    ``c * sum_x sum_t G^-[f][x][t] * f1plus[f][x][(-t) mod nt]``: [nf] float64."""
    g = np.asarray(Gminus, dtype=np.float64)
    f = np.asarray(f1plus, dtype=np.float64)
    nt = g.shape[-1]
    f_rev = f[..., (-np.arange(nt)) % nt]
    return c * (g * f_rev).sum(axis=(-2, -1))
