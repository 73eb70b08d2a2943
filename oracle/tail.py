"""FP64 reference of the series-tail extension (test infrastructure only).

After k passes of Algorithm 1 the remaining terms of the Neumann series are
estimated per trace and added to the focusing functions:

    T_even = sum_{i >= k, i even} N_i  ->  f1- -= T_even(-t)
    T_odd  = sum_{i >= k, i odd}  N_i  ->  f1+ += T_odd

(the same accumulation rule as the series itself).  The
estimate is then judged and refined by plain synthesis: one fixed-point
step of the converged relations (Theory section; f1+ = G_d(-t) + A^2 f1+
and f1- = theta S f1+, with A = theta Rev S),

    f1-  <- theta S f1+,         f1+ <- G_d(-t) + A^2 f1+,

whose residual rho = G_d(-t) + A^2 f1+ - f1+ starts a new Neumann series
carrying the remaining error (odd terms into f1+, even terms into f1- as
in Algorithm 1).  Without a tail estimate this is exactly two more passes of
the original series.

Windows: recorded sample u of a trace holds t = u - T/2.
"""

from __future__ import annotations

import numpy as np

from . import tailnet
from .marchenko import apply_mute, mute_window, rev, signed_time


def window(x: np.ndarray, T: int) -> np.ndarray:
    """[..., nt] -> [..., T] samples t = -T/2 .. T/2 - 1 of the periodic axis."""
    nt = x.shape[-1]
    idx = (np.arange(T) - T // 2) % nt
    return x[..., idx]


def unwindow(w: np.ndarray, nt: int) -> np.ndarray:
    """Inverse of window(): place [..., T] back on [..., nt] (zeros elsewhere)."""
    T = w.shape[-1]
    out = np.zeros(w.shape[:-1] + (nt,))
    out[..., (np.arange(T) - T // 2) % nt] = w
    return out


def history(iterates: np.ndarray, k: int, T: int) -> np.ndarray:
    """[niter][nf][nr][nt] iterates -> [nf][nr][k][T] windows of N_0 .. N_{k-1}."""
    return np.stack([window(iterates[i], T) for i in range(k)], axis=2)


def geometric_tails(hist: np.ndarray):
    """Per trace, N_{i+2} ~ q N_i with q the norm ratio of the last two iterates of a parity."""
    k = hist.shape[2]
    n = np.sqrt((hist.astype(np.float64) ** 2).sum(axis=-1))     # [nf][nr][k]

    def ratio(a, b):
        return np.where(n[..., b] > 0, np.minimum(n[..., a] / np.where(n[..., b] > 0, n[..., b], 1.0), 0.9), 0.0)

    qe = ratio(k - 2, k - 4)
    qo = ratio(k - 1, k - 3)
    te = (qe / (1 - qe))[..., None] * hist[:, :, k - 2, :]
    to = (qo / (1 - qo))[..., None] * hist[:, :, k - 1, :]
    return te, to


def net_tails(hist: np.ndarray, P: dict, f16: bool = False):
    """Tails from the network: input normalised by the RMS of N_0 on the window;
    ``f16`` selects the inference form with half-precision activations."""
    nf, nr, k, T = hist.shape
    h = hist.reshape(nf * nr, k, T).astype(np.float64)
    s = np.sqrt((h[:, 0, :] ** 2).mean(axis=-1))
    inv = np.where(s > 1e-30, 1.0 / np.where(s > 1e-30, s, 1.0), 0.0)
    if f16:
        y = tailnet.forward_f16(P, h * inv[:, None, None])
    else:
        y, _ = tailnet.forward(P, h * inv[:, None, None])
    s = np.where(inv > 0, s, 0.0)
    te = (s[:, None] * y[:, 0, :]).reshape(nf, nr, T)
    to = (s[:, None] * y[:, 1, :]).reshape(nf, nr, T)
    return te, to


def apply_tails(f1p, f1m, te, to, itd, shift):
    """f1+ += T_odd and f1- -= T_even(-t), inside the mute window only."""
    nt = f1p.shape[-1]
    T = te.shape[-1]
    keep = window(mute_window(itd, shift, nt).astype(float), T)
    return f1p + unwindow(keep * to, nt), f1m - rev(unwindow(keep * te, nt))


def restart(S, Gd, itd, shift, f1p, fbands=None, niter=0):
    """Fixed-point step from f1+, then `niter` passes of the residual series."""
    n0 = rev(np.asarray(Gd, dtype=np.float64))

    def step(x):                                   # -A x = theta(-Rev S x)
        return apply_mute(-rev(S(x, fbands)), itd, shift)

    f1m = apply_mute(S(f1p, fbands), itd, shift)   # theta S f1+
    a2 = step(step(f1p))                           # A^2 f1+
    rho = n0 + a2 - f1p
    f1p = n0 + a2
    N = rho
    norms = []
    for it in range(niter):
        N = step(N)
        if it % 2 == 0:
            f1m = f1m - rev(N)
        else:
            f1p = f1p + N
        norms.append(np.sqrt((N * N).sum(axis=(1, 2))))
    norms = np.array(norms) if norms else np.zeros((0, f1p.shape[0]))
    return f1p, f1m, rho, norms


def g_fields(S, f1p, f1m, fbands=None):
    """(G+, G-) with G+ = f1+(-t) - S f1-(-t) and G- = S f1+ - f1- (Algorithm 1, Theory section)."""
    return rev(f1p) - S(rev(f1m), fbands), S(f1p, fbands) - f1m
