"""Layered-earth reflection responses, direct arrivals and focal geometry.

Everything here is seeded (numpy PCG64) and deterministic.  The shapes follow
the workloads of the paper's benchmark (co-located sources and receivers on a
regular surface grid, a flat-layer "oneD"-style model, hundreds to thousands of
shots, one to many focal points); see the Results section of the paper.

Conventions shared with the library's boundary:

* ``Rhat`` is the unnormalised real-to-complex DFT over time of the reflection
  response (numpy ``rfft`` convention, kernel ``exp(-i 2 pi k n / nt)``) for the
  rfft bins ``w`` in the band ``[lo, hi]``, stored receivers x frequencies x
  shots: ``Rhat[r][w - lo][s]``, complex64.
* ``Gd`` is the time-domain direct arrival ``[nf][nr][nt]`` float32, periodic
  time axis with t = 0 at sample 0.
* ``itd[f][r]`` is the first-arrival time of ``Gd`` in samples (int32).

Events are zero-phase Ricker wavelets centred on hyperbolic (flat layers) or
image-source (dipping planes) travel times.  Each event's travel time and
amplitude are symmetric functions of the source/receiver pair, so the
generated R obeys source-receiver reciprocity bit for bit.
"""

from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np


# ---------------------------------------------------------------------------
# geometry and earth models
# ---------------------------------------------------------------------------


@dataclass(frozen=True)
class Geometry:
    """Co-located surface grid of ``n`` sources/receivers at ``x_i = i*dx``."""

    n: int
    dx: float
    nt: int
    dt: float
    fpeak: float = 25.0

    @property
    def nw(self) -> int:
        return self.nt // 2 + 1

    @property
    def x(self) -> np.ndarray:
        return np.arange(self.n, dtype=np.float64) * self.dx

    @property
    def c(self) -> float:
        """Riemann-sum weight of the double integral of Eq. (1): dx * dt."""
        return self.dx * self.dt


@dataclass
class Dip:
    """A dipping planar reflector seen through a constant-velocity overburden."""

    x0: float      # a point of the plane (m)
    z0: float      # depth of that point (m)
    angle: float   # dip (radians), positive = deepening towards +x
    v: float       # overburden velocity (m/s)
    r: float       # reflection coefficient


@dataclass
class LayerModel:
    """Flat interfaces ``z[k]`` with reflection coefficients ``r[k]``.

    ``v[j]`` is the velocity of the layer above interface ``j``; ``v[K]`` is
    the half-space below the last interface.
    """

    z: np.ndarray
    v: np.ndarray
    r: np.ndarray
    dips: List[Dip] = field(default_factory=list)

    def vertical_time_and_vrms(self, depth: float) -> Tuple[float, float]:
        """One-way vertical time to ``depth`` and the Dix RMS velocity."""
        tops = np.concatenate([[0.0], self.z])
        t = 0.0
        v2t = 0.0
        for j in range(len(self.v)):
            top = tops[j]
            bot = self.z[j] if j < len(self.z) else np.inf
            if depth <= top:
                break
            h = min(depth, bot) - top
            dtj = h / self.v[j]
            t += dtj
            v2t += self.v[j] ** 2 * dtj
        return t, math.sqrt(v2t / t)


def random_layer_model(rng: np.random.Generator, nlayers: int,
                       zrange: Tuple[float, float],
                       vrange: Tuple[float, float] = (1800.0, 3000.0),
                       rrange: Tuple[float, float] = (0.05, 0.2),
                       ndips: int = 0, xrange: Tuple[float, float] = (0.0, 1.0),
                       nabove: int = 0, zsplit: float = 0.0) -> LayerModel:
    """Seeded flat-layer stack; ``nabove`` interfaces are forced above ``zsplit``."""
    z_lo, z_hi = zrange
    if nabove > 0:
        za = rng.uniform(z_lo, zsplit - 20.0, size=nabove)
        zb = rng.uniform(zsplit + 20.0, z_hi, size=nlayers - nabove)
        z = np.sort(np.concatenate([za, zb]))
    else:
        z = np.sort(rng.uniform(z_lo, z_hi, size=nlayers))
    # keep interfaces at least 30 m apart so events stay separable
    for k in range(1, nlayers):
        z[k] = max(z[k], z[k - 1] + 30.0)
    v = np.sort(rng.uniform(vrange[0], vrange[1], size=nlayers + 1))
    r = rng.uniform(rrange[0], rrange[1], size=nlayers) * rng.choice([-1.0, 1.0], size=nlayers)
    dips = []
    for _ in range(ndips):
        dips.append(Dip(x0=rng.uniform(*xrange), z0=rng.uniform(250.0, 900.0),
                        angle=math.radians(rng.uniform(5.0, 20.0)) * rng.choice([-1.0, 1.0]),
                        v=rng.uniform(2000.0, 2500.0),
                        r=rng.uniform(0.05, 0.15) * rng.choice([-1.0, 1.0])))
    return LayerModel(z=z, v=v, r=r, dips=dips)


def ricker_spectrum(f: np.ndarray, fpeak: float) -> np.ndarray:
    """Amplitude spectrum of a unit-peak zero-phase Ricker wavelet."""
    f = np.asarray(f, dtype=np.float64)
    return (2.0 / math.sqrt(math.pi)) * f ** 2 / fpeak ** 3 * np.exp(-(f / fpeak) ** 2)


# ---------------------------------------------------------------------------
# reflection response
# ---------------------------------------------------------------------------


def _flat_offset_table(geom: Geometry, model: LayerModel, freqs: np.ndarray,
                       tmax: float) -> np.ndarray:
    """Sum of flat-layer events as a function of |offset| index: [n][B] complex128."""
    h = np.arange(geom.n, dtype=np.float64) * geom.dx
    tab = np.zeros((geom.n, freqs.size), dtype=np.complex128)
    trans = 1.0
    for k in range(len(model.z)):
        t1, vrms = model.vertical_time_and_vrms(model.z[k])
        t0 = 2.0 * t1
        tau = np.sqrt(t0 ** 2 + (h / vrms) ** 2)
        amp = model.r[k] * trans * np.sqrt(t0 / tau)
        amp = np.where(tau <= tmax, amp, 0.0)
        tab += amp[:, None] * np.exp(-2j * np.pi * freqs[None, :] * tau[:, None])
        trans *= 1.0 - model.r[k] ** 2
    return tab


def _dip_tables(geom: Geometry, model: LayerModel, tmax: float):
    """Symmetric travel-time and amplitude matrices [n][n] of each dipping event."""
    x = geom.x
    out = []
    for d in model.dips:
        nx, nz = -math.sin(d.angle), math.cos(d.angle)          # unit normal of the plane
        dist = nx * (x - d.x0) + nz * (0.0 - d.z0)             # signed distance of surface points
        mx = x - 2.0 * dist * nx                               # mirror image of each surface point
        mz = 0.0 - 2.0 * dist * nz
        tau = np.sqrt((x[:, None] - mx[None, :]) ** 2 + (0.0 - mz[None, :]) ** 2) / d.v
        tau = 0.5 * (tau + tau.T)                              # exact symmetry in (r, s)
        tref = 2.0 * abs(d.z0) * math.cos(d.angle) / d.v
        amp = d.r * np.sqrt(tref / tau)
        amp = np.where(tau <= tmax, amp, 0.0)
        out.append((tau, amp))
    return out


def reflection_response(geom: Geometry, model: LayerModel, band: Tuple[int, int],
                        threads: Optional[int] = None, rows: Optional[Sequence[int]] = None) -> np.ndarray:
    """R-hat in receivers x frequencies x shots layout, complex64 [n][B][n]
    (only the receiver rows ``rows``, in that order, when given)."""
    lo, hi = band
    w = np.arange(lo, hi + 1)
    freqs = w / (geom.nt * geom.dt)
    tmax = 0.45 * geom.nt * geom.dt
    wav = ricker_spectrum(freqs, geom.fpeak) / geom.dt
    flat = _flat_offset_table(geom, model, freqs, tmax) * wav[None, :]   # [h][B]
    dips = _dip_tables(geom, model, tmax)
    n = geom.n
    rlist = list(range(n)) if rows is None else [int(r) for r in rows]
    out = np.empty((len(rlist), w.size, n), dtype=np.complex64)
    sidx = np.arange(n)
    twopi_f = (2.0 * np.pi) * freqs

    def row(j: int) -> None:
        r = rlist[j]
        acc = flat[np.abs(r - sidx)].T.copy()                          # [B][s]
        for tau, amp in dips:
            ph = twopi_f[:, None] * tau[r][None, :]
            acc += (wav[:, None] * amp[r][None, :]) * (np.cos(ph) - 1j * np.sin(ph))
        if lo == 0:
            acc[0].imag = 0.0
        if hi == geom.nt // 2:
            acc[-1].imag = 0.0                                          # rfft of a real trace
        out[j] = acc

    nthreads = threads or min(16, os.cpu_count() or 1)
    if len(rlist) * w.size * n < 4_000_000 or nthreads == 1:
        for j in range(len(rlist)):
            row(j)
    else:
        with ThreadPoolExecutor(max_workers=nthreads) as ex:
            list(ex.map(row, range(len(rlist))))
    return out


def sigma_max_per_freq(Rhat: np.ndarray, wsel: Sequence[int], iters: int = 30,
                       seed: int = 7) -> np.ndarray:
    """Largest singular value of each selected frequency slice (power iteration)."""
    rng = np.random.default_rng(seed)
    out = []
    for w in wsel:
        A = np.ascontiguousarray(Rhat[:, w, :]).astype(np.complex128)
        v = rng.standard_normal(A.shape[1]) + 1j * rng.standard_normal(A.shape[1])
        v /= np.linalg.norm(v)
        s = 0.0
        for _ in range(iters):
            u = A @ v
            v = A.conj().T @ u
            nv = np.linalg.norm(v)
            if nv == 0.0:
                break
            s = math.sqrt(nv)
            v /= nv
        out.append(s)
    return np.asarray(out)


def rho_of(Rhat: np.ndarray, c: float, exact: bool = False) -> float:
    """c * max_w sigma_max(Rhat_w): the bound on the Neumann operator's norm."""
    B = Rhat.shape[1]
    if exact or Rhat.shape[0] <= 128:
        return c * max(np.linalg.norm(Rhat[:, w, :].astype(np.complex128), 2) for w in range(B))
    coarse = list(range(0, B, max(1, B // 48)))
    s = sigma_max_per_freq(Rhat, coarse, iters=8)
    top = np.argsort(s)[-3:]
    cand = set()
    step = max(1, B // 48)
    for t in top:
        for w in range(max(0, coarse[t] - step), min(B, coarse[t] + step + 1), max(1, step // 6)):
            cand.add(w)
    s2 = sigma_max_per_freq(Rhat, sorted(cand), iters=40)
    return c * float(max(s2.max(), s.max()))


# ---------------------------------------------------------------------------
# direct arrivals and focal points
# ---------------------------------------------------------------------------


def direct_arrivals(geom: Geometry, model: LayerModel, xf: np.ndarray, zf: np.ndarray):
    """Time-domain G_d [nf][n][nt] float32 and first-arrival samples itd [nf][n]."""
    nf = len(xf)
    w = np.arange(geom.nw)
    freqs = w / (geom.nt * geom.dt)
    wav = ricker_spectrum(freqs, geom.fpeak) / geom.dt
    Gd = np.empty((nf, geom.n, geom.nt), dtype=np.float32)
    itd = np.empty((nf, geom.n), dtype=np.int32)
    x = geom.x
    for f in range(nf):
        t1, vrms = model.vertical_time_and_vrms(float(zf[f]))
        td = np.sqrt(t1 ** 2 + ((x - xf[f]) / vrms) ** 2)
        amp = np.sqrt(t1 / td)
        spec = (wav[None, :] * amp[:, None]) * np.exp(-2j * np.pi * freqs[None, :] * td[:, None])
        spec[:, -1] = spec[:, -1].real
        Gd[f] = np.fft.irfft(spec, geom.nt, axis=-1).astype(np.float32)
        itd[f] = np.rint(td / geom.dt).astype(np.int32)
    return Gd, itd


@dataclass
class Problem:
    """One seeded workload: everything the boundary's calls take."""

    name: str
    geom: Geometry
    model: LayerModel
    Rhat: np.ndarray            # complex64 [nr][B][ns]
    band: Tuple[int, int]       # inclusive rfft-bin band of Rhat
    Gd: np.ndarray              # float32 [nf][nr][nt]
    itd: np.ndarray             # int32 [nf][nr]
    shift: int                  # mute margin in samples
    niter: int
    fbands: Optional[np.ndarray] = None   # int32 [nf][2] per-focal bands, or None
    xf: Optional[np.ndarray] = None
    zf: Optional[np.ndarray] = None
    rho: float = 0.0
    rscale: float = 1.0

    @property
    def c(self) -> float:
        return self.geom.c

    @property
    def nf(self) -> int:
        return self.Gd.shape[0]


def make_problem(name: str, geom: Geometry, model: LayerModel, xf, zf, niter: int,
                 rho_target: Optional[float] = 0.7, band: Optional[Tuple[int, int]] = None,
                 fbands: Optional[np.ndarray] = None, threads: Optional[int] = None,
                 rho_exact: bool = False) -> Problem:
    band = band or (0, geom.nt // 2)
    Rhat = reflection_response(geom, model, band, threads=threads)
    rho = rho_of(Rhat, geom.c, exact=rho_exact)
    scale = 1.0
    if rho_target is not None and rho > 0.0:
        scale = rho_target / rho
        Rhat *= np.float32(scale)
        rho = rho_target
    Gd, itd = direct_arrivals(geom, model, np.asarray(xf, float), np.asarray(zf, float))
    shift = int(math.ceil(1.0 / (geom.fpeak * geom.dt)))
    return Problem(name=name, geom=geom, model=model, Rhat=Rhat, band=band, Gd=Gd, itd=itd,
                   shift=shift, niter=niter, fbands=fbands, xf=np.asarray(xf, float),
                   zf=np.asarray(zf, float), rho=rho, rscale=scale)


# ---------------------------------------------------------------------------
# the benchmark workloads
# ---------------------------------------------------------------------------

CONFIGS = {
    # 101 x 101 at 10 m, nt 512, dt 4 ms, 3 flat layers at 300-900 m, one focal
    # point at 600 m depth, 16 iterations.
    "tiny": dict(n=101, dx=10.0, nt=512, dt=0.004, nlayers=3, zrange=(300.0, 900.0),
                 ndips=0, niter=16, seed=1001),
    # 601 x 601 at 5 m, nt 2048, dt 2 ms, 8 layers + 2 dipping reflectors,
    # focal points on a 500 m deep line, 32 iterations.
    "medium": dict(n=601, dx=5.0, nt=2048, dt=0.002, nlayers=8, zrange=(150.0, 1400.0),
                   ndips=2, niter=32, seed=1002, nabove=3, zsplit=500.0),
    # medium geometry, 512 focal points at depths 200-1200 m with per-focal
    # bands of 20-80 % of Nyquist.
    "mixed": dict(n=601, dx=5.0, nt=2048, dt=0.002, nlayers=8, zrange=(150.0, 1400.0),
                  ndips=2, niter=32, seed=1003, nabove=3, zsplit=500.0),
    # 2001 x 2001 at 5 m, nt 2048, dt 2 ms, 2048 focal points on a 64 x 32 grid.
    "large": dict(n=2001, dx=5.0, nt=2048, dt=0.002, nlayers=8, zrange=(150.0, 1400.0),
                  ndips=2, niter=32, seed=1005, nabove=3, zsplit=500.0),
}


def make_config(name: str, nf: int = 1, n: Optional[int] = None, nt: Optional[int] = None,
                rho_target: Optional[float] = 0.7, niter: Optional[int] = None,
                threads: Optional[int] = None, seed: Optional[int] = None) -> Problem:
    """Build one of the benchmark workloads (optionally shrunk with ``n``/``nt``)."""
    cfg = dict(CONFIGS[name])
    rng = np.random.default_rng(seed if seed is not None else cfg["seed"])
    dx = cfg["dx"]
    if n is not None and n != cfg["n"]:
        dx = dx * (cfg["n"] - 1) / max(1, n - 1)
    geom = Geometry(n=n or cfg["n"], dx=dx, nt=nt or cfg["nt"],
                    dt=cfg["dt"] * (cfg["nt"] / (nt or cfg["nt"])))
    L = (geom.n - 1) * geom.dx
    model = random_layer_model(rng, cfg["nlayers"], cfg["zrange"], ndips=cfg["ndips"],
                               xrange=(0.3 * L, 0.7 * L), nabove=cfg.get("nabove", 0),
                               zsplit=cfg.get("zsplit", 0.0))
    fbands = None
    if name == "tiny":
        xf = np.full(nf, 0.5 * L)
        zf = np.full(nf, 600.0)
    elif name == "medium":
        xf = np.array([0.5 * L]) if nf == 1 else np.linspace(0.2 * L, 0.8 * L, nf)
        zf = np.full(nf, 500.0)
    elif name == "mixed":
        xf = rng.uniform(0.2 * L, 0.8 * L, size=nf)
        zf = rng.uniform(200.0, 1200.0, size=nf)
        u = rng.uniform(0.2, 0.8, size=nf)
        fbands = np.stack([np.zeros(nf, np.int64), np.rint(u * (geom.nt // 2)).astype(np.int64)],
                          axis=1).astype(np.int32)
    elif name == "large":
        nx = max(1, int(round(math.sqrt(nf * 2))))
        nz = max(1, nf // nx)
        gx, gz = np.meshgrid(np.linspace(0.2 * L, 0.8 * L, nx), np.linspace(200.0, 1200.0, nz))
        xf = gx.ravel()[:nf]
        zf = gz.ravel()[:nf]
    else:
        raise KeyError(name)
    return make_problem(name, geom, model, xf, zf, niter if niter is not None else cfg["niter"],
                        rho_target=rho_target, fbands=fbands, threads=threads)


def tail_problem(seed: int, rho_target: Optional[float] = 0.7, threads: Optional[int] = None,
                 n: int = 301, nt: int = 1024) -> Problem:
    """One model of the series-tail workload: 301 x 301 at 10 m, nt 1024 at 4 ms,
    4-12 flat layers at 100-1400 m, half of the models with 1-2 dipping
    reflectors, one focal point at a seeded position below the third interface."""
    rng = np.random.default_rng(seed)
    geom = Geometry(n=n, dx=10.0 * 300 / max(1, n - 1), nt=nt, dt=0.004 * 1024 / nt)
    L = (geom.n - 1) * geom.dx
    nl = int(rng.integers(4, 13))
    ndips = int(rng.integers(1, 3)) if rng.random() < 0.5 else 0
    model = random_layer_model(rng, nl, (100.0, 1400.0), ndips=ndips, xrange=(0.3 * L, 0.7 * L))
    zf = float(rng.uniform(max(300.0, model.z[min(2, nl - 1)] + 20.0), 1500.0))
    xf = float(rng.uniform(0.3 * L, 0.7 * L))
    return make_problem(f"tail{seed}", geom, model, [xf], [zf], 32, rho_target=rho_target,
                        threads=threads)


def small_problem(n: int = 8, nt: int = 64, nf: int = 1, seed: int = 0,
                  rho_target: Optional[float] = 0.5, nlayers: int = 3,
                  band: Optional[Tuple[int, int]] = None, ndips: int = 1,
                  niter: int = 8) -> Problem:
    """A toy workload small enough for brute force and dense direct solves.

    dt = 4 ms with a 60 Hz wavelet keeps the mute margin at 5 samples, so a
    64-sample trace still has a non-trivial window around t = 0.
    """
    rng = np.random.default_rng(seed)
    geom = Geometry(n=n, dx=10.0, nt=nt, dt=0.004, fpeak=60.0)
    L = (n - 1) * geom.dx
    model = random_layer_model(rng, nlayers, (30.0, 100.0), vrange=(1500.0, 2200.0),
                               rrange=(0.1, 0.3), ndips=ndips, xrange=(0.3 * L, 0.7 * L))
    for d in model.dips:
        d.z0 = float(rng.uniform(40.0, 90.0))
        d.v = float(rng.uniform(1500.0, 1800.0))
    xf = rng.uniform(0.3 * L, 0.7 * L, size=nf)
    zf = rng.uniform(120.0, 150.0, size=nf)
    return make_problem("small", geom, model, xf, zf, niter, rho_target=rho_target,
                        band=band, rho_exact=True)
