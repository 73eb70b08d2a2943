"""GPU (torch) evaluation of the layered-earth reflection response.

Same formulas as ``mkgen.layered.reflection_response`` (flat layers through
an offset table, dipping planes through image sources, zero-phase Ricker),
evaluated on the GPU so that the tail network's training set (hundreds of
models) can be built in seconds.  Values agree with the numpy version to
float32 rounding, not bit for bit; inputs that the FP64 oracle checks are
always built with the numpy version.  Holds none of the Marchenko method's
arithmetic.
"""

from __future__ import annotations

import math
from typing import Optional, Tuple

import numpy as np

from .layered import (CONFIGS, Geometry, LayerModel, Problem, _dip_tables, _flat_offset_table, direct_arrivals,
                      random_layer_model, ricker_spectrum)


def reflection_response_gpu(geom: Geometry, model: LayerModel, band: Tuple[int, int], device="cuda"):
    import torch

    lo, hi = band
    w = np.arange(lo, hi + 1)
    freqs = w / (geom.nt * geom.dt)
    tmax = 0.45 * geom.nt * geom.dt
    wav = ricker_spectrum(freqs, geom.fpeak) / geom.dt
    flat = _flat_offset_table(geom, model, freqs, tmax) * wav[None, :]            # [h][B] complex128
    n = geom.n
    idx = torch.arange(n, device=device)
    absd = (idx[:, None] - idx[None, :]).abs()                                      # [r][s]
    tab = torch.from_numpy(flat.astype(np.complex64)).to(device)                    # [h][B]
    R = tab[absd].permute(0, 2, 1).contiguous()                                     # [r][B][s]
    f_t = torch.from_numpy(freqs).to(device=device, dtype=torch.float64)
    wav_t = torch.from_numpy(wav).to(device=device, dtype=torch.float32)
    for tau, amp in _dip_tables(geom, model, tmax):
        tau_t = torch.from_numpy(tau).to(device)                                   # [r][s] float64
        amp_t = torch.from_numpy(amp).to(device=device, dtype=torch.float32)
        for r0 in range(0, n, 64):
            r1 = min(n, r0 + 64)
            ph = torch.remainder(2.0 * math.pi * f_t[None, :, None] * tau_t[r0:r1, None, :], 2.0 * math.pi)
            ph = ph.to(torch.float32)
            mag = wav_t[None, :, None] * amp_t[r0:r1, None, :]
            R[r0:r1] += torch.complex(mag * torch.cos(ph), -mag * torch.sin(ph))
    if lo == 0:
        R[:, 0, :] = R[:, 0, :].real.to(torch.complex64)
    if hi == geom.nt // 2:
        R[:, -1, :] = R[:, -1, :].real.to(torch.complex64)
    return R


def sigma_max_gpu(R, iters: int = 30, seed: int = 7) -> float:
    """max over frequencies of the largest singular value (batched power iteration)."""
    import torch

    A = R.permute(1, 0, 2).contiguous()                                             # [B][r][s]
    g = torch.Generator(device=R.device).manual_seed(seed)
    v = torch.randn(A.shape[0], A.shape[2], 1, device=R.device, generator=g, dtype=torch.float32)
    v = torch.complex(v, torch.zeros_like(v))
    v = v / torch.linalg.vector_norm(v, dim=1, keepdim=True)
    AH = A.conj().transpose(1, 2).contiguous()
    s = None
    for _ in range(iters):
        u = torch.bmm(A, v)
        v = torch.bmm(AH, u)
        nv = torch.linalg.vector_norm(v, dim=1, keepdim=True)
        s = torch.sqrt(nv.squeeze())
        v = v / torch.clamp(nv, min=1e-30)
    return float(s.max().item())


def tail_problem_gpu(seed: int, rho_target: float = 0.7, n: int = 301, nt: int = 1024, device="cuda") -> Problem:
    """``layered.tail_problem`` with R built on the GPU (Rhat is a CUDA complex64 tensor)."""
    rng = np.random.default_rng(seed)
    geom = Geometry(n=n, dx=10.0 * 300 / max(1, n - 1), nt=nt, dt=0.004 * 1024 / nt)
    L = (geom.n - 1) * geom.dx
    nl = int(rng.integers(4, 13))
    ndips = int(rng.integers(1, 3)) if rng.random() < 0.5 else 0
    model = random_layer_model(rng, nl, (100.0, 1400.0), ndips=ndips, xrange=(0.3 * L, 0.7 * L))
    zf = float(rng.uniform(max(300.0, model.z[min(2, nl - 1)] + 20.0), 1500.0))
    xf = float(rng.uniform(0.3 * L, 0.7 * L))
    band = (0, nt // 2)
    R = reflection_response_gpu(geom, model, band, device)
    rho = geom.c * sigma_max_gpu(R)
    scale = rho_target / rho if rho > 0 else 1.0
    R *= scale
    Gd, itd = direct_arrivals(geom, model, np.array([xf]), np.array([zf]))
    shift = int(math.ceil(1.0 / (geom.fpeak * geom.dt)))
    return Problem(name=f"tail{seed}", geom=geom, model=model, Rhat=R, band=band, Gd=Gd, itd=itd, shift=shift,
                   niter=32, xf=np.array([xf]), zf=np.array([zf]), rho=rho_target, rscale=scale)


def medium_problem_gpu(seed: int, nf: int = 64, rho_target: float = 0.7, n: int = 601, nt: int = 2048,
                       device="cuda") -> Problem:
    """A model of the 601 x 601, nt 2048 workload family (8 layers + 2 dips)
    with nf focal points at random positions and depths 200-1200 m; R on the GPU."""
    rng = np.random.default_rng(seed)
    geom = Geometry(n=n, dx=5.0 * 600 / max(1, n - 1), nt=nt, dt=0.002 * 2048 / nt)
    L = (geom.n - 1) * geom.dx
    model = random_layer_model(rng, 8, (150.0, 1400.0), ndips=2, xrange=(0.3 * L, 0.7 * L), nabove=3,
                               zsplit=500.0)
    xf = rng.uniform(0.2 * L, 0.8 * L, size=nf)
    zf = rng.uniform(200.0, 1200.0, size=nf)
    band = (0, nt // 2)
    R = reflection_response_gpu(geom, model, band, device)
    rho = geom.c * sigma_max_gpu(R)
    scale = rho_target / rho if rho > 0 else 1.0
    R *= scale
    Gd, itd = direct_arrivals(geom, model, xf, zf)
    shift = int(math.ceil(1.0 / (geom.fpeak * geom.dt)))
    return Problem(name=f"medium{seed}", geom=geom, model=model, Rhat=R, band=band, Gd=Gd, itd=itd, shift=shift,
                   niter=32, xf=xf, zf=zf, rho=rho_target, rscale=scale)


def large_setup():
    """Geometry, earth model and focal grid of the 2001 x 2001 workload: the
    draws of ``layered.make_config("large")``, with 2048 focal points on a
    64 x 32 grid (x over the middle 60 %, depths 200-1200 m)."""
    cfg = CONFIGS["large"]
    rng = np.random.default_rng(cfg["seed"])
    geom = Geometry(n=cfg["n"], dx=cfg["dx"], nt=cfg["nt"], dt=cfg["dt"])
    L = (geom.n - 1) * geom.dx
    model = random_layer_model(rng, cfg["nlayers"], cfg["zrange"], ndips=cfg["ndips"], xrange=(0.3 * L, 0.7 * L),
                               nabove=cfg["nabove"], zsplit=cfg["zsplit"])
    gx, gz = np.meshgrid(np.linspace(0.2 * L, 0.8 * L, 64), np.linspace(200.0, 1200.0, 32))
    return geom, model, gx.ravel(), gz.ravel()


def rho_all_bins_gpu(R, c: float, chunk: int = 64, iters: int = 25, seed: int = 7) -> float:
    """c times the largest singular value over every frequency slice of R
    (batched power iteration, ``chunk`` bins at a time)."""
    import torch

    B = R.shape[1]
    g = torch.Generator(device=R.device).manual_seed(seed)
    best = 0.0
    for w0 in range(0, B, chunk):
        A = R[:, w0:w0 + chunk, :].permute(1, 0, 2).contiguous()                  # [b][r][s]
        b, _, ns = A.shape
        v = torch.complex(torch.randn(b, ns, 1, device=R.device, generator=g),
                          torch.randn(b, ns, 1, device=R.device, generator=g))
        v = v / torch.linalg.vector_norm(v, dim=1, keepdim=True)
        s = torch.zeros(b, device=R.device)
        for _ in range(iters):
            u = torch.bmm(A, v)                                                     # A v
            vh = torch.bmm(u.conj().transpose(1, 2).contiguous(), A)               # (A^H u)^H
            v = vh.conj().transpose(1, 2).contiguous()
            nv = torch.linalg.vector_norm(v, dim=1, keepdim=True)
            s = torch.sqrt(nv.reshape(-1))
            v = v / torch.clamp(nv, min=1e-30)
        best = max(best, float(s.max().item()))
        del A
    return c * best


def large_focal(geom: Geometry, model: LayerModel, xf, zf, idx):
    """G_d and itd of the focal points ``idx`` of the large workload's grid."""
    idx = np.asarray(idx, dtype=np.int64)
    return direct_arrivals(geom, model, np.asarray(xf)[idx], np.asarray(zf)[idx])


def large_problem_gpu(focal_idx, rho_target: float = 0.7, device="cuda") -> Problem:
    """The 2001 x 2001, nt 2048 workload with R (complex64, 32.8 GB) on the GPU,
    scaled so that c times its largest singular value is ``rho_target``, and
    G_d for the focal points ``focal_idx`` of the 64 x 32 grid."""
    geom, model, xf, zf = large_setup()
    band = (0, geom.nt // 2)
    R = reflection_response_gpu(geom, model, band, device)
    rho = rho_all_bins_gpu(R, geom.c)
    scale = rho_target / rho if rho > 0 else 1.0
    R *= scale
    Gd, itd = large_focal(geom, model, xf, zf, focal_idx)
    shift = int(math.ceil(1.0 / (geom.fpeak * geom.dt)))
    idx = np.asarray(focal_idx, dtype=np.int64)
    return Problem(name="large", geom=geom, model=model, Rhat=R, band=band, Gd=Gd, itd=itd, shift=shift,
                   niter=32, xf=np.asarray(xf)[idx], zf=np.asarray(zf)[idx], rho=rho_target, rscale=scale)


def direct_arrivals_gpu(geom: Geometry, model: LayerModel, xf, zf, device="cuda"):
    """``layered.direct_arrivals`` evaluated on the GPU: G_d [nf][n][nt] float32
    (a CUDA tensor) and itd [nf][n] int32 (numpy).  Same formula; the values
    agree to float32 rounding."""
    import torch

    xf = np.asarray(xf, dtype=np.float64)
    zf = np.asarray(zf, dtype=np.float64)
    nf = xf.size
    w = np.arange(geom.nw)
    freqs = torch.from_numpy(w / (geom.nt * geom.dt)).to(device)
    wav = torch.from_numpy(ricker_spectrum(w / (geom.nt * geom.dt), geom.fpeak) / geom.dt).to(device)
    x = torch.from_numpy(geom.x).to(device)
    t1v = np.empty(nf)
    vr = np.empty(nf)
    for f in range(nf):
        t1v[f], vr[f] = model.vertical_time_and_vrms(float(zf[f]))
    t1 = torch.from_numpy(t1v).to(device)[:, None]
    vrms = torch.from_numpy(vr).to(device)[:, None]
    td = torch.sqrt(t1 ** 2 + ((x[None, :] - torch.from_numpy(xf).to(device)[:, None]) / vrms) ** 2)   # [nf][n]
    amp = torch.sqrt(t1 / td)
    Gd = torch.empty((nf, geom.n, geom.nt), dtype=torch.float32, device=device)
    for f0 in range(0, nf, 16):
        f1 = min(nf, f0 + 16)
        ph = -2.0 * math.pi * freqs[None, None, :] * td[f0:f1, :, None]
        spec = (wav[None, None, :] * amp[f0:f1, :, None]) * torch.exp(1j * ph)
        spec[..., -1] = spec[..., -1].real
        Gd[f0:f1] = torch.fft.irfft(spec, geom.nt, dim=-1).to(torch.float32)
    itd = torch.round(td / geom.dt).to(torch.int32).cpu().numpy()
    return Gd, itd
