"""Shared helpers of the GPU tests: run the HIP path and the oracle on the same inputs."""

import sys

import numpy as np
import pytest

from oracle import SynthesisOperator, marchenko, rel_l2

FIELD_NAMES = ("f1plus", "f1minus", "Gplus", "Gminus")
TOL_FP32 = 1e-5          # relative L2 per field and focal point for the FP32 path


def require_gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_2106_04649_amd import mk

    mk.load_library()      # raises when the HIP library is missing on a GPU machine
    return mk


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run_gpu(p, niter=None, fbands=None, R=None, flags=0, nf_max=None, on_device=False,
            chunks=None, rprec=0, tune=None):
    """Full solve through the C ABI; returns dict of numpy fields + norms."""
    import torch

    mk = require_gpu()
    niter = p.niter if niter is None else niter
    nr, nt = p.Rhat.shape[0], p.geom.nt
    plan = mk.mk_plan(nr, nr, nt, p.geom.dt, p.geom.dx, band=p.band, nf_max=nf_max or p.nf,
                      flags=flags, rprec=rprec)
    Rin = p.Rhat if R is None else R
    if on_device:
        mk.mk_load_R(plan, torch.from_numpy(np.ascontiguousarray(Rin)).cuda())
    else:
        mk.mk_load_R(plan, Rin)
    if tune is not None:
        mk.mk_tune(plan, tune)
    if on_device:
        mk.mk_set_focal(plan, torch.from_numpy(p.Gd).cuda(), torch.from_numpy(p.itd).cuda(), p.shift,
                        None if fbands is None else torch.from_numpy(fbands).cuda())
    else:
        mk.mk_set_focal(plan, p.Gd, p.itd, p.shift, fbands)
    norms = []
    for n in (chunks or [niter]):
        if n == "G":                       # assemble G between chunks: must not disturb the series
            mk.mk_get(plan, "Gplus", np.zeros((p.nf, nr, nt), np.float32))
        elif n:
            norms.append(mk.mk_iterate(plan, n))
    out = {}
    for name in FIELD_NAMES:
        buf = np.zeros((p.nf, nr, nt), dtype=np.float32)
        mk.mk_get(plan, name, buf)
        out[name] = buf
    out["norms"] = np.concatenate(norms) if norms else np.zeros((0, p.nf))
    out["passes"] = mk.mk_passes(plan)
    out["variant"] = mk.mk_contract_variant(plan, p.nf)
    mk.mk_destroy(plan)
    return out


def run_oracle(p, niter=None, fbands=None):
    S = SynthesisOperator(p.Rhat, p.band, p.c, p.geom.nt)
    return marchenko(S, p.Gd, p.itd, p.shift, p.niter if niter is None else niter, fbands=fbands)


def assert_parity(gpu, ref, tol=TOL_FP32, fields=FIELD_NAMES, label=""):
    worst = {}
    for name in fields:
        errs = [rel_l2(gpu[name][f], ref[name][f]) for f in range(ref[name].shape[0])]
        worst[name] = max(errs)
    nerr = 0.0
    if gpu["norms"].size:
        nerr = float(np.max(np.abs(gpu["norms"] - ref["norms"]) / np.maximum(ref["norms"], 1e-300)))
    say(f"parity {label}: " + ", ".join(f"{k}={v:.2e}" for k, v in worst.items()) + f", norms={nerr:.2e}")
    for name, e in worst.items():
        assert e <= tol, f"{label} {name}: rel-L2 {e:.3e} > {tol:.1e}"
    return worst
