"""The mixed-precision batched workload at its full size: 601 x 601, nt 2048,
512 focal points at depths 200-1200 m with per-focal bands of 20-80 % of
Nyquist, FP16 R (per-frequency scales, FP32 accumulation), the passes
replayed as a HIP graph -- the launch configuration the benchmark uses for
batches.  Sampled focal points (the band extremes and one in the middle)
are checked against the FP64 oracle run on those focal points alone; the
bar is the 1e-3 relative L2 the mixed path is held to, for the four fields,
the auxiliary f2+ and p-, and (through the bilinear bound c (2 e + e^2)
||G-|| ||f1+||) the double-focusing image."""

import numpy as np
import pytest

from gpu_common import FIELD_NAMES, require_gpu, say
from mkgen.layered import make_config
from oracle import SynthesisOperator, image, marchenko, rel_l2

pytestmark = pytest.mark.gpu


def test_mixed_512_focal_fp16_bands_graph():
    mk = require_gpu()
    import torch

    say("mixed nf=512 fp16 bands graph")
    p = make_config("mixed", nf=512)
    nr, nt = p.Rhat.shape[0], p.geom.nt
    plan = mk.mk_plan(nr, nr, nt, p.geom.dt, p.geom.dx, band=p.band, nf_max=p.nf,
                      rprec=mk.MK_R_F16S, flags=mk.MK_FLAG_GRAPH)
    mk.mk_load_R(plan, torch.from_numpy(p.Rhat).cuda())
    mk.mk_set_focal(plan, torch.from_numpy(p.Gd).cuda(), torch.from_numpy(p.itd).cuda(), p.shift,
                    torch.from_numpy(p.fbands).cuda())
    norms = mk.mk_iterate(plan, p.niter)
    assert np.all(np.isfinite(norms))
    widths = p.fbands[:, 1] - p.fbands[:, 0]
    sample = sorted({int(np.argmin(widths)), int(np.argmax(widths)), p.nf // 2})
    out = {}
    buf = torch.empty(p.Gd.shape, dtype=torch.float32, device="cuda")
    for name in FIELD_NAMES + ("f2plus", "pminus"):
        mk.mk_get(plan, name, buf)
        out[name] = buf[sample].cpu().numpy()
    img = mk.mk_image(plan)[sample]
    mk.mk_destroy(plan)
    del buf
    torch.cuda.empty_cache()

    S = SynthesisOperator(p.Rhat, p.band, p.c, nt)
    ref = marchenko(S, p.Gd[sample], p.itd[sample], p.shift, p.niter, fbands=p.fbands[sample])
    for name, rname in [(n, n) for n in FIELD_NAMES] + [("f2plus", "f2p"), ("pminus", "pmin")]:
        e = max(rel_l2(out[name][j], ref[rname][j]) for j in range(len(sample)))
        say(f"  {name}: {e:.2e} (focal points {sample})")
        assert e <= 1e-3, (name, e)
    want = image(ref["Gminus"], ref["f1plus"], p.c)
    for j in range(len(sample)):
        bound = p.c * np.linalg.norm(ref["Gminus"][j]) * np.linalg.norm(ref["f1plus"][j])
        say(f"  image focal {sample[j]}: {img[j]:.6e} oracle {want[j]:.6e} |diff|/bound "
            f"{abs(img[j] - want[j]) / bound:.2e}")
        assert abs(img[j] - want[j]) <= 1e-3 * (2 + 1e-3) * bound
