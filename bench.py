"""Benchmark of the Marchenko synthesis hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--nf 1]

Workload: 601 x 601 co-located shots/receivers at 5 m, nt = 2048 at 2 ms,
complex64 R (all 1025 rfft bins, 2.96 GB), 8 seeded flat layers plus two
dipping reflectors, focal point(s) on the 500 m deep line, 32 Neumann passes.

One step = one whole solve of the focal batch: mk_set_focal (G_d(-t), first
forward transform), 32 passes of mk_iterate (contraction + fused per-trace
epilogue + FP64 norms), and the G+/G- assembly of mk_get.  All inputs are in
HBM before the timed region starts.  value = Neumann passes per second
(32 x steps / wall time of the steps).

The JSON line adds:
  roofline      the contraction kernel's algorithmic HBM bytes per launch
                divided by its average duration (HIP events on the plan's
                stream, from a separate profiled step), against 8 TB/s;
  cpu_baseline  the FP64 oracle timed on this host on a bounded sample of
                the same workload.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def contract_bytes(nr: int, ns: int, B: int, ncols: int, r_elem_bytes: int = 8) -> int:
    """Algorithmic HBM bytes of one contraction launch: R once, X in, Y out."""
    return r_elem_bytes * nr * ns * B + 8 * ns * B * ncols + 8 * nr * B * ncols


def cpu_baseline(p, passes: int) -> dict:
    """The FP64 oracle on this host: `passes` Neumann passes + its G assembly."""
    from oracle import SynthesisOperator, marchenko

    try:
        from threadpoolctl import threadpool_info

        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    t0 = time.perf_counter()
    S = SynthesisOperator(p.Rhat, p.band, p.c, p.geom.nt)
    t1 = time.perf_counter()
    marchenko(S, p.Gd, p.itd, p.shift, passes)
    t2 = time.perf_counter()
    return {
        "value": passes / (t2 - t1),
        "unit": "iters/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": (f"{passes} Neumann passes plus the G+/G- assembly (2 more syntheses) of the same "
                   f"workload, nf={p.nf}, numpy FP64 (pocketfft + OpenBLAS zgemm); "
                   f"{t2 - t1:.1f} s, R upcast {t1 - t0:.1f} s not counted"),
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nf", type=int, default=1)
    ap.add_argument("--niter", type=int, default=32)
    ap.add_argument("--cpu-passes", type=int, default=32)
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run a plain 1 GiB device copy (calibrates HBM byte counters)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(focal points or receiver rows would shard across GPUs; see the design notes)",
              file=sys.stderr)
        return 2

    import torch

    if args.copy_calib:
        x = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        log("copied 3 x 1 GiB")
        return 0

    from mkgen.layered import make_config
    from paper_2106_04649_amd import mk

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    log(f"generating workload (nf={args.nf})")
    t = time.perf_counter()
    p = make_config("medium", nf=args.nf)
    nr, nt, B = p.Rhat.shape[0], p.geom.nt, p.Rhat.shape[1]
    log(f"generated in {time.perf_counter() - t:.1f} s: R {p.Rhat.nbytes / 1e9:.2f} GB")

    stream = torch.cuda.current_stream()
    R_d = torch.from_numpy(p.Rhat).cuda()
    Gd_d = torch.from_numpy(p.Gd).cuda()
    itd_d = torch.from_numpy(p.itd).cuda()
    out_p = torch.empty(p.Gd.shape, dtype=torch.float32, device="cuda")
    out_m = torch.empty_like(out_p)

    def make_plan(flags=0):
        pl = mk.mk_plan(nr, nr, nt, p.geom.dt, p.geom.dx, band=p.band, nf_max=p.nf, flags=flags,
                        stream=stream.cuda_stream)
        mk.mk_load_R(pl, R_d)
        return pl

    def step(pl):
        mk.mk_set_focal(pl, Gd_d, itd_d, p.shift)
        mk.mk_iterate(pl, args.niter, want_norms=False)
        mk.mk_get(pl, "Gplus", out_p)
        mk.mk_get(pl, "Gminus", out_m)

    plan = make_plan()
    del R_d
    torch.cuda.empty_cache()
    for i in range(args.warmup):
        step(plan)
        log(f"warmup step {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for i in range(args.steps):
        step(plan)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    log(f"timed {args.steps} steps: wall {wall * 1e3:.1f} ms, events {gpu_ms:.1f} ms")
    ms_per_step = wall * 1e3 / args.steps
    value = args.niter * args.steps / wall
    # convergence check outside the timed region: one more solve with norms
    mk.mk_set_focal(plan, Gd_d, itd_d, p.shift)
    norms = mk.mk_iterate(plan, args.niter)
    mk.mk_destroy(plan)

    roof = None
    extra = {}
    if not args.no_profile:
        R_d = torch.from_numpy(p.Rhat).cuda()
        pplan = make_plan(mk.MK_FLAG_PROFILE)
        del R_d
        torch.cuda.empty_cache()
        step(pplan)
        for kind in mk.KERNEL_KINDS:
            mk.mk_profile(pplan, kind, reset=True)
        step(pplan)
        times = {kind: mk.mk_profile(pplan, kind) for kind in mk.KERNEL_KINDS}
        mk.mk_destroy(pplan)
        ms, n = times["contract"]
        avg_s = ms / n / 1e3
        nbytes = contract_bytes(nr, nr, B, p.nf)
        achieved = nbytes / avg_s / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "k_contract_c64", "avg_us": round(avg_s * 1e6, 2),
                "bytes_per_launch": nbytes}
        extra["kernel_ms_per_step"] = {k: round(v[0], 3) for k, v in times.items()}
        extra["kernel_launches_per_step"] = {k: v[1] for k, v in times.items()}
        log(f"contraction avg {avg_s * 1e6:.1f} us -> {achieved:.0f} GB/s "
            f"({achieved / HBM_PEAK_GBS * 100:.1f} % of 8 TB/s)")

    cpu = None
    if not args.no_cpu:
        log(f"timing the FP64 oracle on {args.cpu_passes} passes")
        cpu = cpu_baseline(p, args.cpu_passes)
        log(f"oracle: {cpu['value']:.3f} iters/s on {cpu['cores']} threads")

    rec = {
        "metric": "Marchenko iters/s + HBM TB/s; mixed+learned vs plain FP32 at rel.err 1e-3",
        "value": round(value, 2),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded layered-earth R, analytic direct arrivals)",
        "config": {"workload": f"601x601 shots/receivers, nt=2048, complex64 R 2.96 GB, "
                               f"plain FP32, nf={p.nf}, {args.niter} passes + G assembly",
                   "nr": nr, "ns": nr, "nt": nt, "bins": B, "nf": p.nf, "niter": args.niter,
                   "path": "plain-fp32"},
        "hbm_tbs": round(roof["achieved"] / 1e3, 3) if roof else None,
        "roofline": roof,
        "cpu_baseline": cpu,
        "norm_decay": float((norms[-1] / norms[0]).max()),
    }
    rec.update(extra)
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
