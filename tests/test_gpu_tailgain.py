"""What the trained series-tail network gains, and that the plain iteration
still carries a solve when the network is wrong.

Held-out models of the tail family (301 x 301 at 10 m, nt 1024 at 4 ms,
4-12 layers, half with dipping reflectors, one focal point; seeds that
neither the network's training set nor its validation curve used), against
the FP64 oracle's converged series (40 terms).  The network shipped for this
family (k = 4 recorded passes) runs through the library; every path costs
the same k + 2 syntheses:

* plain: k + 2 passes of the series;
* geometric: k passes, the geometric extrapolation of the parity-split
  tails, and the restart that judges it (two syntheses);
* learned: k passes, the network's tails, and the same restart.

The gain test asserts, for every output field, that the median error over
the models orders learned < geometric < plain, and that the network beats
the geometric tail on most models.  The fallback test loads garbage weights:
the restart's residual flags them, and the library's stopping rule then
runs plain passes until every output is within 1e-3 of the oracle.
"""

import os

import numpy as np
import pytest

from gpu_common import FIELD_NAMES, require_gpu, say
from mkgen.layered import tail_problem
from oracle import SynthesisOperator, marchenko, rel_l2

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "paper_2106_04649_amd", "tailnet_k4.npz")
HELD_OUT = list(range(10016, 10032))


def _network():
    w = np.load(WEIGHTS)
    return w["params"].astype(np.float32), int(w["k"]), int(w["T"])


class _Solver:
    def __init__(self, mk, p, k, T, params):
        self.mk, self.p, self.k = mk, p, k
        nr, nt = p.Rhat.shape[0], p.geom.nt
        self.plan = mk.mk_plan(nr, nr, nt, p.geom.dt, p.geom.dx, band=p.band, nf_max=p.nf)
        mk.mk_load_R(self.plan, p.Rhat)
        mk.mk_tail_record(self.plan, k, T)
        mk.mk_tail_load(self.plan, params)

    def fields(self):
        return {f: self.mk.mk_get(self.plan, f, np.zeros(self.p.Gd.shape, np.float32)) for f in FIELD_NAMES}

    def plain(self, passes):
        self.mk.mk_set_focal(self.plan, self.p.Gd, self.p.itd, self.p.shift)
        self.mk.mk_iterate(self.plan, passes, want_norms=False)
        return self.fields()

    def tail(self, mode):
        self.mk.mk_set_focal(self.plan, self.p.Gd, self.p.itd, self.p.shift)
        self.mk.mk_iterate(self.plan, self.k, want_norms=False)
        resid = self.mk.mk_tail_apply(self.plan, mode)
        return resid

    def destroy(self):
        self.mk.mk_destroy(self.plan)


def _converged(p):
    S = SynthesisOperator(p.Rhat, p.band, p.c, p.geom.nt)
    return marchenko(S, p.Gd, p.itd, p.shift, 40)


def _err(got, ref):
    return {f: rel_l2(got[f][0], ref[f][0]) for f in FIELD_NAMES}


def test_network_beats_geometric_and_plain_on_held_out_models():
    mk = require_gpu()
    params, k, T = _network()
    rows = []
    for seed in HELD_OUT:
        p = tail_problem(seed)
        ref = _converged(p)
        s = _Solver(mk, p, k, T, params)
        row = {"plain": _err(s.plain(k + 2), ref)}
        s.tail(mk.TAIL_GEOMETRIC)
        row["geometric"] = _err(s.fields(), ref)
        s.tail(mk.TAIL_NET)
        row["learned"] = _err(s.fields(), ref)
        s.destroy()
        rows.append(row)
        say(f"seed {seed}: " + "; ".join(f"{name} " + " ".join(f"{row[name][f]:.1e}" for f in FIELD_NAMES)
                                        for name in ("plain", "geometric", "learned")))
    for f in FIELD_NAMES:
        med = {name: float(np.median([r[name][f] for r in rows])) for name in ("plain", "geometric", "learned")}
        wins = sum(r["learned"][f] < r["geometric"][f] for r in rows)
        say(f"{f}: median plain {med['plain']:.2e}, geometric {med['geometric']:.2e}, "
            f"learned {med['learned']:.2e}; learned below geometric on {wins}/{len(rows)} models")
        assert med["learned"] < med["geometric"] < med["plain"], (f, med)
        assert wins >= (3 * len(rows)) // 4, (f, wins)


def test_garbage_weights_are_flagged_and_the_plain_iteration_recovers():
    mk = require_gpu()
    params, k, T = _network()
    rng = np.random.default_rng(3)
    # the trained values shuffled and tripled: weights of the right size and no meaning
    garbage = (3.0 * rng.permutation(params)).astype(np.float32)
    p = tail_problem(HELD_OUT[0])
    ref = _converged(p)
    out = {}
    for name, w in (("trained", params), ("garbage", garbage)):
        s = _Solver(mk, p, k, T, w)
        resid = s.tail(mk.TAIL_NET)
        n, est = mk.mk_iterate_tol(s.plan, 1e-3, 60)
        got = s.fields()
        s.destroy()
        out[name] = (float(resid[0]), n, _err(got, ref), float(est[0]))
        say(f"{name}: judge residual {resid[0]:.2e}, then {n} passes (estimate {est[0]:.1e}); " +
            ", ".join(f"{f}={e:.2e}" for f, e in out[name][2].items()))
    (r_ok, n_ok, e_ok, _), (r_bad, n_bad, e_bad, _) = out["trained"], out["garbage"]
    assert r_bad > 20.0 * r_ok             # the restart's residual exposes the bad tail
    assert n_bad > n_ok                    # the plain iteration does the work instead
    for f in FIELD_NAMES:
        assert e_ok[f] <= 1e-3 and e_bad[f] <= 1e-3, (f, e_ok[f], e_bad[f])
