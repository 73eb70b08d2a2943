"""HIP-graph replay of the passes: every replay equals the eager passes bit
for bit, with eager work and synchronisations between replays."""

import numpy as np
import pytest

from gpu_common import FIELD_NAMES, require_gpu, say
from mkgen.layered import small_problem

pytestmark = pytest.mark.gpu


def _fields(mk, plan, shape):
    out = {}
    for k in FIELD_NAMES:
        out[k] = mk.mk_get(plan, k, np.zeros(shape, np.float32))
    return out


@pytest.mark.parametrize("rprec,nf,use_stream", [(0, 2, False), (1, 12, True), (0, 9, True)])
def test_graph_replays_match_eager(rprec, nf, use_stream):
    mk = require_gpu()
    import torch

    say(f"graph rprec={rprec} nf={nf} stream={use_stream}")
    p = small_problem(seed=61, n=40, nt=128, nf=nf, niter=8)
    stream = torch.cuda.Stream() if use_stream else None
    sid = stream.cuda_stream if stream is not None else 0
    eager = mk.mk_plan(40, 40, 128, p.geom.dt, p.geom.dx, nf_max=nf, rprec=rprec, stream=sid)
    graph = mk.mk_plan(40, 40, 128, p.geom.dt, p.geom.dx, nf_max=nf, rprec=rprec, stream=sid,
                       flags=mk.MK_FLAG_GRAPH)
    for pl in (eager, graph):
        mk.mk_load_R(pl, p.Rhat)
    shape = p.Gd.shape
    for rep in range(3):
        Gd = (p.Gd * np.float32(1.0 + 0.25 * rep)).astype(np.float32)
        res = []
        for pl in (eager, graph):
            mk.mk_set_focal(pl, Gd, p.itd, p.shift)
            n1 = mk.mk_iterate(pl, 3)
            mid = _fields(mk, pl, shape)              # eager G assembly between replays
            torch.cuda.synchronize()
            n2 = mk.mk_iterate(pl, 3)
            n3 = mk.mk_iterate(pl, 2)
            res.append((np.concatenate([n1, n2, n3]), mid, _fields(mk, pl, shape)))
        (na, ma, fa), (nb, mb, fb) = res
        assert np.array_equal(na, nb), f"norms differ at replay {rep}"
        for k in FIELD_NAMES:
            assert np.array_equal(ma[k], mb[k]), f"{k} (mid) differs at replay {rep}"
            assert np.array_equal(fa[k], fb[k]), f"{k} differs at replay {rep}"
    mk.mk_destroy(eager)
    mk.mk_destroy(graph)


def test_graph_cache_follows_focal_state():
    """Replays across focal sets that change the batch width, the mute margin
    and the bands (each needs its own executable) equal the eager passes."""
    mk = require_gpu()
    say("graph cache across focal states")
    p = small_problem(seed=62, n=40, nt=128, nf=6, niter=8)
    eager = mk.mk_plan(40, 40, 128, p.geom.dt, p.geom.dx, nf_max=6)
    graph = mk.mk_plan(40, 40, 128, p.geom.dt, p.geom.dx, nf_max=6, flags=mk.MK_FLAG_GRAPH)
    for pl in (eager, graph):
        mk.mk_load_R(pl, p.Rhat)
    band = np.array([[0, 40], [3, 64], [0, 64], [5, 30], [0, 50], [2, 64]], np.int32)
    states = [(6, p.shift, None), (4, p.shift, None), (6, p.shift + 3, None), (6, p.shift, band),
              (4, p.shift, None), (6, p.shift, None)]
    for nf, shift, bd in states:
        res = []
        for pl in (eager, graph):
            mk.mk_set_focal(pl, p.Gd[:nf], p.itd[:nf], shift, None if bd is None else bd[:nf])
            n1 = mk.mk_iterate(pl, 3)
            n2 = mk.mk_iterate(pl, 4)
            res.append((np.concatenate([n1, n2]), _fields(mk, pl, (nf,) + p.Gd.shape[1:])))
        (na, fa), (nb, fb) = res
        assert np.array_equal(na, nb), (nf, shift, bd is not None)
        for k in FIELD_NAMES:
            assert np.array_equal(fa[k], fb[k]), (k, nf, shift, bd is not None)
    mk.mk_destroy(eager)
    mk.mk_destroy(graph)
