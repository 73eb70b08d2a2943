"""The seeded input generators (mkgen): the row-subset form of R used by the
full-size checks, reciprocity, and the torch evaluation of the same formulas
(run on the CPU here)."""

import numpy as np

from mkgen.layered import direct_arrivals, reflection_response, small_problem


def test_row_subset_matches_full_R():
    p = small_problem(seed=5, n=24, nt=64, ndips=2)
    R = reflection_response(p.geom, p.model, p.band)
    rows = [17, 0, 23, 5]
    assert np.array_equal(reflection_response(p.geom, p.model, p.band, rows=rows), R[rows])


def test_R_is_reciprocal():
    p = small_problem(seed=6, n=20, nt=64, ndips=2)
    R = reflection_response(p.geom, p.model, p.band)
    assert np.array_equal(R, R.transpose(2, 1, 0))


def test_torch_generators_match_numpy():
    from mkgen.torchgen import direct_arrivals_gpu, large_setup, reflection_response_gpu

    p = small_problem(seed=7, n=30, nt=128, ndips=2)
    R = reflection_response(p.geom, p.model, p.band)
    Rt = reflection_response_gpu(p.geom, p.model, p.band, device="cpu").numpy()
    assert np.abs(Rt - R).max() <= 1e-6 * np.abs(R).max()
    xf, zf = np.array([60.0, 150.0]), np.array([70.0, 90.0])
    G, itd = direct_arrivals(p.geom, p.model, xf, zf)
    Gt, itdt = direct_arrivals_gpu(p.geom, p.model, xf, zf, device="cpu")
    assert np.array_equal(itd, itdt)
    assert np.abs(Gt.numpy() - G).max() <= 1e-6 * np.abs(G).max()
    geom, model, gx, gz = large_setup()
    assert geom.n == 2001 and geom.nt == 2048 and len(gx) == 2048
    assert gx.min() == 0.2 * 10000.0 and gz.max() == 1200.0
