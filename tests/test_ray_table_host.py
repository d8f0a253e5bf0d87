"""The plan's ray table (osscir_ray_table: host computation in the library,
no device) evaluated with the kernels' chord formula in FP32 on the CPU,
against the oracle's exact chords: every (ray, pixel) weight of X.

The formula is emulated here from its statement in include/osscir.h (FP64
signed distance, rounded once to FP32, FP32 trapezoid), so this checks the
plan's geometry, including rays lying exactly on a pixel edge (even n, odd
n_bins, views at multiples of 90 degrees), without a GPU."""
import os

import numpy as np
import pytest

import synth
from oracle import projector as pj

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1801_06263_amd", "libosscir.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libosscir.so not built")


def library_weights(geom):
    """Dense [L, n*n] of the library's FP32 chord weights (cm)."""
    from paper_1801_06263_amd.osscir import ray_table
    rays, src = ray_table(geom)
    n = geom.n
    iy, ix = np.divmod(np.arange(n * n), n)
    v = np.repeat(np.arange(geom.n_views), geom.n_bins)
    dx = src[v, 0][:, None] - ix[None, :].astype(np.float64)
    dy = src[v, 1][:, None] - iy[None, :].astype(np.float64)
    sigk = rays[:, 0:1] * dx + rays[:, 1:2] * dy
    ak = rays[:, 2:3].astype(np.float32)
    hmax = rays[:, 3:4].astype(np.float32)
    w = ak - np.abs(sigk.astype(np.float32))
    return np.clip(w, np.float32(0.0), hmax).astype(np.float64)


@pytest.mark.parametrize("args", [(8, 20.0, 4, 3), (16, 20.0, 8, 33), (64, 20.0, 64, 127), (12, 20.0, 4, 21),
                                  (16, 20.0, 12, 32), (15, 20.0, 8, 33)])
def test_library_chords_equal_oracle(args):
    geom = synth.make_geometry(*args)
    W = library_weights(geom)
    X = pj.system_matrix(geom).toarray()
    pix = geom.pixel_cm
    # FP32 weights: a few ulps of the pixel size
    assert np.abs(W - X).max() <= 4e-6 * pix
    # the same nonzero pattern except sub-ulp grazing chords
    diff = (W > 0) != (X > 0)
    assert np.all(np.minimum(W, X)[diff] == 0) and np.all(np.maximum(W, X)[diff] <= 4e-6 * pix)


@pytest.mark.parametrize("args", [(8, 20.0, 4, 3), (16, 20.0, 8, 33), (64, 20.0, 64, 127)])
def test_rays_on_a_pixel_edge_are_counted_once(args):
    # even n and odd n_bins: the detector-centre ray of every view at a
    # multiple of 90 degrees lies on the grid line through the isocentre
    geom = synth.make_geometry(*args)
    W = library_weights(geom).reshape(geom.n_views, geom.n_bins, geom.n, geom.n)
    c = (geom.n_bins - 1) // 2
    for v in range(0, geom.n_views, geom.n_views // 4):
        w = W[v, c]
        assert abs(w.sum() - geom.n * geom.pixel_cm) <= 1e-5 * geom.n * geom.pixel_cm
        # one row (or column) of full chords, on the + side of the edge
        rows, cols = np.nonzero(w)
        if v % (geom.n_views // 2) == 0:
            assert set(rows) == {geom.n // 2} and len(cols) == geom.n
        else:
            assert set(cols) == {geom.n // 2} and len(rows) == geom.n
        np.testing.assert_allclose(w[w > 0], geom.pixel_cm, rtol=1e-6)


def test_oracle_counts_an_edge_ray_once():
    # the oracle's half-open pixels: brute-force clipping counts a line on a
    # shared edge in both closed squares; the matrix keeps the + side only
    geom = synth.make_geometry(8, 20.0, 4, 3)
    X = pj.system_matrix(geom).toarray().reshape(4, 3, 8, 8)
    B = pj.dense_matrix_bruteforce(geom).reshape(4, 3, 8, 8)
    for v in range(4):
        assert X[v, 1].sum() == pytest.approx(20.0, rel=1e-12)
        assert B[v, 1].sum() == pytest.approx(40.0, rel=1e-12)   # both closed squares
        on_plus = X[v, 1][4, :] if v % 2 == 0 else X[v, 1][:, 4]
        np.testing.assert_allclose(on_plus, 2.5, rtol=1e-12)
    # every other ray: Siddon equals brute force
    np.testing.assert_allclose(np.delete(X, 1, axis=1), np.delete(B, 1, axis=1), atol=1e-12)
