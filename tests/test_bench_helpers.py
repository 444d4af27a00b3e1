"""The FP64 references bench.py reports errors against (CPU): the windowed
Jacobi against a whole-array FP64 Jacobi, and the numpy 7-point adjoint
against the oracle's FP64 adjoint."""
import numpy as np

import bench
import oracle as O


def test_jacobi64_window_matches_whole_array():
    rng = np.random.default_rng(0)
    b0 = rng.random((64, 48), dtype=np.float32)
    W = b0.astype(np.float64)
    for _ in range(7):
        new = W.copy()
        new[1:-1, 1:-1] = (((W[1:-1, :-2] + W[1:-1, 2:]) + W[:-2, 1:-1]) + W[2:, 1:-1]) * 0.25
        W = new
    for r0, r1 in ((0, 10), (20, 30), (50, 64)):
        assert np.array_equal(bench.jacobi64_window(b0, r0, r1, 7), W[r0:r1])


def test_s3d64_adjoint_matches_oracle():
    rng = np.random.default_rng(1)
    u0, w = rng.random((12, 12, 12)), rng.random((12, 12, 12))
    c = np.array([0.28, 0.06, 0.14, 0.09, 0.11, 0.07, 0.13])
    g, gc = bench.s3d64_adjoint(u0, c, 5, w)
    g2, gc2 = O.s3d_adjoint64(u0, c, 5, w)
    assert np.max(np.abs(g - g2)) <= 1e-12 * np.max(np.abs(g2))
    assert np.max(np.abs(gc - gc2)) <= 1e-12 * np.max(np.abs(gc2))
