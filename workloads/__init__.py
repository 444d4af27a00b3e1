"""Seeded synthetic inputs for the five ApplyKernel workloads.

This module only draws numbers: array values, sizes, partition counts and
irregular cut points.  It holds none of the method's arithmetic (no regions,
no splits, no communication sets, no kernels), so both the HIP path and the
CPU oracle may use it.  Every draw comes from ``numpy.random.default_rng``
with a fixed seed, in the order documented per function.

Workloads (stand-ins for the paper's PolyBench/ACC GEMM and Jacobi inputs,
which are not available; shapes follow the paper's kernels scaled to one
GPU's share):

  jacobi_small   256 x 256 fp32 U[0,1), 4 row partitions, 10 iterations
  jacobi_large   8192 x 8192 fp32 U[0,1), 4 x 4 block partitions, 100 iterations
  matmul         4096 x 4096 fp32 A, B U[-1,1), 8 row partitions
  batched        64 independent 2-D arrays, sides log-uniform in [512, 4096],
                 2..32 irregular row partitions, stencil or lower-triangular
  stencil3d      512^3 fp32 U[0,1) (and a 32^3 copy), 2 x 2 x 2 blocks, T = 64
"""
import numpy as np

JACOBI_SMALL = dict(name="jacobi_small", n=256, ndev=4, iters=10, seed=1)
JACOBI_LARGE = dict(name="jacobi_large", n=8192, ndev=16, iters=100, seed=2)
MATMUL = dict(name="matmul", n=4096, ndev=8, seed=3)
BATCHED = dict(name="batched", narrays=64, side_min=512, side_max=4096, pmin=2, pmax=32, steps=50, seed=4)
STENCIL3D = dict(name="stencil3d", n=512, n_small=32, ndev=8, T=64, ckpt=8, seed=5)

# 7-point stencil weights (centre, -i, +i, -j, +j, -k, +k), rounded to fp32.
# Their sum is 0.88 < 1 (contractive) and the +/- pairs differ, so a mirrored
# adjoint shows up as an error.
S3D_COEFFS = np.array([0.28, 0.06, 0.14, 0.09, 0.11, 0.07, 0.13], dtype=np.float32)

# 3 x 3 convolution weights (row by row over the window), rounded to fp32;
# no two are equal and the sum is 0.95 < 1, so a transposed or mirrored
# window and a dropped term all change the result.
CONV9_WEIGHTS = np.array([0.03, 0.12, 0.05, 0.10, 0.31, 0.08, 0.06, 0.11, 0.09], dtype=np.float32)


def uniform01(shape, rng):
    """U[0,1) fp32 (multiples of 2^-24, no subnormals)."""
    return rng.random(shape, dtype=np.float32)


def uniform_pm1(shape, rng):
    """U[-1,1) fp32: 2u - 1 is exact in fp32 for u a multiple of 2^-24."""
    return (2.0 * rng.random(shape, dtype=np.float32) - 1.0).astype(np.float32)


def jacobi_inputs(n, seed):
    """Two n x n U[0,1) arrays (A, B), drawn A then B."""
    rng = np.random.default_rng(seed)
    return uniform01((n, n), rng), uniform01((n, n), rng)


def matmul_inputs(n, seed):
    """A, B in U[-1,1), drawn A then B."""
    rng = np.random.default_rng(seed)
    return uniform_pm1((n, n), rng), uniform_pm1((n, n), rng)


def ternary_matmul_inputs(n, seed):
    """Integer-valued A, B in {-1, 0, 1} (every partial sum exact in fp32 for n < 2^24)."""
    rng = np.random.default_rng(seed)
    return (rng.integers(-1, 2, (n, n)).astype(np.float32), rng.integers(-1, 2, (n, n)).astype(np.float32))


def batched_instance(seed=4, narrays=64, side_min=512, side_max=4096, pmin=2, pmax=32, scale=1.0):
    """Metadata of the batched workload, drawn from default_rng(seed) in order,
    for each array: kind (0 = 5-point stencil, 1 = lower-triangular, p = 1/2);
    stencil: H then W, each round(exp(U(ln side_min, ln side_max)));
    triangular: one side n from the same law (square array);
    then P ~ U{pmin..pmax} partitions and P-1 distinct sorted cut rows from
    [1, H-1].  ``scale`` shrinks the sides (for CPU-sized copies) before the
    partition draws; the draw sequence is unchanged.
    Array values come from ``batched_values(seed, i, shape)``."""
    rng = np.random.default_rng(seed)
    lo, hi = np.log(side_min), np.log(side_max)
    out = []
    for i in range(narrays):
        kind = int(rng.random() < 0.5)
        if kind == 0:
            H = int(round(np.exp(rng.uniform(lo, hi))))
            W = int(round(np.exp(rng.uniform(lo, hi))))
        else:
            H = int(round(np.exp(rng.uniform(lo, hi))))
            W = H
        if scale != 1.0:
            H = max(int(round(H * scale)), 8)
            W = H if kind == 1 else max(int(round(W * scale)), 8)
        P = int(rng.integers(pmin, pmax + 1))
        P = min(P, H - 1)
        cuts = np.sort(rng.choice(np.arange(1, H), size=P - 1, replace=False)).astype(np.int64)
        out.append(dict(index=i, kind=kind, shape=(H, W), P=P, cuts=cuts))
    return out


def batched_values(seed, index, shape):
    """Values of array ``index`` of the batched workload: two U[0,1) arrays
    (A, B) from default_rng([seed, index])."""
    rng = np.random.default_rng([seed, index])
    return uniform01(shape, rng), uniform01(shape, rng)


def stencil3d_inputs(n, seed=5):
    """u0 and the loss weights w, both U[0,1) fp32 of shape (n, n, n), drawn u0 then w."""
    rng = np.random.default_rng([seed, n])
    return uniform01((n, n, n), rng), uniform01((n, n, n), rng)
