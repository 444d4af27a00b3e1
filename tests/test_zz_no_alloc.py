"""hdarray_reduce_noalloc against hdarray_reduce, through the C ABI.

Two calls in a row, the second on a smaller array: for each, the array is
written over row partitions, one Jacobi step defines it, and the reduce uses
a block partition, so the reduce's communication step moves data.  The
no-allocation call must give the same bits as hdarray_reduce (same kernels,
same combination order) and leave the library's allocation count unchanged;
without an earlier hdarray_reduce on the same array and partition it must
refuse with HD_ENOPLAN and run nothing.
"""
import sys

import numpy as np
import pytest

from workloads import jacobi_inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def hd():
    import paper_1809_05657_amd as hdm
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    hdm.load()
    return hdm


def _case(hd, rt, n, ndev_rows, ndev_blocks, seed):
    A0, B0 = jacobi_inputs(n, seed)
    A, B = rt.create(A0), rt.create(B0)
    pr = rt.partition(hd.ROW, (n, n), ndev=ndev_rows)
    kname = f"jac{n}"
    rt.kernel(kname, hd.K_JACOBI2D)
    rt.set_offsets(kname, 1, 0, [(0, 0), (0, -1), (0, 1), (-1, 0), (1, 0)])
    rt.set_offsets(kname, 0, 1, [(0, 0)])
    rt.write(A, A0, pr)
    rt.write(B, B0, pr)
    rt.apply(kname, pr, [A, B])
    g = (A, B, pr)
    pb = rt.partition(hd.BLOCK, (n, n), ndev=ndev_blocks)
    iv = (np.arange(n * n, dtype=np.int64).reshape(n, n) * 7919 - 3 * n * n).astype(np.int32)
    ivn = iv | 1  # odd values: the wrapped integer product never collapses to zero
    Ig = rt.create(shape=(n, n), type_=hd.I32)
    rt.write(Ig, ivn, g[2])
    D0 = np.random.default_rng(seed).random((n, n)) + 0.5
    Dg = rt.create(shape=(n, n), type_=hd.F64)
    rt.write(Dg, D0, g[2])
    return [g[0], Ig, Dg], pb


def test_reduce_noalloc_matches_reduce(hd):
    rt = hd.Runtime()
    for n, nr, nb, seed in ((300, 6, 16, 11), (70, 3, 4, 12)):
        say(f"case reduce_noalloc n={n} rows={nr} blocks={nb}")
        arrs, pb = _case(hd, rt, n, nr, nb, seed)
        for arr in arrs:
            for op in (hd.SUM, hd.PROD, hd.MAX, hd.MIN):
                ref = rt.reduce(arr, op, pb)
                a0 = rt.stats()["allocs"]
                got = rt.reduce_noalloc(arr, op, pb)
                assert rt.stats()["allocs"] == a0, "the no-allocation reduce allocated"
                dt = arr.dtype
                assert np.array_equal(np.array([got], dt).view(np.uint8), np.array([ref], dt).view(np.uint8)), \
                    f"n={n} {dt} op={op}: {got!r} != {ref!r}"
        # a second call in a row on the same array gives the same bits again
        again = rt.reduce_noalloc(arrs[0], hd.SUM, pb)
        assert np.float32(again) == np.float32(rt.reduce(arrs[0], hd.SUM, pb))
    rt.close()


def test_reduce_noalloc_needs_plan(hd):
    rt = hd.Runtime()
    n = 32
    A = rt.create(np.ones((n, n), np.float32))
    p = rt.partition(hd.ROW, (n, n), ndev=2)
    a0 = rt.stats()["allocs"]
    with pytest.raises(hd.HDArrayError) as e:
        rt.reduce_noalloc(A, hd.SUM, p)
    assert e.value.code == hd.ENOPLAN
    assert rt.stats()["allocs"] == a0
    assert rt.reduce(A, hd.SUM, p) == n * n
    assert rt.reduce_noalloc(A, hd.SUM, p) == n * n
    rt.close()
