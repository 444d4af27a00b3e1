"""The parity cases of the 2-D paths again with compact buffer windows
(init option --hd-windows=compact: a device keeps only a box around the
sections it holds or reads, with its own row stride), and the window
growth paths: a stencil on compact windows followed by calls that need the
whole array (matmul, device pointers).  Same bar as the default layout:
messages, pack buffers, GDEF and stencil data bit-exact with the oracle."""
import sys

import numpy as np
import pytest

import oracle as O
from tests.test_gpu_parity import (same_call, test_block_parity, test_conv2d_parity, test_degenerate_parity,
                                   test_random_programs_parity, test_stencil_shapes_parity, test_trapezoid_parity)
from workloads import programs as prog
from workloads import matmul_inputs

pytestmark = pytest.mark.gpu

__all__ = ["test_block_parity", "test_conv2d_parity", "test_degenerate_parity", "test_random_programs_parity",
           "test_stencil_shapes_parity", "test_trapezoid_parity"]


class _Compact:
    """The binding module with compact windows as the runtime default."""

    def __init__(self, m):
        self._m = m

    def __getattr__(self, k):
        return getattr(self._m, k)

    def Runtime(self, *a, **kw):
        kw.setdefault("windows", "compact")
        return self._m.Runtime(*a, **kw)


@pytest.fixture(scope="module")
def hd():
    import paper_1809_05657_amd as hdm
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    hdm.load()
    return _Compact(hdm)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_window_growth_matmul(hd):
    """Jacobi steps on compact windows (4 blocks), then C = A.B with the row
    split on the same arrays (the matmul indexes whole arrays: every window
    grows to the whole array, keeping what the devices hold), then Jacobi
    again."""
    n, P = 96, 4
    say(f"case window growth matmul n={n} P={P}")
    a0, b0 = matmul_inputs(n, 21)
    rt, orc = hd.Runtime(), O.Oracle()
    g = prog.jacobi_blocks(rt, a0, b0, P)
    o = prog.jacobi_blocks(orc, a0, b0, P)
    pairs = [(g[0], o[0]), (g[1], o[1])]
    for step in range(3):
        k, ag, ao = ("jacAB", [g[0], g[1]], [o[0], o[1]]) if step % 2 == 0 else ("jacBA", [g[1], g[0]], [o[1], o[0]])
        rt.apply(k, g[2], ag)
        orc.apply(k, o[2], ao)
        same_call(rt, orc, pairs, f"jacobi {step}")
    mm = []
    for api, (A, B, _) in ((rt, g), (orc, o)):
        Cc = api.create(shape=(n, n))
        p = api.partition(prog.ROW, (n, n), ndev=P)
        api.kernel("gemm", prog.K_MATMUL)
        api.set_offsets("gemm", 0, 0, [(0, "*")])
        api.set_offsets("gemm", 1, 0, [("*", 0)])
        api.set_offsets("gemm", 2, 1, [(0, 0)])
        api.apply("gemm", p, [A, B, Cc])
        mm.append((Cc, p))
    same_call(rt, orc, pairs + [(mm[0][0], mm[1][0])], "gemm", pack=True)
    ag, bg = rt.read(g[0], g[2]), rt.read(g[1], g[2])
    ao, bo = orc.read(o[0], o[2]), orc.read(o[1], o[2])
    assert np.array_equal(ag, ao) and np.array_equal(bg, bo)
    cg = rt.read(mm[0][0], mm[0][1]).astype(np.float64)
    ref = ao.astype(np.float64) @ bo.astype(np.float64)
    bound = n * 2.0 ** -24 * (np.abs(ao).astype(np.float64) @ np.abs(bo).astype(np.float64))
    assert np.all(np.abs(cg - ref) <= bound)
    rt.apply("jacBA", g[2], [g[1], g[0]])
    orc.apply("jacBA", o[2], [o[1], o[0]])
    same_call(rt, orc, pairs, "jacobi after growth")
    assert np.array_equal(rt.read(g[1], g[2]), orc.read(o[1], o[2]))


def test_window_debug_buffer(hd):
    """A device's buffer dump at full extent: the values it holds where it
    holds them, zeros outside its window; a device pointer widens the window
    to the whole array without losing those values."""
    n, P = 64, 4
    say(f"case window debug buffer n={n} P={P}")
    rng = np.random.default_rng(77)
    x0 = rng.random((n, n), dtype=np.float32)
    rt = hd.Runtime()
    X = rt.create(x0)
    p = rt.partition(prog.ROW, (n, n), ndev=P)
    rt.write(X, x0, p)
    rt.sync()
    for d in range(P):
        lo, hi = rt.part_region(p, d)
        r0, r1 = lo[1], hi[1]
        buf = rt.device_buffer(X, d)
        assert np.array_equal(buf[r0:r1], x0[r0:r1])
        assert not buf[:r0].any() and not buf[r1:].any()
    ptr = rt.device_ptr(X, 1)
    assert ptr
    lo, hi = rt.part_region(p, 1)
    buf = rt.device_buffer(X, 1)
    assert np.array_equal(buf[lo[1]:hi[1]], x0[lo[1]:hi[1]])
    assert np.array_equal(rt.read(X, p), x0)
