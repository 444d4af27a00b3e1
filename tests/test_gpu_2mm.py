"""2MM (Sec. 5.1): two dependent matrix products, D = A x B then E = C x D,
with ROW and with COL partitions of one GPU's share.  Message tables, pack
buffers and GDEF equal the oracle's at every call; the communication
volumes follow Table 3's pattern (ROW: B gathered once, D every iteration;
COL: A and C gathered once, nothing afterwards); values are bit-exact for
ternary inputs and within the FP32 accumulation bound for random ones."""
import sys

import numpy as np
import pytest

import oracle as O
from workloads import programs as prog
from tests.test_gpu_parity import same_call
from workloads import matmul_inputs, ternary_matmul_inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hd():
    import paper_1809_05657_amd as hdm
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    hdm.load()
    return hdm


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def bound(x, y, n):
    return n * 2.0 ** -24 * (np.abs(x).astype(np.float64) @ np.abs(y).astype(np.float64))


@pytest.mark.parametrize("layout", ["row", "col"])
@pytest.mark.parametrize("kind", ["ternary", "random"])
def test_2mm(hd, layout, kind):
    n, P = 160, 8
    say(f"case 2mm {layout} {kind} n={n} P={P}")
    lay = prog.ROW if layout == "row" else prog.COL
    if kind == "ternary":
        a0, b0 = ternary_matmul_inputs(n, 11)
        c0, _ = ternary_matmul_inputs(n, 12)
    else:
        a0, b0 = matmul_inputs(n, 13)
        c0, _ = matmul_inputs(n, 14)
    rt, orc = hd.Runtime(), O.Oracle()
    g = prog.mm2(rt, a0, b0, c0, P, lay)
    o = prog.mm2(orc, a0, b0, c0, P, lay)
    full = n * n * 4
    vols = []
    for it in range(3):
        v = []
        for k, idx in (("mm1", (0, 1, 3)), ("mm2", (2, 3, 4))):
            rt.apply(k, g[5], [g[i] for i in idx])
            orc.apply(k, o[5], [o[i] for i in idx])
            # random inputs: D is the matrix cores' FP32 sum, not the oracle's,
            # so the gathered D payload is compared through the value bound
            same_call(rt, orc, [(g[i], o[i]) for i in range(5)], f"iter {it} {k}",
                      pack=kind == "ternary" or k == "mm1")
            v.append(int(rt.messages()[:, 11].sum()) if len(rt.messages()) else 0)
        vols.append(v)
    # off-device bytes of a gather: every device receives the other P-1 parts
    gather = full * (P - 1)
    if layout == "row":
        assert vols == [[gather, gather], [0, gather], [0, gather]], vols
    else:
        assert vols == [[gather, gather], [0, 0], [0, 0]], vols
    d = rt.read(g[3], g[5])
    e = rt.read(g[4], g[5])
    if kind == "ternary":
        d64 = a0.astype(np.float64) @ b0.astype(np.float64)
        e64 = c0.astype(np.float64) @ d64
        assert np.array_equal(d, d64.astype(np.float32))
        assert np.array_equal(e, e64.astype(np.float32))
    else:
        d64 = a0.astype(np.float64) @ b0.astype(np.float64)
        assert np.all(np.abs(d - d64) <= bound(a0, b0, n))
        # E against the exact product of C and the computed D
        e64 = c0.astype(np.float64) @ d.astype(np.float64)
        assert np.all(np.abs(e - e64) <= bound(c0, d, n))
