"""Plan cache (Sec. 4.2) on the HIP path: with the cache on, every call's
message table, pack buffer, GDEF and data must equal the oracle's (which
always derives), bit-exact, and calls whose arrays' GDEF repeats must reuse
the table (counted as hits)."""
import sys

import numpy as np
import pytest

import oracle as O
from workloads import programs as prog
from tests.test_gpu_parity import same_call
from workloads import CONV9_WEIGHTS, S3D_COEFFS

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


def pingpong(rt, orc, g, o, steps, what, coef=None, names=("jacAB", "jacBA")):
    for it in range(steps):
        k, gi = (names[0], (0, 1)) if it % 2 == 0 else (names[1], (1, 0))
        args = [] if coef is None else [coef]
        rt.apply(k, g[2], [g[gi[0]], g[gi[1]]], *args)
        orc.apply(k, o[2], [o[gi[0]], o[gi[1]]], *args)
        same_call(rt, orc, [(g[0], o[0]), (g[1], o[1])], f"{what} step {it}")


@pytest.mark.parametrize("n0,n1,ndev,use_box", [(130, 520, 8, True), (96, 80, 16, False)])
def test_cache_jacobi(hd, n0, n1, ndev, use_box):
    """Ping-pong Jacobi: the key of a call repeats from the fifth call on
    (the writes that start both histories are behind it), so every later
    call hits; a Write in between restarts the histories."""
    say(f"case cache jacobi {n0}x{n1} ndev={ndev} box={use_box}")
    rng = np.random.default_rng(n0 + n1)
    A0 = rng.random((n0, n1), dtype=np.float32)
    B0 = rng.random((n0, n1), dtype=np.float32)
    rt, orc = hd.Runtime(), O.Oracle()
    rt.set_plan_cache(True)
    g = prog.jacobi_blocks(rt, A0, B0, ndev, use_box)
    o = prog.jacobi_blocks(orc, A0, B0, ndev, use_box)
    pingpong(rt, orc, g, o, 8, "first")
    st = rt.stats()
    assert st["cache_misses"] == 4 and st["cache_hits"] == 4, st
    # a Write of B (whole array, no use) starts B's history afresh
    rt.write(g[1], B0, g[2])
    orc.write(o[1], B0, o[2])
    pingpong(rt, orc, g, o, 6, "after write")
    st = rt.stats()
    assert st["cache_hits"] + st["cache_misses"] == 14 and st["cache_hits"] >= 6, st
    for i in range(2):
        assert np.array_equal(rt.read(g[i], g[2]), orc.read(o[i], o[2]))


def test_cache_toggle(hd):
    """Calls made with the cache off still advance the histories: turning it
    on mid-run gives the same messages as deriving every call."""
    say("case cache toggle 64x64 ndev=16")
    rng = np.random.default_rng(5)
    A0 = rng.random((64, 64), dtype=np.float32)
    B0 = rng.random((64, 64), dtype=np.float32)
    rt, orc = hd.Runtime(), O.Oracle()
    g = prog.jacobi_blocks(rt, A0, B0, 16, False)
    o = prog.jacobi_blocks(orc, A0, B0, 16, False)
    pingpong(rt, orc, g, o, 4, "off")
    rt.set_plan_cache(True)
    pingpong(rt, orc, g, o, 6, "on")
    rt.set_plan_cache(False)
    pingpong(rt, orc, g, o, 2, "off again")
    rt.set_plan_cache(True)
    pingpong(rt, orc, g, o, 4, "on again")
    assert rt.stats()["cache_hits"] > 0
    assert np.array_equal(rt.read(g[0], g[2]), orc.read(o[0], o[2]))


@pytest.mark.parametrize("shape,ndev", [((12, 12, 12), 8), ((9, 33, 65), 12)])
def test_cache_stencil3d(hd, shape, ndev):
    """3-D arrays (the two-level derivation) with the cache on."""
    say(f"case cache stencil3d {shape} ndev={ndev}")
    rng = np.random.default_rng(sum(shape) + 1)
    u0 = rng.random(shape, dtype=np.float32)
    coef = [float(c) for c in S3D_COEFFS]
    rt, orc = hd.Runtime(), O.Oracle()
    rt.set_plan_cache(True)
    g = prog.stencil3d(rt, u0, ndev)
    o = prog.stencil3d(orc, u0, ndev)
    pingpong(rt, orc, g, o, 7, "s3d", coef, ("s3dUV", "s3dVU"))
    assert rt.stats()["cache_hits"] >= 2
    assert np.array_equal(rt.read(g[0], g[2]), orc.read(o[0], o[2]))


@pytest.mark.parametrize("seed", range(4))
def test_cache_random_programs(hd, seed):
    """Random copy kernels with random extra use boxes, run as a sequence
    twice over with a Read and a Write between; partial definitions keep the
    histories growing, so hits and misses both occur."""
    say(f"case cache random program seed={seed}")
    rng = np.random.default_rng(900 + seed)
    dim = 2 if seed % 2 else 3
    shape = tuple(int(x) for x in rng.integers(5, 40 if dim == 2 else 9, size=dim))
    x0 = rng.random(shape, dtype=np.float32)
    y0 = rng.random(shape, dtype=np.float32)
    ndev = int(rng.integers(2, 9))
    kind = int(rng.integers(0, 3))
    nk = 3
    decs = []
    for _ in range(nk):
        dec = []
        for d in range(ndev):
            boxes = []
            for _ in range(int(rng.integers(0, 3))):
                blo = [int(rng.integers(0, s)) for s in shape]
                bhi = [int(rng.integers(b + 1, s + 1)) for b, s in zip(blo, shape)]
                boxes.append((blo, bhi))
            dec.append(boxes)
        decs.append(dec)
    # some kernels work on the interior only (a second partition that leaves
    # out the outer cells, as in Sec. 5.1's ghost-cell layout): their
    # definitions do not cover the array, so its history grows
    partial = [bool(rng.integers(0, 2)) for _ in range(nk)]
    rt, orc = hd.Runtime(), O.Oracle()
    rt.set_plan_cache(True)
    res = []
    for api in (rt, orc):
        X, Y = api.create(x0), api.create(y0)
        p = api.partition(kind, shape, ndev=ndev)
        pin = api.partition(kind, shape, tuple([1] * dim), tuple(s - 1 for s in shape), ndev=ndev)
        api.write(X, x0, p)
        api.write(Y, y0, p)
        pk = []
        for q in range(nk):
            out, inp = (X, Y) if q % 2 else (Y, X)
            kname = f"k{q}"
            pq = pin if partial[q] else p
            pk.append(pq)
            api.kernel(kname, prog.K_COPY)
            for d in range(ndev):
                lo, hi = api.part_region(pq, d)
                if any(a >= b for a, b in zip(lo, hi)):
                    continue
                dlo, dhi = lo[3 - dim:], hi[3 - dim:]
                api.set_absolute(kname, pq, out, d, 1, dlo, dhi)
                api.set_absolute(kname, pq, inp, d, 0, dlo, dhi)
                for blo, bhi in decs[q][d]:
                    api.set_absolute(kname, pq, inp, d, 0, blo, bhi)
        res.append((X, Y, p, pk))
    seq = [int(rng.integers(0, nk)) for _ in range(5)]
    step = 0
    for rep in range(3):
        for q in seq + seq:
            for (X, Y, p, pk), api in zip(res, (rt, orc)):
                out, inp = (X, Y) if q % 2 else (Y, X)
                api.apply(f"k{q}", pk[q], [out, inp])
            same_call(rt, orc, [(res[0][0], res[1][0]), (res[0][1], res[1][1])], f"rep {rep} step {step} k{q}")
            step += 1
        if rep == 0:
            assert np.array_equal(rt.read(res[0][0], res[0][2]), orc.read(res[1][0], res[1][2]))
        if rep == 1:
            for (X, Y, p, pk), api in zip(res, (rt, orc)):
                api.write(Y, y0, p)
    st = rt.stats()
    assert st["cache_hits"] + st["cache_misses"] == step, st
    for i in range(2):
        assert np.array_equal(rt.read(res[0][i], res[0][2]), orc.read(res[1][i], res[1][2]))


@pytest.mark.parametrize("n0,n1,ndev,kind", [(70, 300, 16, prog.BLOCK), (130, 45, 6, prog.ROW)])
def test_cache_gdef_compare(hd, n0, n1, ndev, kind):
    """Second step (Sec. 4.2): the convolution's input is never redefined,
    so its history grows with every call (a new key each call, dropped past
    8 entries) and the host cannot decide; the GPU compares the input's
    lists with those the plan's last derivation read, finds them unchanged
    from the third call on (every halo is held after the first) and reuses
    the table.  Every call checked against the oracle, which derives."""
    say(f"case cache gdef compare {n0}x{n1} ndev={ndev} kind={kind}")
    rng = np.random.default_rng(n0 * 11 + n1)
    f0 = rng.random((n0, n1), dtype=np.float32)
    w = [float(x) for x in CONV9_WEIGHTS]
    rt, orc = hd.Runtime(), O.Oracle()
    rt.set_plan_cache(True)
    g = prog.conv2d(rt, f0, ndev, kind)
    o = prog.conv2d(orc, f0, ndev, kind)
    calls = 12
    for it in range(calls):
        rt.apply("convAB", g[2], [g[0], g[1]], w)
        orc.apply("convAB", o[2], [o[0], o[1]], w)
        same_call(rt, orc, [(g[0], o[0]), (g[1], o[1])], f"call {it}")
    st = rt.stats()
    assert st["cache_hits"] == 0, st
    assert st["cache_gdef_hits"] == calls - 2, st
    # a redefinition of the input makes the lists differ again: derived
    rt.apply("convBA", g[2], [g[1], g[0]], w)
    orc.apply("convBA", o[2], [o[1], o[0]], w)
    same_call(rt, orc, [(g[0], o[0]), (g[1], o[1])], "redefine")
    rt.apply("convAB", g[2], [g[0], g[1]], w)
    orc.apply("convAB", o[2], [o[0], o[1]], w)
    same_call(rt, orc, [(g[0], o[0]), (g[1], o[1])], "after redefine")
    assert rt.stats()["cache_gdef_hits"] == calls - 2
    for i in range(2):
        assert np.array_equal(rt.read(g[i], g[2]), orc.read(o[i], o[2]))
