"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bar: message tables, pack buffers, expanded GDEF maps and integer / FP32
stencil data bit-exact; matmul within K * 2^-24 * (|A||B|)_ij (K = inner
dimension, FP32 accumulation in another order).  Every case runs the same
program (tests/programs.py) on both sides from the same seeded inputs.
"""
import os
import sys

import numpy as np
import pytest

import oracle as O
from tests import canon
from workloads import programs as prog
from workloads import CONV9_WEIGHTS, S3D_COEFFS, jacobi_inputs, stencil3d_inputs, matmul_inputs, ternary_matmul_inputs

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


def same_call(rt, orc, arrays, what, pack=True):
    """messages, pack bytes and GDEF of the given array pairs must match
    (pack=False: the payload holds values computed in another rounding
    order, so only its size is compared)."""
    mg, mo = rt.messages(), orc.messages()
    assert mg.shape == mo.shape, f"{what}: {len(mg)} vs {len(mo)} messages"
    # array ids may differ between the two runtimes only if creation order did
    assert np.array_equal(mg, mo), f"{what}: message tables differ\n{mg[:8]}\n{mo[:8]}"
    pg, po = rt.pack(), orc.pack()
    if pack:
        assert np.array_equal(pg, po), f"{what}: pack buffers differ"
    else:
        assert pg.shape == po.shape, f"{what}: pack sizes differ"
    for ag, ao in arrays:
        og, hg = rt.gdef(ag)
        oo, ho = orc.gdef(ao)
        assert np.array_equal(og, oo), f"{what}: owner map differs"
        assert np.array_equal(hg, ho), f"{what}: holder map differs"


def test_jacobi_small_parity(hd):
    """jacobi_small: 256^2, 4 row partitions, absolute use +-1, 10 steps."""
    say("case jacobi_small 256x256 ndev=4 steps=10")
    A0, B0 = jacobi_inputs(256, 1)
    rt, orc = hd.Runtime(), O.Oracle()
    g = prog.jacobi_rows(rt, A0, B0)
    o = prog.jacobi_rows(orc, A0, B0)
    for it in range(10):
        if it % 2 == 0:
            rt.apply("jacAB", g[2], [g[0], g[1]])
            orc.apply("jacAB", o[2], [o[0], o[1]])
        else:
            rt.apply("jacBA", g[2], [g[1], g[0]])
            orc.apply("jacBA", o[2], [o[1], o[0]])
        same_call(rt, orc, [(g[0], o[0]), (g[1], o[1])], f"step {it}")
    for ag, ao in ((g[0], o[0]), (g[1], o[1])):
        assert np.array_equal(rt.read(ag, g[2]), orc.read(ao, o[2]))
    assert orc.bad_reads() == 0


def test_jacobi_paper_mode_parity(hd):
    """Sec. 5.1 paper mode: A = J(B) then B = A each iteration."""
    say("case jacobi paper mode 64x48 ndev=3")
    A0, B0 = jacobi_inputs(64, 7)
    A0, B0 = A0[:, :48].copy(), B0[:, :48].copy()
    rt, orc = hd.Runtime(), O.Oracle()
    res = []
    for api in (rt, orc):
        A, B, p = prog.jacobi_rows(api, A0, B0, ndev=3)
        api.kernel("cp", prog.K_COPY)
        api.set_offsets("cp", 1, 0, [(0, 0)])
        api.set_offsets("cp", 0, 1, [(0, 0)])
        res.append((A, B, p))
    for it in range(4):
        for (A, B, p), api in zip(res, (rt, orc)):
            api.apply("jacAB", p, [A, B])
        same_call(rt, orc, [(res[0][0], res[1][0]), (res[0][1], res[1][1])], f"jacobi {it}")
        for (A, B, p), api in zip(res, (rt, orc)):
            api.apply("cp", p, [B, A])
        same_call(rt, orc, [(res[0][1], res[1][1])], f"copy {it}")
        assert len(rt.messages()) == 0
    assert np.array_equal(rt.read(res[0][1], res[0][2]), orc.read(res[1][1], res[1][2]))


@pytest.mark.parametrize("n0,n1,ndev,use_box", [(64, 64, 16, False), (96, 80, 16, False), (70, 45, 6, True),
                                                (37, 300, 4, False), (130, 520, 8, True)])
def test_block_parity(hd, n0, n1, ndev, use_box):
    """BLOCK partitions with 5-point offsets (cross) or a full-box use; sizes
    that span several tiles and leave ragged tails."""
    say(f"case block {n0}x{n1} ndev={ndev} box={use_box}")
    rng = np.random.default_rng(n0 * 1000 + n1)
    A0 = rng.random((n0, n1), dtype=np.float32)
    B0 = rng.random((n0, n1), dtype=np.float32)
    rt, orc = hd.Runtime(), O.Oracle()
    g = prog.jacobi_blocks(rt, A0, B0, ndev, use_box)
    o = prog.jacobi_blocks(orc, A0, B0, ndev, use_box)
    for it in range(4):
        k, ag, ao = ("jacAB", [g[0], g[1]], [o[0], o[1]]) if it % 2 == 0 else ("jacBA", [g[1], g[0]], [o[1], o[0]])
        rt.apply(k, g[2], ag)
        orc.apply(k, o[2], ao)
        same_call(rt, orc, [(g[0], o[0]), (g[1], o[1])], f"step {it}")
    assert np.array_equal(rt.read(g[0], g[2]), orc.read(o[0], o[2]))
    assert np.array_equal(rt.read(g[1], g[2]), orc.read(o[1], o[2]))


@pytest.mark.parametrize("shape,ndev,kind", [((1, 300), 4, prog.ROW), ((5, 5), 16, prog.BLOCK),
                                             ((3, 700), 1, prog.BLOCK), ((2, 2), 4, prog.BLOCK),
                                             ((7, 1), 3, prog.ROW), ((6, 9), 8, prog.COL)])
def test_degenerate_parity(hd, shape, ndev, kind):
    """Degenerate partitions: devices with empty boxes (more devices than
    rows), one-cell and one-column boxes, a single device (no messages),
    arrays narrower than one lane's four columns."""
    say(f"case degenerate {shape} ndev={ndev} kind={kind}")
    rng = np.random.default_rng(shape[0] * 31 + shape[1])
    A0 = rng.random(shape, dtype=np.float32)
    B0 = rng.random(shape, dtype=np.float32)
    rt, orc = hd.Runtime(), O.Oracle()
    g = prog.jacobi_blocks(rt, A0, B0, ndev, False, kind)
    o = prog.jacobi_blocks(orc, A0, B0, ndev, False, kind)
    for it in range(3):
        k, ag, ao = ("jacAB", [g[0], g[1]], [o[0], o[1]]) if it % 2 == 0 else ("jacBA", [g[1], g[0]], [o[1], o[0]])
        rt.apply(k, g[2], ag)
        orc.apply(k, o[2], ao)
        same_call(rt, orc, [(g[0], o[0]), (g[1], o[1])], f"step {it}")
    assert np.array_equal(rt.read(g[0], g[2]), orc.read(o[0], o[2]))
    assert np.array_equal(rt.read(g[1], g[2]), orc.read(o[1], o[2]))


@pytest.mark.parametrize("n0,n1,ndev,kind", [(64, 64, 16, prog.BLOCK), (70, 300, 16, prog.BLOCK),
                                             (37, 530, 4, prog.COL), (130, 45, 6, prog.ROW)])
def test_conv2d_parity(hd, n0, n1, ndev, kind):
    """3 x 3 convolution (Sec. 5.1's eight-neighbour kernel): FP32 fused
    multiply-add chain bit-exact against the C library's fmaf; ping-pong steps
    exchange strips and corner cells every step; repeated steps on an input
    that is never redefined communicate once."""
    say(f"case conv2d {n0}x{n1} ndev={ndev} kind={kind}")
    rng = np.random.default_rng(n0 * 7 + n1)
    f0 = rng.random((n0, n1), dtype=np.float32)
    w = [float(x) for x in CONV9_WEIGHTS]
    rt, orc = hd.Runtime(), O.Oracle()
    g = prog.conv2d(rt, f0, ndev, kind)
    o = prog.conv2d(orc, f0, ndev, kind)
    for it in range(4):
        k, gi = ("convAB", (0, 1)) if it % 2 == 0 else ("convBA", (1, 0))
        rt.apply(k, g[2], [g[gi[0]], g[gi[1]]], w)
        orc.apply(k, o[2], [o[gi[0]], o[gi[1]]], w)
        same_call(rt, orc, [(g[0], o[0]), (g[1], o[1])], f"step {it}")
        assert len(rt.messages()) > 0 or ndev == 1
    for it in range(2):
        rt.apply("convAB", g[2], [g[0], g[1]], w)
        orc.apply("convAB", o[2], [o[0], o[1]], w)
        same_call(rt, orc, [(g[0], o[0]), (g[1], o[1])], f"repeat {it}")
        if it:
            assert len(rt.messages()) == 0
    for i in range(2):
        assert np.array_equal(rt.read(g[i], g[2]), orc.read(o[i], o[2]))
    assert orc.bad_reads() == 0


@pytest.mark.parametrize("rows,waves,order", [(4, 1, 1), (8, 1, 1), (16, 1, 1), (4, 1, 0), (8, 1, 0), (16, 1, 0),
                                               (4, 4, 1), (8, 4, 1), (16, 4, 1), (32, 0, 1), (64, 0, 1)])
def test_stencil_shapes_parity(hd, rows, waves, order):
    """Every 2-D stencil tile shape (tiles of 4/8/16 rows with one or four
    waves in either tile order, tall strips of 32/64 rows) gives the
    oracle's bits for Jacobi,
    lower-triangular Jacobi and the 3 x 3 convolution, on sizes with ragged
    tails in both dimensions and strips longer than some boxes."""
    say(f"case stencil shape rows={rows} waves={waves} order={order}")
    rng = np.random.default_rng(rows * 10 + waves + 100 * order)
    w = [float(x) for x in CONV9_WEIGHTS]
    # Jacobi, BLOCK 8 with full-box use
    A0 = rng.random((150, 530), dtype=np.float32)
    B0 = rng.random((150, 530), dtype=np.float32)
    rt, orc = hd.Runtime(), O.Oracle()
    rt.set_stencil_shape(rows, waves, order)
    g = prog.jacobi_blocks(rt, A0, B0, 8, True)
    o = prog.jacobi_blocks(orc, A0, B0, 8, True)
    for it in range(3):
        k, ag, ao = ("jacAB", [g[0], g[1]], [o[0], o[1]]) if it % 2 == 0 else ("jacBA", [g[1], g[0]], [o[1], o[0]])
        rt.apply(k, g[2], ag)
        orc.apply(k, o[2], ao)
        same_call(rt, orc, [(g[0], o[0]), (g[1], o[1])], f"jacobi step {it}")
        st = rt.stats()
        assert st["stencil_rows"] == rows
        assert rows >= 32 or (st["stencil_waves"] == waves and st["stencil_order"] == (1 if waves == 4 else order))
    assert np.array_equal(rt.read(g[0], g[2]), orc.read(o[0], o[2]))
    # triangular on irregular row splits
    T0, U0 = jacobi_inputs(150, 9)
    rt, orc = hd.Runtime(), O.Oracle()
    rt.set_stencil_shape(rows, waves, order)
    g = prog.tri(rt, T0, U0, [0, 1, 40, 41, 97, 150])
    o = prog.tri(orc, T0, U0, [0, 1, 40, 41, 97, 150])
    for it in range(3):
        k, ag, ao = ("triAB", [g[0], g[1]], [o[0], o[1]]) if it % 2 == 0 else ("triBA", [g[1], g[0]], [o[1], o[0]])
        rt.apply(k, g[2], ag)
        orc.apply(k, o[2], ao)
        same_call(rt, orc, [(g[0], o[0]), (g[1], o[1])], f"tri step {it}")
    assert np.array_equal(rt.read(g[0], g[2]), orc.read(o[0], o[2]))
    # convolution, COL 5 with unaligned column blocks
    f0 = rng.random((75, 613), dtype=np.float32)
    rt, orc = hd.Runtime(), O.Oracle()
    rt.set_stencil_shape(rows, waves, order)
    g = prog.conv2d(rt, f0, 5, prog.COL)
    o = prog.conv2d(orc, f0, 5, prog.COL)
    for it in range(3):
        k, gi = ("convAB", (0, 1)) if it % 2 == 0 else ("convBA", (1, 0))
        rt.apply(k, g[2], [g[gi[0]], g[gi[1]]], w)
        orc.apply(k, o[2], [o[gi[0]], o[gi[1]]], w)
        same_call(rt, orc, [(g[0], o[0]), (g[1], o[1])], f"conv step {it}")
    assert np.array_equal(rt.read(g[0], g[2]), orc.read(o[0], o[2]))
    # float4-aligned boxes (row lengths and box starts multiples of 4: the
    # stacked shape's LDS path), heights not a multiple of the tile, widths
    # past one 256-column tile
    # (more than 16 boxes: the boxes are read from the plan, not passed by value)
    for n0, n1, nd, kind in ((150, 520, 8, prog.BLOCK), (77, 1040, 4, prog.COL), (210, 520, 20, prog.ROW)):
        say(f"  aligned boxes {n0}x{n1} ndev={nd}")
        A0 = rng.random((n0, n1), dtype=np.float32)
        B0 = rng.random((n0, n1), dtype=np.float32)
        rt, orc = hd.Runtime(), O.Oracle()
        rt.set_stencil_shape(rows, waves, order)
        g = prog.jacobi_blocks(rt, A0, B0, nd, False, kind)
        o = prog.jacobi_blocks(orc, A0, B0, nd, False, kind)
        for it in range(3):
            k, ag, ao = ("jacAB", [g[0], g[1]], [o[0], o[1]]) if it % 2 == 0 else ("jacBA", [g[1], g[0]], [o[1], o[0]])
            rt.apply(k, g[2], ag)
            orc.apply(k, o[2], ao)
            same_call(rt, orc, [(g[0], o[0]), (g[1], o[1])], f"aligned jacobi step {it}")
            assert rows >= 32 or waves == 1 or rt.stats()["stencil_vec"] == (1 if nd > 16 else 2)
        rt, orc = hd.Runtime(), O.Oracle()
        rt.set_stencil_shape(rows, waves, order)
        g = prog.conv2d(rt, A0, nd, kind)
        o = prog.conv2d(orc, A0, nd, kind)
        for it in range(3):
            k, gi = ("convAB", (0, 1)) if it % 2 == 0 else ("convBA", (1, 0))
            rt.apply(k, g[2], [g[gi[0]], g[gi[1]]], w)
            orc.apply(k, o[2], [o[gi[0]], o[gi[1]]], w)
            same_call(rt, orc, [(g[0], o[0]), (g[1], o[1])], f"aligned conv step {it}")
        assert np.array_equal(rt.read(g[0], g[2]), orc.read(o[0], o[2]))
    T0, U0 = jacobi_inputs(152, 10)
    rt, orc = hd.Runtime(), O.Oracle()
    rt.set_stencil_shape(rows, waves, order)
    g = prog.tri(rt, T0, U0, [0, 4, 40, 44, 100, 152])
    o = prog.tri(orc, T0, U0, [0, 4, 40, 44, 100, 152])
    for it in range(3):
        k, ag, ao = ("triAB", [g[0], g[1]], [o[0], o[1]]) if it % 2 == 0 else ("triBA", [g[1], g[0]], [o[1], o[0]])
        rt.apply(k, g[2], ag)
        orc.apply(k, o[2], ao)
        same_call(rt, orc, [(g[0], o[0]), (g[1], o[1])], f"aligned tri step {it}")
    assert np.array_equal(rt.read(g[0], g[2]), orc.read(o[0], o[2]))


@pytest.mark.parametrize("n,P", [(64, 4), (96, 3), (256, 2)])
def test_gemm_parity(hd, n, P):
    """Listings 2-3 GEMM: the gather of B (first call), then no messages;
    random inputs within the FP32 bound, ternary inputs bit-exact.  64 / 4
    and 96 / 3 take the bounds-checked tile path (boxes of 16 and 32 rows),
    256 / 2 the unchecked one (two 128 x 256 boxes of whole tiles)."""
    say(f"case gemm n={n} P={P}")
    for kind, (a0, b0) in (("random", matmul_inputs(n, 3)), ("ternary", ternary_matmul_inputs(n, 4))):
        rt, orc = hd.Runtime(), O.Oracle()
        g = prog.gemm(rt, a0, b0, P)
        o = prog.gemm(orc, a0, b0, P)
        for it in range(2):
            rt.apply("gemm", g[3], list(g[:3]))
            orc.apply("gemm", o[3], list(o[:3]))
            same_call(rt, orc, [(g[1], o[1]), (g[2], o[2])], f"{kind} call {it}")
        cg = rt.read(g[2], g[3])
        c64 = a0.astype(np.float64) @ b0.astype(np.float64)
        if kind == "ternary":
            assert np.array_equal(cg, c64.astype(np.float32))
        else:
            bound = n * 2.0 ** -24 * (np.abs(a0).astype(np.float64) @ np.abs(b0).astype(np.float64))
            assert np.all(np.abs(cg - c64) <= bound)


@pytest.mark.parametrize("n,cuts", [(32, [0, 10, 21, 32]), (150, [0, 1, 40, 41, 97, 150])])
def test_trapezoid_parity(hd, n, cuts):
    say(f"case trapezoid n={n} cuts={cuts}")
    A0, B0 = jacobi_inputs(n, 9)
    rt, orc = hd.Runtime(), O.Oracle()
    g = prog.tri(rt, A0, B0, cuts)
    o = prog.tri(orc, A0, B0, cuts)
    for it in range(4):
        k, ag, ao = ("triAB", [g[0], g[1]], [o[0], o[1]]) if it % 2 == 0 else ("triBA", [g[1], g[0]], [o[1], o[0]])
        rt.apply(k, g[2], ag)
        orc.apply(k, o[2], ao)
        same_call(rt, orc, [(g[0], o[0]), (g[1], o[1])], f"step {it}")
    assert orc.bad_reads() == 0
    assert np.array_equal(rt.read(g[0], g[2]), orc.read(o[0], o[2]))


def _trapezoid_copy_program(api, A0, B0, traps, boxes):
    """Copy kernels A <- B and B <- A on a manual partition whose work boxes
    lie inside general trapezoids (Table 2 SetTrapezoidUse): each device uses
    its trapezoid of the input (a use larger than what the copy reads) and
    defines its own box of the output."""
    A, B = api.create(A0), api.create(B0)
    p = api.partition_manual([b[0] for b in boxes], [b[1] for b in boxes])
    for k, out, inp in (("cpAB", A, B), ("cpBA", B, A)):
        api.kernel(k, prog.K_COPY)
        api.set_offsets(k, 0, 1, [(0, 0)])
        for d, c in enumerate(traps):
            api.set_trapezoid(k, p, inp, d, 0, c)
    api.write(A, A0, p)
    return A, B, p


def test_general_trapezoid_parity(hd):
    """Trapezoids with non-unit and negative edge slopes, clipped on both
    sides, a one-row trapezoid and crossed edges (the hand-derived fixture
    cases) as use sections of copy kernels: messages, pack buffers, GDEF and
    values bit-exact over four alternating calls."""
    import json
    say("case general trapezoids 16x20 ndev=5")
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "trapezoid_rows.json")))
    traps = [c["corners"] for c in gold["cases"]]
    # a work box inside each trapezoid, pairwise disjoint
    boxes = [((2, 3), (8, 6)), ((0, 6), (2, 9)), ((10, 7), (14, 15)), ((15, 4), (16, 10)), ((8, 0), (9, 2))]
    rng = np.random.default_rng(1616)
    A0 = rng.random((16, 20), dtype=np.float32)
    B0 = rng.random((16, 20), dtype=np.float32)
    rt, orc = hd.Runtime(), O.Oracle()
    g = _trapezoid_copy_program(rt, A0, B0, traps, boxes)
    o = _trapezoid_copy_program(orc, A0, B0, traps, boxes)
    for it in range(4):
        k, gi = ("cpAB", (0, 1)) if it % 2 == 0 else ("cpBA", (1, 0))
        rt.apply(k, g[2], [g[gi[0]], g[gi[1]]])
        orc.apply(k, o[2], [o[gi[0]], o[gi[1]]])
        same_call(rt, orc, [(g[0], o[0]), (g[1], o[1])], f"step {it}")
        assert len(rt.messages()) > 0
    for i in range(2):
        assert np.array_equal(rt.read(g[i], g[2]), orc.read(o[i], o[2]))
    assert orc.bad_reads() == 0


@pytest.mark.parametrize("shape,ndev", [((12, 12, 12), 8), ((20, 17, 300), 8), ((9, 33, 65), 12)])
def test_stencil3d_parity(hd, shape, ndev):
    """7-point stencil on 3-D blocks: boxes stacked over rows and planes,
    FP32 fused multiply-adds bit-exact against the C library's fmaf."""
    say(f"case stencil3d {shape} ndev={ndev}")
    rng = np.random.default_rng(sum(shape))
    u0 = rng.random(shape, dtype=np.float32)
    coef = [float(c) for c in S3D_COEFFS]
    rt, orc = hd.Runtime(), O.Oracle()
    g = prog.stencil3d(rt, u0, ndev)
    o = prog.stencil3d(orc, u0, ndev)
    for it in range(3):
        k, ag, ao = ("s3dUV", [g[0], g[1]], [o[0], o[1]]) if it % 2 == 0 else ("s3dVU", [g[1], g[0]], [o[1], o[0]])
        rt.apply(k, g[2], ag, coef)
        orc.apply(k, o[2], ao, coef)
        same_call(rt, orc, [(g[0], o[0]), (g[1], o[1])], f"step {it}")
    assert np.array_equal(rt.read(g[0], g[2]), orc.read(o[0], o[2]))


@pytest.mark.parametrize("seed", range(8))
def test_random_programs_parity(hd, seed):
    """Random Write / copy-kernel sequences with random absolute use boxes and
    partitions (2-D and 3-D), including ragged and empty regions."""
    say(f"case random program seed={seed}")
    rng = np.random.default_rng(500 + seed)
    dim = 2 if seed % 3 else 3
    shape = tuple(int(x) for x in rng.integers(5, 40 if dim == 2 else 9, size=dim))
    x0 = rng.random(shape, dtype=np.float32)
    y0 = rng.random(shape, dtype=np.float32)
    ndev = int(rng.integers(2, 9))
    kind = int(rng.integers(0, 3))
    steps = []
    for step in range(6):
        dec = []
        for d in range(ndev):
            boxes = []
            for _ in range(int(rng.integers(0, 3))):
                blo = [int(rng.integers(0, s)) for s in shape]
                bhi = [int(rng.integers(b + 1, s + 1)) for b, s in zip(blo, shape)]
                boxes.append((blo, bhi))
            dec.append(boxes)
        steps.append(dec)
    rt, orc = hd.Runtime(), O.Oracle()
    res = []
    for api in (rt, orc):
        X, Y = api.create(x0), api.create(y0)
        p = api.partition(kind, shape, ndev=ndev)
        api.write(X, x0, p)
        for step, dec in enumerate(steps):
            out, inp = (X, Y) if step % 2 else (Y, X)
            kname = f"k{step}"
            api.kernel(kname, prog.K_COPY)
            for d in range(ndev):
                lo, hi = api.part_region(p, d)
                if any(a >= b for a, b in zip(lo, hi)):
                    continue
                dlo, dhi = lo[3 - dim:], hi[3 - dim:]
                api.set_absolute(kname, p, out, d, 1, dlo, dhi)
                api.set_absolute(kname, p, inp, d, 0, dlo, dhi)
                for blo, bhi in dec[d]:
                    api.set_absolute(kname, p, inp, d, 0, blo, bhi)
        res.append((X, Y, p))
    for step in range(6):
        for (X, Y, p), api in zip(res, (rt, orc)):
            out, inp = (X, Y) if step % 2 else (Y, X)
            api.apply(f"k{step}", p, [out, inp])
        same_call(rt, orc, [(res[0][0], res[1][0]), (res[0][1], res[1][1])], f"step {step}")
    for i in range(2):
        assert np.array_equal(rt.read(res[0][i], res[0][2]), orc.read(res[1][i], res[1][2]))
        same_call(rt, orc, [(res[0][i], res[1][i])], f"read {i}")


@pytest.mark.parametrize("case", ["rows2d", "rows3d", "rows3d_large"])
def test_many_rows_parity(hd, case):
    """Levels with more than 32768 use rows, where the runs are found one
    row per lane (with the wave taking the rows that do not fit): a tall
    2-D array with column partitions, and 3-D arrays of many rows (the
    larger one past 2^18 slices, where the band scan takes 1024 threads)."""
    rng = np.random.default_rng(91)
    rt, orc = hd.Runtime(), O.Oracle()
    if case == "rows2d":
        say("case many rows 40000x24 COL ndev=3")
        A0 = rng.random((40000, 24), dtype=np.float32)
        B0 = rng.random((40000, 24), dtype=np.float32)
        g = prog.jacobi_blocks(rt, A0, B0, 3, kind=prog.COL)
        o = prog.jacobi_blocks(orc, A0, B0, 3, kind=prog.COL)
        names = ("jacAB", "jacBA")
        coef = None
    else:
        shape = (40, 1000, 12) if case == "rows3d" else (300, 1000, 8)
        say(f"case many rows 3-D {shape} ndev=8")
        u0 = rng.random(shape, dtype=np.float32)
        g = prog.stencil3d(rt, u0, 8)
        o = prog.stencil3d(orc, u0, 8)
        names = ("s3dUV", "s3dVU")
        coef = [float(c) for c in S3D_COEFFS]
    for it in range(3):
        k, gi = (names[0], (0, 1)) if it % 2 == 0 else (names[1], (1, 0))
        args = [] if coef is None else [coef]
        rt.apply(k, g[2], [g[gi[0]], g[gi[1]]], *args)
        orc.apply(k, o[2], [o[gi[0]], o[gi[1]]], *args)
        same_call(rt, orc, [(g[0], o[0]), (g[1], o[1])], f"step {it}")
    assert np.array_equal(rt.read(g[0], g[2]), orc.read(o[0], o[2]))


def test_runs_wave_form_parity(hd):
    """The one-wave-per-use-row form of the runs kernel (selected for small
    levels through HD_RUNS_WAVE_MAX) gives the same messages and GDEF."""
    say("case runs wave form (HD_RUNS_WAVE_MAX) block 130x520 ndev=8 and 3-D 12^3")
    os.environ["HD_RUNS_WAVE_MAX"] = "1000000"
    try:
        rng = np.random.default_rng(17)
        A0 = rng.random((130, 520), dtype=np.float32)
        B0 = rng.random((130, 520), dtype=np.float32)
        rt, orc = hd.Runtime(), O.Oracle()
        g = prog.jacobi_blocks(rt, A0, B0, 8, True)
        o = prog.jacobi_blocks(orc, A0, B0, 8, True)
        for it in range(3):
            k, gi = ("jacAB", (0, 1)) if it % 2 == 0 else ("jacBA", (1, 0))
            rt.apply(k, g[2], [g[gi[0]], g[gi[1]]])
            orc.apply(k, o[2], [o[gi[0]], o[gi[1]]])
            same_call(rt, orc, [(g[0], o[0]), (g[1], o[1])], f"2-D step {it}")
        u0 = rng.random((12, 12, 12), dtype=np.float32)
        coef = [float(c) for c in S3D_COEFFS]
        rt, orc = hd.Runtime(), O.Oracle()
        g = prog.stencil3d(rt, u0, 8)
        o = prog.stencil3d(orc, u0, 8)
        for it in range(3):
            k, gi = ("s3dUV", (0, 1)) if it % 2 == 0 else ("s3dVU", (1, 0))
            rt.apply(k, g[2], [g[gi[0]], g[gi[1]]], coef)
            orc.apply(k, o[2], [o[gi[0]], o[gi[1]]], coef)
            same_call(rt, orc, [(g[0], o[0]), (g[1], o[1])], f"3-D step {it}")
    finally:
        del os.environ["HD_RUNS_WAVE_MAX"]
        hd.Runtime()  # back to the default form for later tests


def test_wide_rows_parity(hd):
    """60 column partitions of a 6 x 900 array: every row has about 118 runs
    (more than a row's run slot, so the spill pool is used) and about 180
    GDEF intervals (more boundaries than the register-only update handles,
    so the LDS path runs), and the definitions tile whole rows."""
    say("case wide rows 6x900 COL ndev=60 row_cap=256 steps=4")
    rng = np.random.default_rng(77)
    A0 = rng.random((6, 900), dtype=np.float32)
    B0 = rng.random((6, 900), dtype=np.float32)
    rt, orc = hd.Runtime(row_cap=256), O.Oracle()
    g = prog.jacobi_blocks(rt, A0, B0, ndev=60, kind=prog.COL)
    o = prog.jacobi_blocks(orc, A0, B0, ndev=60, kind=prog.COL)
    for it in range(4):
        k, gi, oi = ("jacAB", (0, 1), (0, 1)) if it % 2 == 0 else ("jacBA", (1, 0), (1, 0))
        rt.apply(k, g[2], [g[gi[0]], g[gi[1]]])
        orc.apply(k, o[2], [o[oi[0]], o[oi[1]]])
        same_call(rt, orc, [(g[0], o[0]), (g[1], o[1])], f"step {it}")
        assert len(rt.messages()) == 118
    for i in range(2):
        assert np.array_equal(rt.read(g[i], g[2]), orc.read(o[i], o[2]))


def test_read_write_reduce_parity(hd):
    say("case read/write/reduce")
    n = 40
    A0, B0 = jacobi_inputs(n, 4)
    rt, orc = hd.Runtime(), O.Oracle()
    g = prog.jacobi_rows(rt, A0, B0, ndev=3)
    o = prog.jacobi_rows(orc, A0, B0, ndev=3)
    assert np.array_equal(rt.read(g[1], g[2]), B0)
    rt.apply("jacAB", g[2], [g[0], g[1]])
    orc.apply("jacAB", o[2], [o[0], o[1]])
    a = rt.read(g[0], g[2])
    assert np.array_equal(a, orc.read(o[0], o[2]))
    same_call(rt, orc, [(g[0], o[0])], "read")
    s_g = rt.reduce(g[0], prog.ROW * 0 + 0, g[2])
    s_o = orc.reduce(o[0], 0, o[2])
    assert abs(s_g - s_o) <= 2 * n * n * 2.0 ** -24 * float(np.sum(np.abs(a)))
    for op in (2, 3):
        assert rt.reduce(g[0], op, g[2]) == np.float32(orc.reduce(o[0], op, o[2]))
    iv = (np.arange(n * n, dtype=np.int64).reshape(n, n) * 7919 - 3 * n * n).astype(np.int32)
    Ig, Io = rt.create(shape=(n, n), type_=1), orc.create(shape=(n, n), type_=1)
    rt.write(Ig, iv, g[2])
    orc.write(Io, iv, o[2])
    for op in range(4):
        assert rt.reduce(Ig, op, g[2]) == orc.reduce(Io, op, o[2])
    D0 = np.random.default_rng(1).random((n, n))
    Dg, Do = rt.create(shape=(n, n), type_=2), orc.create(shape=(n, n), type_=2)
    rt.write(Dg, D0, g[2])
    orc.write(Do, D0, o[2])
    assert np.array_equal(rt.read(Dg, g[2]), D0)
    for op in (2, 3):
        assert rt.reduce(Dg, op, g[2]) == orc.reduce(Do, op, o[2])


def test_error_paths_gpu(hd):
    rt = hd.Runtime()
    n = 16
    A, B = rt.create(shape=(n, n)), rt.create(shape=(n, n))
    p = rt.partition(prog.ROW, (n, n), ndev=2)
    rt.kernel("jac", prog.K_JACOBI2D)
    rt.set_absolute("jac", p, A, 0, 1, (0, 0), (9, n))
    rt.set_absolute("jac", p, A, 1, 1, (8, 0), (n, n))
    with pytest.raises(hd.HDArrayError) as e:
        rt.apply("jac", p, [A, B])
    assert e.value.code == hd.ERACE
    with pytest.raises(hd.HDArrayError) as e:
        rt.set_absolute("jac", p, A, 0, 0, (0, 0), (n + 1, n))
    assert e.value.code == hd.EBOUNDS
    with pytest.raises(hd.HDArrayError) as e:
        rt.set_trapezoid("jac", p, A, 0, 0, [0, 0, 1, 3, 5, 0, 5, 5])
    assert e.value.code == hd.EINVAL
    with pytest.raises(hd.HDArrayError):
        rt.apply("jac", p, [A, A])
    with pytest.raises(hd.HDArrayError) as e:
        rt.kernel("bad", "nosuchkernel")
    assert e.value.code == hd.EKERNEL
    q = rt.partition_manual([(0, 0), (4, 0)], [(8, n), (n, n)])
    with pytest.raises(hd.HDArrayError) as e:
        rt.write(A, np.zeros((n, n), np.float32), q)
    assert e.value.code == hd.EINVAL
