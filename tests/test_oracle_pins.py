"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every test here runs on the CPU (no ``gpu`` marker).  Sources of truth:
hand-derived message lists from the paper's equations (golden fixtures),
Table 3's printed volumes, closed forms of the kernels, invariants of the
GDEF map, library routines (numpy) for special cases, and a fault-injection
test of the oracle's own coherence check.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
from tests import canon
from workloads import CONV9_WEIGHTS, S3D_COEFFS, jacobi_inputs

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def msgs_list(o):
    return [list(map(int, m)) for m in o.messages()]


# ---------------------------------------------------------------- programs
def jacobi_row_program(o, n=256, ndev=4, A0=None, B0=None):
    """256^2 Jacobi, absolute use = own rows +-1, def = own rows (Table 2)."""
    if A0 is None:
        A0, B0 = jacobi_inputs(n, 1)
    A, B = o.create(A0), o.create(B0)
    p = o.partition(O.ROW, (n, n), ndev=ndev)
    for k in ("jacAB", "jacBA"):
        o.kernel(k, O.K_JACOBI2D)
    for d in range(ndev):
        (_, r0, _), (_, r1, _) = o.part_region(p, d)
        for k, out, inp in (("jacAB", A, B), ("jacBA", B, A)):
            o.set_absolute(k, p, inp, d, 0, (max(r0 - 1, 0), 0), (min(r1 + 1, n), n))
            o.set_absolute(k, p, out, d, 1, (r0, 0), (r1, n))
    o.write(A, A0, p)
    o.write(B, B0, p)
    return A, B, p


def test_h1_jacobi_row_halo_messages():
    """Eq. 1-2 on the 256^2 / 4-row-block Jacobi: exactly the 6 halo rows."""
    gold = json.load(open(os.path.join(GOLD, "h1_jacobi_row4_messages.json")))
    o = O.Oracle()
    A, B, p = jacobi_row_program(o)
    for it in range(4):
        o.apply("jacAB" if it % 2 == 0 else "jacBA", p, [A, B] if it % 2 == 0 else [B, A])
        got = [[m[2], m[3], m[5], m[8], m[6], m[9]] for m in msgs_list(o)]
        assert got == gold["messages"], f"iteration {it}"
    assert o.bad_reads() == 0


def test_h1_paper_mode_copy_step_has_no_messages():
    """Sec. 5.1 Jacobi: the copy kernel B = A uses zero offsets, so it needs
    nothing from other devices."""
    o = O.Oracle()
    A, B, p = jacobi_row_program(o)
    o.kernel("copyBA", O.K_COPY)
    o.set_offsets("copyBA", 1, 0, [(0, 0)])
    o.set_offsets("copyBA", 0, 1, [(0, 0)])
    for it in range(3):
        o.apply("jacAB", p, [A, B])
        assert len(o.messages()) == 6
        o.apply("copyBA", p, [B, A])
        assert len(o.messages()) == 0
    assert o.bad_reads() == 0


@pytest.mark.parametrize("P,n", [(2, 64), (4, 64), (2, 1024)])
def test_h2_gemm_case_study_all_gather_once(P, n):
    """Sec. 3.2 Listings 2-3 and Sec. 5.1: use(A,(0,*)) use(B,(*,0)) def(C,(0,0))
    with a ROW partition: B is gathered once (every device gets every other
    device's rows), A and C need nothing; later calls communicate nothing."""
    o = O.Oracle(simulate_devices=(n <= 64), eval_kernels=(n <= 64))
    rng = np.random.default_rng(7)
    a0, b0 = [rng.random((n, n), dtype=np.float32) for _ in range(2)]
    A, B, Cc = o.create(a0), o.create(b0), o.create(shape=(n, n))
    p = o.partition(O.ROW, (n, n), ndev=P)
    o.kernel("gemm", O.K_MATMUL)
    o.set_offsets("gemm", 0, 0, [(0, "*")])
    o.set_offsets("gemm", 1, 0, [("*", 0)])
    o.set_offsets("gemm", 2, 1, [(0, 0)])
    for arr, v in ((A, a0), (B, b0), (Cc, np.zeros((n, n), np.float32))):
        o.write(arr, v, p)
    o.apply("gemm", p, [A, B, Cc])
    ms = msgs_list(o)
    rows = n // P
    expect = []
    for q in range(P):
        for d in range(P):
            if d != q:
                expect.append([1, B.id, q, d, 0, rows * q, 0, 1, rows * q + rows, n])
    assert [m[:10] for m in ms] == expect
    assert sum(m[11] for m in ms) == (P - 1) * n * n * 4
    o.apply("gemm", p, [A, B, Cc])
    assert len(o.messages()) == 0
    if n <= 64:
        c = o.read(Cc, p)
        ref = a0.astype(np.float64) @ b0.astype(np.float64)
        assert np.max(np.abs(c - ref)) <= n * 2.0 ** -24 * np.max(np.abs(a0) @ np.abs(b0))


def block_cross_program(o, n, use_box=False, ndev=16):
    A0, B0 = jacobi_inputs(n, 2)
    A, B = o.create(A0), o.create(B0)
    p = o.partition(O.BLOCK, (n, n), ndev=ndev)
    o.kernel("jac", O.K_JACOBI2D)
    if use_box:
        for d in range(ndev):
            (_, r0, c0), (_, r1, c1) = o.part_region(p, d)
            o.set_absolute("jac", p, B, d, 0, (max(r0 - 1, 0), max(c0 - 1, 0)), (min(r1 + 1, n), min(c1 + 1, n)))
            o.set_absolute("jac", p, A, d, 1, (r0, c0), (r1, c1))
    else:
        o.set_offsets("jac", 1, 0, [(0, 0), (0, -1), (0, 1), (-1, 0), (1, 0)])
        o.set_offsets("jac", 0, 1, [(0, 0)])
    o.write(A, A0, p)
    o.write(B, B0, p)
    return A, B, p


@pytest.mark.parametrize("use_box", [False, True])
def test_h3_block_grid_halo_messages(use_box):
    """4x4 BLOCK partition, 5-point offsets (Sec. 5.1 Jacobi clauses): 24 row
    strips + 24 column strips; a full-box absolute use adds 36 corners."""
    n = 64
    o = O.Oracle()
    A, B, p = block_cross_program(o, n, use_box)
    o.apply("jac", p, [A, B])
    ms = msgs_list(o)
    strips = [m for m in ms if (m[8] - m[5]) * (m[9] - m[6]) == 16]
    corners = [m for m in ms if (m[8] - m[5]) * (m[9] - m[6]) == 1]
    assert len(strips) == 48
    assert len(corners) == (36 if use_box else 0)
    assert len(ms) == len(strips) + len(corners)
    assert o.bad_reads() == 0


def test_h4_overwrite_kill():
    """Reading of Eq. 3-4 with two writers: the last definer is the only
    source.  d0 defines row 3, then d2 defines it without using it, then d1
    uses it: exactly one message, 2 -> 1."""
    o = O.Oracle()
    n = 8
    X = o.create(np.arange(n * n, dtype=np.float32).reshape(n, n))
    Y = o.create(np.ones((n, n), np.float32))
    pall = o.partition(O.ROW, (n, n), ndev=3)
    o.write(X, np.zeros((n, n), np.float32), pall)
    o.write(Y, np.ones((n, n), np.float32), pall)
    parts = {}
    for d in range(3):
        lo = [(3, 0) if e == d else (0, 0) for e in range(3)]
        hi = [(4, n) if e == d else (0, 0) for e in range(3)]
        parts[d] = o.partition_manual(lo, hi)
    o.kernel("cp", O.K_COPY)
    o.set_offsets("cp", 1, 0, [(0, 0)])
    o.set_offsets("cp", 0, 1, [(0, 0)])
    o.apply("cp", parts[0], [X, Y])
    o.apply("cp", parts[2], [X, Y])
    o.apply("cp", parts[1], [Y, X])
    ms = msgs_list(o)
    assert [(m[2], m[3], m[5], m[8]) for m in ms] == [(2, 1, 3, 4)]
    assert o.bad_reads() == 0


def test_h5_trapezoid_messages():
    """Table 2 SetTrapezoidDef/Use: lower-triangular rows [a,b) per device; a
    use one row above / below gives 1-row messages of length a and b+1."""
    n = 32
    cuts = [0, 10, 21, 32]
    o = O.Oracle()
    A0, B0 = jacobi_inputs(n, 9)
    A, B = o.create(A0), o.create(B0)
    p = o.partition_manual([(cuts[d], 0) for d in range(3)], [(cuts[d + 1], n) for d in range(3)])
    o.kernel("tri", O.K_TRI2D)
    for d in range(3):
        a, b = cuts[d], cuts[d + 1]
        o.set_trapezoid("tri", p, B, d, 0, [a - 1, 0, a - 1, a - 1, b, 0, b, b])
        o.set_trapezoid("tri", p, A, d, 1, [a, 0, a, a, b - 1, 0, b - 1, b - 1])
    o.write(A, A0, p)
    o.write(B, B0, p)
    o.apply("tri", p, [A, B])
    ms = msgs_list(o)
    exp = []
    for d in range(3):
        a, b = cuts[d], cuts[d + 1]
        if d > 0:
            exp.append((d - 1, d, a - 1, a))  # row a-1, cols [0, a-1]: length a
        if d < 2:
            exp.append((d + 1, d, b, b + 1))  # row b, cols [0, b]: length b+1
    exp.sort(key=lambda t: (t[2], t[1]))
    assert [(m[2], m[3], m[5], m[9] - m[6]) for m in ms] == exp
    assert o.bad_reads() == 0


# ------------------------------------------------------------ Table 3 pins
def _gib(b):
    return b / 2 ** 30


def _run_volume(program, calls):
    """Run calls on a metadata-only oracle; returns per-call off-device bytes
    (host messages excluded) and whether each array's messages were an
    all-gather (every device got every other device's part)."""
    out = []
    for fn in calls:
        fn()
        ms = msgs_list(program)
        out.append(ms)
    return out


def _gemm_like(P, n, layout, kinds):
    o = O.Oracle(simulate_devices=False, eval_kernels=False)
    arrs = {nm: o.create(shape=(n, n)) for nm in ("A", "B", "C", "D", "E")}
    p = o.partition(layout, (n, n), ndev=P)
    for nm in "ABCDE":
        o.write(arrs[nm], np.zeros((n, n), np.float32), p)
    for k in kinds:
        o.kernel(k, O.K_MATMUL)
        o.set_offsets(k, 0, 0, [(0, "*")])
        o.set_offsets(k, 1, 0, [("*", 0)])
        o.set_offsets(k, 2, 1, [(0, 0)])
    return o, arrs, p


def _allgather_bytes(ms, P):
    """Self-inclusive accounting of gathers (each of the P devices receives the
    whole array): off-device bytes * P / (P - 1)."""
    return sum(m[11] for m in ms) * P / (P - 1)


def test_table3_gemm_and_2mm():
    gold = json.load(open(os.path.join(GOLD, "table3_comm_volume.json")))["rows"]
    P, n = 32, 64
    # GEMM: one gather of B on the first call, none afterwards
    o, a, p = _gemm_like(P, n, O.ROW, ["gemm"])
    vols = []
    for it in range(3):
        o.apply("gemm", p, [a["A"], a["B"], a["C"]])
        vols.append(_allgather_bytes(msgs_list(o), P))
    assert vols[0] == P * n * n * 4 and vols[1] == 0 and vols[2] == 0
    N = gold["gemm_row"]["n"]
    assert math.floor(_gib(P * N * N * 4)) == gold["gemm_row"]["printed"]
    # 2MM ROW: D = A x B then E = C x D; B gathered once, D every iteration
    o, a, p = _gemm_like(P, n, O.ROW, ["mm1", "mm2"])
    per = []
    for it in range(3):
        o.apply("mm1", p, [a["A"], a["B"], a["D"]])
        v1 = _allgather_bytes(msgs_list(o), P)
        o.apply("mm2", p, [a["C"], a["D"], a["E"]])
        v2 = _allgather_bytes(msgs_list(o), P)
        per.append((v1, v2))
    full = P * n * n * 4
    assert per[0] == (full, full) and per[1] == (0, full) and per[2] == (0, full)
    iters = gold["2mm_row"]["iters"]
    assert math.floor(_gib((iters + 1) * P * N * N * 4)) == gold["2mm_row"]["printed"]
    # 2MM COL: only A and C are gathered, once
    o, a, p = _gemm_like(P, n, O.COL, ["mm1", "mm2"])
    per = []
    for it in range(3):
        o.apply("mm1", p, [a["A"], a["B"], a["D"]])
        v1 = _allgather_bytes(msgs_list(o), P)
        o.apply("mm2", p, [a["C"], a["D"], a["E"]])
        v2 = _allgather_bytes(msgs_list(o), P)
        per.append((v1, v2))
    assert per[0] == (full, full) and per[1] == (0, 0) and per[2] == (0, 0)
    assert math.floor(_gib(2 * P * N * N * 4)) == gold["2mm_col"]["printed"]


def _stencil_ghost(P, ni, offsets, two_kernels):
    """Sec. 5.1 Jacobi/Convolution host layout: arrays with ghost cells,
    a data partition over the whole array, a work partition without them."""
    n = ni + 2
    o = O.Oracle(simulate_devices=False, eval_kernels=False)
    A, B = o.create(shape=(n, n)), o.create(shape=(n, n))
    pdata = o.partition(O.ROW, (n, n), ndev=P)
    pwork = o.partition(O.ROW, (n, n), (1, 1), (n - 1, n - 1), ndev=P)
    o.write(A, np.zeros((n, n), np.float32), pdata)
    o.write(B, np.zeros((n, n), np.float32), pdata)
    o.kernel("st", O.K_JACOBI2D)
    o.set_offsets("st", 1, 0, offsets)
    o.set_offsets("st", 0, 1, [(0, 0)])
    if two_kernels:
        o.kernel("cp", O.K_COPY)
        o.set_offsets("cp", 1, 0, [(0, 0)])
        o.set_offsets("cp", 0, 1, [(0, 0)])
    vols = []
    for it in range(4):
        o.apply("st", pwork, [A, B])
        v = sum(m[11] for m in msgs_list(o))
        if two_kernels:
            o.apply("cp", pwork, [B, A])
            v += sum(m[11] for m in msgs_list(o))
        vols.append(v)
    return vols


def test_table3_jacobi_and_convolution():
    gold = json.load(open(os.path.join(GOLD, "table3_comm_volume.json")))["rows"]
    P = 32
    jac = [(0, -1), (0, 1), (-1, 0), (1, 0)]
    conv = jac + [(-1, -1), (-1, 1), (1, -1), (1, 1)]
    for ni in (64, 96):
        v = _stencil_ghost(P, ni, jac, True)
        # steady state: one halo row per direction per internal boundary
        assert v[1] == v[2] == v[3] == 2 * (P - 1) * ni * 4
        c = _stencil_ghost(P, ni, conv, False)
        # no data dependency: the halo (ghost corners included) moves once
        assert c[1] == c[2] == c[3] == 0
        assert 2 * (P - 1) * ni * 4 <= c[0] <= 2 * (P - 1) * (ni + 2) * 4 * 2
    N, iters = gold["jacobi_row"]["n_interior"], gold["jacobi_row"]["iters"]
    assert math.floor(_gib(iters * 2 * (P - 1) * N * 4)) == gold["jacobi_row"]["printed"]
    c64 = _stencil_ghost(P, 64, conv, False)[0]
    c96 = _stencil_ghost(P, 96, conv, False)[0]
    slope = (c96 - c64) / 32
    conv_total = c64 + slope * (N - 64)
    assert round(conv_total / 1e6) == gold["convolution_row"]["printed"]


# -------------------------------------------------------- kernel closed forms
def _one_jacobi(field, ndev=4):
    n = field.shape[0]
    o = O.Oracle()
    A, B, p = jacobi_row_program(o, n=n, ndev=ndev, A0=np.zeros_like(field), B0=field)
    o.apply("jacAB", p, [A, B])
    assert o.bad_reads() == 0
    return o.read(A, p), o.truth64(A)


def test_jacobi_closed_forms():
    """Sec. 5.1 Jacobi update: a constant, the bilinear field i*j and any
    linear field are discretely harmonic (fixed points, bit for bit); i^2 gains
    exactly 1/2 on the interior; boundary cells are copied."""
    n = 32
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    for f in (np.full((n, n), 0.5), 3.0 * i + 5.0 * j + 1, i * j, 7.0 * i - 2.0 * j + 100):
        f = f.astype(np.float32)
        a, a64 = _one_jacobi(f)
        assert np.array_equal(a, f)
        assert np.array_equal(a64, f.astype(np.float64))
    q = (i * i).astype(np.float32)
    a, _ = _one_jacobi(q)
    want = q.copy()
    want[1:-1, 1:-1] += 0.5
    assert np.array_equal(a, want)
    # single hot cell: weight 1/4 on each of the four neighbours, 0 at centre
    h = np.zeros((n, n), np.float32)
    h[10, 17] = 1.0
    a, _ = _one_jacobi(h)
    nz = {tuple(x): a[tuple(x)] for x in np.argwhere(a != 0)}
    assert nz == {(9, 17): 0.25, (11, 17): 0.25, (10, 16): 0.25, (10, 18): 0.25}


def test_jacobi_fp32_order_matches_numpy_fp32():
    """numpy float32 arithmetic is IEEE single per operation: the left-to-right
    sum of the paper's formula, then /4, in numpy equals the oracle bitwise."""
    n = 64
    A0, B0 = jacobi_inputs(n, 11)
    o = O.Oracle()
    A, B, p = jacobi_row_program(o, n=n, ndev=4, A0=A0, B0=B0)
    o.apply("jacAB", p, [A, B])
    got = o.read(A, p)
    b = B0
    s = b[1:-1, :-2] + b[1:-1, 2:]
    s = s + b[:-2, 1:-1]
    s = s + b[2:, 1:-1]
    want = b.copy()
    want[1:-1, 1:-1] = s / np.float32(4)
    assert np.array_equal(got, want)


def test_matmul_special_cases():
    """Sec. 3.2 GEMM: B = I gives C = A exactly; ternary inputs make every
    partial sum an exact integer, equal to numpy's int64 product."""
    n = 48
    rng = np.random.default_rng(3)
    a0 = rng.random((n, n), dtype=np.float32)
    o, arrs, p = _mm_program(a0, np.eye(n, dtype=np.float32), 4)
    o.apply("gemm", p, [arrs[0], arrs[1], arrs[2]])
    assert np.array_equal(o.read(arrs[2], p), a0)
    t = rng.integers(-1, 2, (2, n, n))
    o, arrs, p = _mm_program(t[0].astype(np.float32), t[1].astype(np.float32), 4)
    o.apply("gemm", p, [arrs[0], arrs[1], arrs[2]])
    assert np.array_equal(o.read(arrs[2], p), (t[0] @ t[1]).astype(np.float32))
    assert o.bad_reads() == 0


def _mm_program(a0, b0, P):
    n = a0.shape[0]
    o = O.Oracle()
    A, B, Cc = o.create(a0), o.create(b0), o.create(shape=(n, b0.shape[1]))
    p = o.partition(O.ROW, (n, b0.shape[1]), ndev=P)
    o.kernel("gemm", O.K_MATMUL)
    o.set_offsets("gemm", 0, 0, [(0, "*")])
    o.set_offsets("gemm", 1, 0, [("*", 0)])
    o.set_offsets("gemm", 2, 1, [(0, 0)])
    o.write(A, a0, p)
    o.write(B, b0, p)
    return o, (A, B, Cc), p


def _s3d_once(u, coeffs, ndev=8):
    n = u.shape[0]
    o = O.Oracle()
    U, V = o.create(np.zeros_like(u)), o.create(u)
    p = o.partition(O.BLOCK, u.shape, ndev=ndev)
    o.kernel("s3d", O.K_STENCIL3D7)
    o.set_offsets("s3d", 1, 0, [(0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)])
    o.set_offsets("s3d", 0, 1, [(0, 0, 0)])
    o.write(U, np.zeros_like(u), p)
    o.write(V, u, p)
    o.apply("s3d", p, [U, V], list(map(float, coeffs)))
    ms = o.messages()
    assert o.bad_reads() == 0
    return o, o.read(U, p), o.truth64(U), ms


def test_stencil3d_closed_forms():
    """7-point stencil: a linear field along one axis gives sum(c)*f + (c_plus -
    c_minus) on the interior (catches swapped or dropped neighbour terms);
    weights summing to one in powers of two keep a constant field exactly;
    boundary cells are copied; 2x2x2 blocks exchange 24 faces."""
    n = 12
    c = [float(x) for x in S3D_COEFFS]
    c64 = np.array(S3D_COEFFS, dtype=np.float64)
    ii = np.indices((n, n, n)).astype(np.float64)
    for axis, (cm, cp) in enumerate(((1, 2), (3, 4), (5, 6))):
        f = ii[axis] + 1.0
        _, _, u64, ms = _s3d_once(f.astype(np.float32), c)
        want = f.copy()
        want[1:-1, 1:-1, 1:-1] = (c64.sum() * f + (c64[cp] - c64[cm]))[1:-1, 1:-1, 1:-1]
        assert np.allclose(u64, want, rtol=0, atol=1e-12)
        assert len(ms) == 24
    cexact = [0.25] + [0.125] * 6
    f = np.full((n, n, n), 3.5, np.float32)
    _, u, _, _ = _s3d_once(f, cexact)
    assert np.array_equal(u, f)


CONV_OFFSETS = [(di, dj) for di in (-1, 0, 1) for dj in (-1, 0, 1)]


def _conv_once(f, w, ndev=4, kind=None):
    o = O.Oracle()
    n0, n1 = f.shape
    A, B = o.create(np.zeros_like(f)), o.create(f)
    p = o.partition(O.BLOCK if kind is None else kind, f.shape, ndev=ndev)
    o.kernel("conv", O.K_CONV2D9)
    o.set_offsets("conv", 1, 0, CONV_OFFSETS)
    o.set_offsets("conv", 0, 1, [(0, 0)])
    o.write(A, np.zeros_like(f), p)
    o.write(B, f, p)
    o.apply("conv", p, [A, B], [float(x) for x in w])
    ms = o.messages()
    assert o.bad_reads() == 0
    return o, o.read(A, p), o.truth64(A), ms, (A, B, p)


def test_conv2d_closed_forms():
    """3 x 3 convolution (the eight-neighbour kernel of Sec. 5.1): a unit
    impulse reproduces the weights at the mirrored window positions exactly
    (catches a transposed or mirrored window and a dropped term); a linear
    field along each axis gives sum(w) f + (far-side minus near-side weights)
    in FP64; dyadic weights summing to one keep a constant field exactly;
    boundary cells are copied; a 2 x 2 block grid exchanges 8 strips and
    4 corner cells."""
    w = [float(x) for x in CONV9_WEIGHTS]
    n = 14
    f = np.zeros((n, n), np.float32)
    r, c = 6, 7
    f[r, c] = 1.0
    _, u, _, ms, _ = _conv_once(f, w)
    want = np.zeros_like(f)
    for k, (di, dj) in enumerate(CONV_OFFSETS):
        want[r - di, c - dj] = np.float32(w[k])
    want[0, :], want[-1, :], want[:, 0], want[:, -1] = f[0, :], f[-1, :], f[:, 0], f[:, -1]
    assert np.array_equal(u, want)
    # 2 x 2 blocks: each device receives two strips and one corner cell
    assert len(ms) == 8 + 4
    assert sorted(int(m[11]) for m in ms)[:4] == [4, 4, 4, 4]
    w64 = np.array(CONV9_WEIGHTS, dtype=np.float64).reshape(3, 3)
    ii = np.indices((n, n)).astype(np.float64)
    for axis in (0, 1):
        g = ii[axis] + 1.0
        _, _, u64, _, _ = _conv_once(g.astype(np.float32), w)
        lo, hi = (w64[0, :].sum(), w64[2, :].sum()) if axis == 0 else (w64[:, 0].sum(), w64[:, 2].sum())
        want = g.copy()
        want[1:-1, 1:-1] = (w64.sum() * g + (hi - lo))[1:-1, 1:-1]
        assert np.allclose(u64, want, rtol=0, atol=1e-12)
    dy = [1 / 16, 1 / 8, 1 / 16, 1 / 8, 1 / 4, 1 / 8, 1 / 16, 1 / 8, 1 / 16]
    f = np.full((n, 11), 2.75, np.float32)
    _, u, _, _, _ = _conv_once(f, dy, ndev=3, kind=O.ROW)
    assert np.array_equal(u, f)


def test_conv2d_fp32_within_bound_and_comm_once():
    """FP32 run vs the FP64 run within the error bound of a 9-term
    multiply-add chain; repeated calls with the input never redefined move
    their halo once (Table 3's Convolution row)."""
    w = [float(x) for x in CONV9_WEIGHTS]
    rng = np.random.default_rng(21)
    f = rng.random((40, 37), dtype=np.float32)
    o, u, u64, ms, (A, B, p) = _conv_once(f, w, ndev=6)
    aw = np.abs(np.array(CONV9_WEIGHTS, dtype=np.float64))
    mag = np.zeros_like(u64)
    fa = np.abs(f.astype(np.float64))
    for k, (di, dj) in enumerate(CONV_OFFSETS):
        mag[1:-1, 1:-1] += aw[k] * fa[1 + di:f.shape[0] - 1 + di, 1 + dj:f.shape[1] - 1 + dj]
    gamma = 9 * 2.0 ** -24 / (1 - 9 * 2.0 ** -24)
    assert np.all(np.abs(u - u64) <= gamma * mag)
    assert len(ms) > 0
    for _ in range(2):
        o.apply("conv", p, [A, B], w)
        assert len(o.messages()) == 0


def test_s3d_adjoint_fp64_dot_product_and_fd():
    """The FP64 adjoint is the transpose: <S^T w, v> = <w, S v> for one step
    (dot-product test), and L = sum(w * u_T) is linear in u0, so central
    differences along random directions are exact up to rounding; the
    coefficient gradient matches central differences with h = 1e-6."""
    n, T = 8, 3
    rng = np.random.default_rng(5)
    c = np.array(S3D_COEFFS, dtype=np.float64)
    u0 = rng.random((n, n, n))
    w = rng.random((n, n, n))
    v = rng.random((n, n, n))
    g1, _ = O.s3d_adjoint64(u0, c, 1, w)
    sv = O.s3d_forward64(v, c, 1)
    assert abs(np.sum(g1 * v) - np.sum(w * sv)) <= 1e-12 * abs(np.sum(w * sv))
    g, gc = O.s3d_adjoint64(u0, c, T, w)

    def loss(u, cc):
        return float(np.sum(w * O.s3d_forward64(u, cc, T)))

    for _ in range(3):
        d = rng.standard_normal((n, n, n))
        fd = (loss(u0 + d, c) - loss(u0 - d, c)) / 2
        assert abs(fd - np.sum(g * d)) <= 1e-10 * abs(fd)
    h = 1e-6
    for e in range(7):
        cp, cm = c.copy(), c.copy()
        cp[e] += h
        cm[e] -= h
        fd = (loss(u0, cp) - loss(u0, cm)) / (2 * h)
        assert abs(fd - gc[e]) <= 1e-6 * abs(fd)


def _s3d_gather_adjoint(u0, c, T, w, sign=1):
    """The adjoint of the fixed-boundary 7-point step in gather form (the
    transposed stencil): every point x collects c_e g(x - o_e) from the
    interior points that read it through offset o_e, plus g(x) itself when x
    is a boundary point (copied forward).  sign=-1 mirrors every offset."""
    n = u0.shape
    inner = np.zeros(n, dtype=bool)
    inner[1:-1, 1:-1, 1:-1] = True
    offs = [(0, 0), (0, -1), (0, 1), (1, -1), (1, 1), (2, -1), (2, 1)]
    states = [u0]
    for _ in range(T):
        states.append(O.s3d_forward64(states[-1], c, 1))
    g = w.copy()
    gc = np.zeros(7)
    for t in range(T - 1, -1, -1):
        gi = np.where(inner, g, 0.0)  # zero on the boundary planes: rolls wrap in zeros
        h = np.where(inner, 0.0, g)
        for e, (ax, o) in enumerate(offs):
            h += c[e] * np.roll(gi, sign * o, axis=ax)
            gc[e] += np.sum(gi * np.roll(states[t], -sign * o, axis=ax))
        g = h
    return g, gc


def test_s3d_adjoint_gather_form_matches_scatter_add():
    """The oracle's adjoint scatters c_e g(y) into y + o_e from every interior
    y; the gather form (transposed stencil, the form the GPU adjoint kernel
    evaluates) reaches the same dL/du0 and dL/dc within 1e-6 relative on a
    non-cubic block over several steps; mirroring the offsets in the gather
    form breaks the agreement (the asymmetric coefficients see to it)."""
    rng = np.random.default_rng(61)
    c = np.array(S3D_COEFFS, dtype=np.float64)
    u0 = rng.random((7, 9, 6))
    w = rng.random((7, 9, 6))
    T = 4
    gs, gcs = O.s3d_adjoint64(u0, c, T, w)
    gg, gcg = _s3d_gather_adjoint(u0, c, T, w)
    assert np.max(np.abs(gg - gs)) <= 1e-6 * np.max(np.abs(gs))
    assert np.all(np.abs(gcg - gcs) <= 1e-6 * np.abs(gcs))
    gm, gcm = _s3d_gather_adjoint(u0, c, T, w, sign=-1)
    assert np.max(np.abs(gm - gs)) > 1e-3 * np.max(np.abs(gs))
    assert np.max(np.abs(gcm - gcs) / np.abs(gcs)) > 1e-3


# --------------------------------------------------------------- partitions
def test_partition_even_and_manual():
    """Table 2 Partition splits the region evenly; Listing 1's manual regions
    (0,3008),(3008,7232) share the cut, i.e. are half-open."""
    o = O.Oracle(simulate_devices=False, eval_kernels=False)
    p = o.partition(O.ROW, (1024, 1024), ndev=2)
    assert o.part_region(p, 0) == ((0, 0, 0), (1, 512, 1024))
    assert o.part_region(p, 1) == ((0, 512, 0), (1, 1024, 1024))
    p = o.partition(O.ROW, (10, 4), ndev=3)
    assert [o.part_region(p, d)[0][1] for d in range(3)] == [0, 3, 6]
    q = o.partition_manual([(0, 0), (3008, 0)], [(3008, 10240), (7232, 10240)])
    assert o.part_region(q, 0)[1][1] == o.part_region(q, 1)[0][1] == 3008
    b = o.partition(O.BLOCK, (64, 64), ndev=16)
    assert {o.part_region(b, d)[0][1:] for d in range(16)} == {(r, c) for r in range(0, 64, 16) for c in range(0, 64, 16)}
    assert o.part_region(b, 1)[0] == (0, 0, 16)  # device ids row-major over the grid
    b8 = o.partition(O.BLOCK, (64, 64), ndev=8)
    assert o.part_region(b8, 0)[1] == (1, 16, 32)  # 4 x 2 grid
    b3 = o.partition(O.BLOCK, (8, 8, 8), ndev=8)
    assert o.part_region(b3, 7) == ((4, 4, 4), (8, 8, 8))
    c = o.partition(O.COL, (8, 12), ndev=3)
    assert o.part_region(c, 2) == ((0, 0, 8), (1, 8, 12))


# -------------------------------------------------------------- invariants
def _masks_for_program(shape, shapes_by_dst):
    ns = canon.nshape(shape)
    out = {}
    for d, boxes in shapes_by_dst.items():
        m = np.zeros(ns, dtype=bool)
        for lo, hi in boxes:
            m[tuple(slice(a, b) for a, b in zip(lo, hi))] = True
        out[d] = m
    return out


@pytest.mark.parametrize("seed", range(12))
def test_random_programs_canonical_messages_and_gdef(seed):
    """Random sequences of Write / ApplyKernel (random absolute use and def
    boxes, random partitions) / Read on small 2-D and 3-D arrays: the message
    table satisfies the canonical-decomposition properties against the element
    sets computed here from the GDEF dump (Eq. 1-2); GDEF after the call obeys
    Eq. 3-4 with overwrite kill; owner is always a holder; the oracle's own
    coherence check passes and no kernel read is incoherent."""
    rng = np.random.default_rng(100 + seed)
    dim = 2 if seed % 3 else 3
    shape = tuple(int(x) for x in rng.integers(5, 14 if dim == 2 else 7, size=dim))
    o = O.Oracle()
    X = o.create(rng.random(shape, dtype=np.float32))
    Y = o.create(rng.random(shape, dtype=np.float32))
    ndev = int(rng.integers(2, 7))
    part = o.partition(int(rng.integers(0, 3)), shape, ndev=ndev)
    o.write(X, rng.random(shape, dtype=np.float32), part)
    ns = canon.nshape(shape)
    for step in range(6):
        kname = f"k{step}"
        o.kernel(kname, O.K_COPY)
        out, inp = (X, Y) if step % 2 else (Y, X)
        use, dfn = {}, {}
        for d in range(ndev):
            lo, hi = o.part_region(part, d)
            if any(a >= b for a, b in zip(lo, hi)):
                continue
            # def = own work region (the copy kernel writes exactly that)
            dlo, dhi = lo[3 - dim:], hi[3 - dim:]
            o.set_absolute(kname, part, out, d, 1, dlo, dhi)
            dfn[d] = [(lo, hi)]
            boxes = [(lo, hi)]
            for _ in range(int(rng.integers(0, 3))):
                blo = [int(rng.integers(0, s)) for s in shape]
                bhi = [int(rng.integers(b + 1, s + 1)) for b, s in zip(blo, shape)]
                o.set_absolute(kname, part, inp, d, 0, blo, bhi)
                boxes.append((tuple([0] * (3 - dim) + blo), tuple([1] * (3 - dim) + bhi)))
            o.set_absolute(kname, part, inp, d, 0, dlo, dhi)
            use[d] = boxes
        own_b, hold_b = o.gdef(inp)
        own_b, hold_b = own_b.reshape(ns), hold_b.reshape(ns)
        o.apply(kname, part, [out, inp])
        ms = o.messages()
        exp = canon.expected_sets(_masks_for_program(shape, use), own_b, hold_b)
        canon.check_array_messages(ms, exp)
        canon.check_order_and_offsets(ms, {X.id: 4, Y.id: 4})
        assert np.array_equal(o.pack(), canon.pack_from_values(ms, {inp.id: o.truth(inp)}))
        own_a, hold_a = o.gdef(inp)
        want = hold_b.copy()
        for d, e in exp.items():
            want[e >= 0] |= np.uint64(1) << np.uint64(d)
        assert np.array_equal(hold_a.reshape(ns), want)
        assert np.array_equal(own_a.reshape(ns), own_b)
        own_o, hold_o = o.gdef(out)
        own_o, hold_o = own_o.reshape(ns), hold_o.reshape(ns)
        for d, bl in dfn.items():
            (lo, hi), = bl
            sl = tuple(slice(a, b) for a, b in zip(lo, hi))
            assert np.all(own_o[sl] == d) and np.all(hold_o[sl] == np.uint64(1) << np.uint64(d))
        for arr in (X, Y):
            ow, ho = o.gdef(arr)
            bit = (ho >> ow.astype(np.uint64)) & np.uint64(1)
            assert np.all(bit == 1)
    assert o.bad_reads() == 0
    got = o.read(X, part)
    assert np.array_equal(got, o.truth(X))


def test_dropped_message_is_detected():
    """Self-check of the oracle: losing one message breaks the coherence
    invariant (every element a device uses holds the last-defined value)."""
    o = O.Oracle()
    A, B, p = jacobi_row_program(o)
    o.inject_drop(2)
    with pytest.raises(O.OracleError) as e:
        o.apply("jacAB", p, [A, B])
    assert e.value.code == O.ECOHERENCE


def test_under_declared_use_is_flagged():
    """A use region without the halo leaves the stencil reading values the
    device does not hold; the oracle counts those reads."""
    n = 32
    o = O.Oracle()
    A0, B0 = jacobi_inputs(n, 1)
    A, B = o.create(A0), o.create(B0)
    p = o.partition(O.ROW, (n, n), ndev=4)
    o.kernel("jac", O.K_JACOBI2D)
    o.set_offsets("jac", 1, 0, [(0, 0)])
    o.set_offsets("jac", 0, 1, [(0, 0)])
    o.write(A, A0, p)
    o.write(B, B0, p)
    # make the halo rows stale on the neighbours first
    o.apply("jac", p, [A, B])
    assert o.bad_reads() > 0


# ------------------------------------------------------------- error paths
def test_error_paths():
    o = O.Oracle()
    n = 16
    A, B = o.create(shape=(n, n)), o.create(shape=(n, n))
    p = o.partition(O.ROW, (n, n), ndev=2)
    o.kernel("jac", O.K_JACOBI2D)
    o.set_absolute("jac", p, A, 0, 1, (0, 0), (9, n))
    o.set_absolute("jac", p, A, 1, 1, (8, 0), (n, n))
    with pytest.raises(O.OracleError) as e:
        o.apply("jac", p, [A, B])
    assert e.value.code == O.ERACE
    with pytest.raises(O.OracleError) as e:
        o.set_absolute("jac", p, A, 0, 0, (0, 0), (n + 1, n))
    assert e.value.code == O.EBOUNDS
    with pytest.raises(O.OracleError) as e:
        o.set_trapezoid("jac", p, A, 0, 0, [0, 0, 1, 3, 5, 0, 5, 5])
    assert e.value.code == O.EINVAL
    with pytest.raises(O.OracleError):
        o.apply("jac", p, [A, A])
    with pytest.raises(O.OracleError):
        o.kernel("bad", 99)
    q = o.partition_manual([(0, 0), (4, 0)], [(8, n), (n, n)])
    with pytest.raises(O.OracleError) as e:
        o.write(A, np.zeros((n, n), np.float32), q)
    assert e.value.code == O.EINVAL


# -------------------------------------------------------- read/write/reduce
def test_read_write_reduce():
    """Table 2 Read/Write/Reduce: write then read returns the data; a read
    after a kernel brings each section from its owner to the host; reductions
    match numpy (FP64 sums within one rounding per term, integer SUM wraps)."""
    n = 24
    o = O.Oracle()
    A0, B0 = jacobi_inputs(n, 4)
    A, B, p = jacobi_row_program(o, n=n, ndev=3, A0=A0, B0=B0)
    assert np.array_equal(o.read(B, p), B0)
    assert len(o.messages()) == 0  # host already holds what Write gave it
    o.apply("jacAB", p, [A, B])
    a = o.read(A, p)
    ms = msgs_list(o)
    assert {m[3] for m in ms} == {O.HOST} and sorted({m[2] for m in ms}) == [0, 1, 2]
    assert np.array_equal(a, o.truth(A))
    assert len(o.messages()) > 0
    o.read(A, p)
    assert len(o.messages()) == 0
    s = o.reduce(A, O.SUM, p)
    assert abs(s - float(np.sum(a.astype(np.float64)))) <= n * n * 2 ** -52 * float(np.sum(np.abs(a)))
    assert o.reduce(A, O.MAX, p) == float(a.max())
    assert o.reduce(A, O.MIN, p) == float(a.min())
    iv = np.arange(n * n, dtype=np.int32).reshape(n, n) * 7919
    I = o.create(shape=(n, n), type_=O.I32)
    o.write(I, iv, p)
    assert o.reduce(I, O.SUM, p) == int(np.sum(iv.astype(np.int64))) % 2 ** 32 - (
        2 ** 32 if int(np.sum(iv.astype(np.int64))) % 2 ** 32 >= 2 ** 31 else 0)
    assert o.reduce(I, O.MAX, p) == int(iv.max())
