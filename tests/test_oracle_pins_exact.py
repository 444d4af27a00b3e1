"""More pins of the CPU oracle (CPU only): trapezoid rasterisation against a
hand-written fixture, the FP32 operation chains of the 7-point stencil, the
3 x 3 convolution and the Jacobi update against an exact rational evaluation
rounded once per operation, the FP64 whole-array stencil against closed forms
and the partitioned oracle, and the PROD reduction against exact products.

Each pin is chosen so that a plausible mistake in the oracle (truncation for
floor, swapped corners, an unfused multiply-add, a reordered chain, a
mirrored neighbour, a wrong PROD identity) fails it; the discriminating tests
also check that the mistaken variant really gives a different answer on the
chosen input.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from tests import exact_f32 as X
from workloads import CONV9_WEIGHTS, S3D_COEFFS

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------ exact helper
def test_round_f32_ties_and_ranges():
    """The rounding helper itself, on values whose binary32 rounding is known
    from the format: ties go to the even significand, halfway cases above and
    below 1, the subnormal spacing 2^-149 and the largest finite value."""
    one = Fraction(1)
    u = Fraction(1, 2 ** 23)  # spacing of [1, 2)
    assert X.round_f32(one + u / 2) == 1.0                      # tie, 1 is even
    assert X.round_f32(one + 3 * u / 2) == float(one + 2 * u)  # tie, 1+u is odd -> up
    assert X.round_f32(one + u / 2 + Fraction(1, 2 ** 60)) == float(one + u)
    assert X.round_f32(one - Fraction(1, 2 ** 25)) == 1.0       # tie below 1 (spacing 2^-24): to even 1
    assert X.round_f32(Fraction(3, 2 ** 150)) == 2.0 ** -148    # 1.5 subnormal ulps: tie to even (2)
    assert X.round_f32(Fraction(1, 3)) == float(Fraction(11184811, 2 ** 25))
    big = (2 - Fraction(1, 2 ** 23)) * Fraction(2) ** 127
    assert X.round_f32(big) == float(big)
    assert X.round_f32(-Fraction(5, 4)) == -1.25


# -------------------------------------------------------------- trapezoids
def _trap_masks(shape, corners):
    """Use and def masks the oracle derives for one trapezoid on one device:
    the use shows up as holder bit 0 of the input after the call (it arrives
    from the host), the def as owner 0 of the output."""
    o = O.Oracle(simulate_devices=False, eval_kernels=False)
    A = o.create(np.zeros(shape, np.float32))
    B = o.create(np.arange(np.prod(shape), dtype=np.float32).reshape(shape))
    p = o.partition(O.ROW, shape, ndev=1)
    o.kernel("cp", O.K_COPY)
    o.set_trapezoid("cp", p, B, 0, 0, corners)
    o.set_trapezoid("cp", p, A, 0, 1, corners)
    o.apply("cp", p, [A, B])
    own_a, _ = o.gdef(A)
    _, hold_b = o.gdef(B)
    msgs = o.messages()
    o.close()
    return (hold_b & 1).astype(bool), own_a == 0, msgs


def test_trapezoid_rows_match_hand_derivation():
    """Table 2 SetTrapezoidUse/Def: every row span of five trapezoids with
    non-unit and negative edge slopes, clipping on both sides, a one-row
    trapezoid and crossed edges, as derived by hand in the fixture."""
    gold = json.load(open(os.path.join(GOLD, "trapezoid_rows.json")))
    shape = tuple(gold["array_shape"])
    for case in gold["cases"]:
        want = np.zeros(shape, bool)
        for r, c0, c1 in case["rows"]:
            want[r, c0:c1 + 1] = True
        use, dfn, msgs = _trap_masks(shape, case["corners"])
        assert np.array_equal(use, want), case["name"]
        assert np.array_equal(dfn, want), case["name"]
        # every message comes from the host and the rectangles tile the mask
        got = np.zeros(shape, bool)
        for m in msgs:
            assert m[2] == O.HOST and m[3] == 0
            assert not got[m[5]:m[8], m[6]:m[9]].any()
            got[m[5]:m[8], m[6]:m[9]] = True
        assert np.array_equal(got, want), case["name"]


def test_trapezoid_fixture_discriminates_truncation():
    """Truncating the edge quotients toward zero instead of flooring them
    changes a row of the first fixture case (so the pin above catches it)."""
    gold = json.load(open(os.path.join(GOLD, "trapezoid_rows.json")))
    c = gold["cases"][0]["corners"]
    r0, r1 = c[0], c[4]
    trunc_left = [c[1] + int((r - r0) * (c[5] - c[1]) / (r1 - r0)) for r in range(r0, r1 + 1)]
    assert trunc_left != [row[1] for row in gold["cases"][0]["rows"]]


# ------------------------------------------------------ FP32 chains, exact
def _s3d_exact(u, c, fused=True, order=(0, 1, 2, 3, 4, 5, 6)):
    """7-point stencil by exact arithmetic: acc = round(c0*u), then per
    neighbour (-i, +i, -j, +j, -k, +k) one rounding of c_e*u_e + acc
    (fused), or of the product and then of the sum (unfused)."""
    n0, n1, n2 = u.shape
    out = u.astype(np.float64).copy()
    offs = [(0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
    for i in range(1, n0 - 1):
        for j in range(1, n1 - 1):
            for k in range(1, n2 - 1):
                e0 = order[0]
                di, dj, dk = offs[e0]
                acc = X.mul(c[e0], u[i + di, j + dj, k + dk])
                for e in order[1:]:
                    di, dj, dk = offs[e]
                    v = u[i + di, j + dj, k + dk]
                    acc = X.fma(c[e], v, acc) if fused else X.add(X.mul(c[e], v), acc)
                out[i, j, k] = acc
    return out.astype(np.float32)


def _s3d_oracle(u, coeffs, ndev=8):
    o = O.Oracle()
    U, V = o.create(np.zeros_like(u)), o.create(u)
    p = o.partition(O.BLOCK, u.shape, ndev=ndev)
    o.kernel("s3d", O.K_STENCIL3D7)
    o.set_offsets("s3d", 1, 0, [(0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)])
    o.set_offsets("s3d", 0, 1, [(0, 0, 0)])
    o.write(U, np.zeros_like(u), p)
    o.write(V, u, p)
    o.apply("s3d", p, [U, V], list(map(float, coeffs)))
    assert o.bad_reads() == 0
    out = o.read(U, p)
    o.close()
    return out


def test_stencil3d_fp32_chain_exact():
    """The oracle's FP32 7-point stencil equals, bit for bit, the exact
    evaluation with one rounding per fused multiply-add in the stated order
    (centre product first, then -i, +i, -j, +j, -k, +k), on random inputs
    where an unfused chain or another order gives different bits."""
    rng = np.random.default_rng(77)
    u = rng.random((6, 7, 9), dtype=np.float32)
    c = [np.float32(x) for x in S3D_COEFFS]
    want = _s3d_exact(u, c)
    got = _s3d_oracle(u, c)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    assert not np.array_equal(_s3d_exact(u, c, fused=False), want)
    assert not np.array_equal(_s3d_exact(u, c, order=(0, 2, 1, 3, 4, 5, 6)), want)


def _conv_exact(f, w, fused=True, row_major=True):
    n0, n1 = f.shape
    out = f.astype(np.float64).copy()
    cells = [(di, dj) for di in (-1, 0, 1) for dj in (-1, 0, 1)]
    order = list(range(9)) if row_major else [3 * (k % 3) + k // 3 for k in range(9)]
    for i in range(1, n0 - 1):
        for j in range(1, n1 - 1):
            acc = None
            for k in order:
                di, dj = cells[k]
                v = f[i + di, j + dj]
                if acc is None:
                    acc = X.mul(w[k], v)
                else:
                    acc = X.fma(w[k], v, acc) if fused else X.add(X.mul(w[k], v), acc)
            out[i, j] = acc
    return out.astype(np.float32)


def test_conv2d_fp32_chain_exact():
    """The oracle's FP32 3 x 3 convolution equals the exact evaluation with
    the first product rounded and then one rounding per fused multiply-add,
    window row by row; an unfused chain or a column-by-column window differ
    on the same input."""
    rng = np.random.default_rng(78)
    f = rng.random((9, 13), dtype=np.float32)
    w = [np.float32(x) for x in CONV9_WEIGHTS]
    o = O.Oracle()
    A, B = o.create(np.zeros_like(f)), o.create(f)
    p = o.partition(O.BLOCK, f.shape, ndev=4)
    o.kernel("conv", O.K_CONV2D9)
    o.set_offsets("conv", 1, 0, [(di, dj) for di in (-1, 0, 1) for dj in (-1, 0, 1)])
    o.set_offsets("conv", 0, 1, [(0, 0)])
    o.write(A, np.zeros_like(f), p)
    o.write(B, f, p)
    o.apply("conv", p, [A, B], [float(x) for x in w])
    got = o.read(A, p)
    o.close()
    want = _conv_exact(f, w)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    assert not np.array_equal(_conv_exact(f, w, fused=False), want)
    assert not np.array_equal(_conv_exact(f, w, row_major=False), want)


def test_jacobi_fp32_chain_exact():
    """Sec. 5.1 Jacobi in the oracle: ((w + e) + n) + s, each sum rounded,
    then divided by 4, equals the exact evaluation; summing in another order
    differs on the same input."""
    rng = np.random.default_rng(79)
    b = rng.random((11, 10), dtype=np.float32)
    o = O.Oracle()
    A, B = o.create(np.zeros_like(b)), o.create(b)
    p = o.partition(O.ROW, b.shape, ndev=3)
    o.kernel("jac", O.K_JACOBI2D)
    o.set_offsets("jac", 1, 0, [(0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)])
    o.set_offsets("jac", 0, 1, [(0, 0)])
    o.write(A, np.zeros_like(b), p)
    o.write(B, b, p)
    o.apply("jac", p, [A, B])
    got = o.read(A, p)
    o.close()

    def exact(order):
        out = b.astype(np.float64).copy()
        for i in range(1, b.shape[0] - 1):
            for j in range(1, b.shape[1] - 1):
                t = [b[i, j - 1], b[i, j + 1], b[i - 1, j], b[i + 1, j]]
                s = X.add(t[order[0]], t[order[1]])
                s = X.add(s, t[order[2]])
                s = X.add(s, t[order[3]])
                out[i, j] = X.div(s, 4.0)
        return out.astype(np.float32)

    want = exact((0, 1, 2, 3))
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    assert not np.array_equal(exact((2, 3, 0, 1)), want)


# ------------------------------------------------- FP64 whole-array stencil
def test_s3d_forward64_closed_forms_and_partitioned_oracle():
    """The whole-array FP64 stencil (reference of the adjoint tests): a linear
    field along each axis gives sum(c) f + (c_plus - c_minus) on the interior
    and the boundary copied (a mirrored neighbour swaps the +/- weights and
    fails); three steps equal, bit for bit, the FP64 shadow of the partitioned
    oracle run for three ping-pong ApplyKernel calls."""
    n = 9
    c64 = np.array(S3D_COEFFS, dtype=np.float64)
    ii = np.indices((n, n, n)).astype(np.float64)
    for axis, (cm, cp) in enumerate(((1, 2), (3, 4), (5, 6))):
        f = 2.0 * ii[axis] + 1.0
        got = O.s3d_forward64(f, c64, 1)
        want = f.copy()
        want[1:-1, 1:-1, 1:-1] = (c64.sum() * f + 2.0 * (c64[cp] - c64[cm]))[1:-1, 1:-1, 1:-1]
        assert np.allclose(got, want, rtol=0, atol=1e-12)
        mirrored = f.copy()
        mirrored[1:-1, 1:-1, 1:-1] = (c64.sum() * f + 2.0 * (c64[cm] - c64[cp]))[1:-1, 1:-1, 1:-1]
        assert not np.allclose(got, mirrored, rtol=0, atol=1e-6)
    rng = np.random.default_rng(80)
    u0 = rng.random((7, 8, 6), dtype=np.float32)
    o = O.Oracle()
    U, V = o.create(u0), o.create(np.zeros_like(u0))
    p = o.partition(O.BLOCK, u0.shape, ndev=8)
    offs = [(0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
    for k in ("uv", "vu"):
        o.kernel(k, O.K_STENCIL3D7)
        o.set_offsets(k, 1, 0, offs)
        o.set_offsets(k, 0, 1, [(0, 0, 0)])
    o.write(U, u0, p)
    o.write(V, np.zeros_like(u0), p)
    cs = [float(x) for x in S3D_COEFFS]
    o.apply("uv", p, [V, U], cs)
    o.apply("vu", p, [U, V], cs)
    o.apply("uv", p, [V, U], cs)
    shadow = o.truth64(V)
    o.close()
    ref = O.s3d_forward64(u0.astype(np.float64), c64, 3)
    assert np.array_equal(ref, shadow)


# ----------------------------------------------------------- reduce PROD
def _reduce_program(vals, type_, ndev=3):
    o = O.Oracle()
    A = o.create(shape=vals.shape, type_=type_)
    p = o.partition(O.ROW, vals.shape, ndev=ndev)
    o.write(A, vals, p)
    return o, A, p


def test_reduce_prod_integer_wraps_mod_2_32():
    """Table 2 Reduce with PROD on int data: the product of all elements
    modulo 2^32 as a signed 32-bit value (exact Python integers), including
    negative factors and a product that overflows many times."""
    rng = np.random.default_rng(81)
    # odd factors (an even product would soon be 0 modulo 2^32)
    vals = (2 * rng.integers(-6, 6, (12, 7)) + 1).astype(np.int32)
    o, A, p = _reduce_program(vals, O.I32)
    prod = 1
    for v in vals.ravel().tolist():
        prod = (prod * v) % 2 ** 32
    want = prod - 2 ** 32 if prod >= 2 ** 31 else prod
    assert abs(math.prod(vals.ravel().tolist())) > 2 ** 64  # really wraps
    assert o.reduce(A, O.PROD, p) == want
    # an identity of 0 or a dropped partial changes the result
    part = math.prod(vals[4:].ravel().tolist()) % 2 ** 32
    assert want != 0 and want != (part - 2 ** 32 if part >= 2 ** 31 else part)
    o.close()


def test_reduce_prod_float_against_exact_product():
    """PROD on fp32 data: FP64 accumulation agrees with the exact rational
    product within n * 2^-53 relative; a zero anywhere gives exactly 0 and
    the sign follows the count of negative factors."""
    rng = np.random.default_rng(82)
    k = rng.integers(-8, 9, (10, 9))
    vals = (1.0 + k / 64.0).astype(np.float32)
    vals[3, 4] = -vals[3, 4]
    o, A, p = _reduce_program(vals, O.F32)
    exact = Fraction(1)
    for v in vals.ravel().tolist():
        exact *= Fraction(v)
    got = o.reduce(A, O.PROD, p)
    n = vals.size
    assert got < 0
    assert abs(Fraction(got) - exact) <= abs(exact) * Fraction(n + 3, 2 ** 53)
    o.close()
    vals[7, 1] = 0.0
    o, A, p = _reduce_program(vals, O.F32)
    assert o.reduce(A, O.PROD, p) == 0.0
    o.close()
