"""Parity at the workloads' full sizes (through the C ABI):

  jacobi_large  8192 x 8192, 4 x 4 blocks, 5-point offsets: two ping-pong
                steps, message tables, pack buffers, GDEF maps and values
                bit-exact;
  matmul        4096 x 4096, 8 row blocks (and 1000 / 3, 1024 / 4: more than
                128 rows per device, sizes not a multiple of the tile): the
                gather of B on the first call and no message on the second,
                GDEF bit-exact; C against the FP64 product within
                K * 2^-24 * (|A||B|)_ij everywhere, and bit-exact for ternary
                inputs (every partial sum exact);
  batched       the whole seed-4 instance (64 arrays, 279 M elements per
                array set): two batched steps against the per-call oracle.

The oracle runs without its per-device simulation here (the global values,
messages, pack buffers and GDEF it reports are the same; the simulation only
re-checks coherence, which the smaller cases cover).
"""
import sys

import numpy as np
import pytest

import oracle as O
from tests.test_gpu_batch import _check_tables, _oracle_step, _record
from workloads import batched_instance, jacobi_inputs, matmul_inputs, ternary_matmul_inputs
from workloads import programs as prog

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


def _same_gdef(rt, orc, pairs, what):
    for ag, ao in pairs:
        og, hg = rt.gdef(ag)
        oo, ho = orc.gdef(ao)
        assert np.array_equal(og, oo), f"{what}: owner map differs"
        assert np.array_equal(hg, ho), f"{what}: holder map differs"
        del og, hg, oo, ho


@pytest.mark.timeout(600)
def test_jacobi_large_fullsize(hd):
    """8192^2 Jacobi on 16 devices (4 x 4 blocks, 5-point offsets): 48 halo
    messages per step, everything bit-exact over two ping-pong steps."""
    say("case jacobi_large 8192x8192 ndev=16 steps=2")
    A0, B0 = jacobi_inputs(8192, 2)
    rt, orc = hd.Runtime(), O.Oracle(simulate_devices=False)
    g = prog.jacobi_blocks(rt, A0, B0, 16)
    o = prog.jacobi_blocks(orc, A0, B0, 16)
    for it in range(2):
        k, ag, ao = ("jacAB", [g[0], g[1]], [o[0], o[1]]) if it % 2 == 0 else ("jacBA", [g[1], g[0]], [o[1], o[0]])
        rt.apply(k, g[2], ag)
        orc.apply(k, o[2], ao)
        mg, mo = rt.messages(), orc.messages()
        assert len(mo) == 48
        assert np.array_equal(mg, mo), f"step {it}: message tables differ"
        assert np.array_equal(rt.pack(), orc.pack()), f"step {it}: pack buffers differ"
        _same_gdef(rt, orc, [(g[0], o[0]), (g[1], o[1])], f"step {it}")
        say(f"  step {it}: tables, pack and GDEF equal")
    for ag, ao in ((g[0], o[0]), (g[1], o[1])):
        assert np.array_equal(rt.read(ag, g[2]), orc.read(ao, o[2]))
    rt.close()
    orc.close()


def _check_product(cg, a0, b0, exact):
    a64, b64 = a0.astype(np.float64), b0.astype(np.float64)
    c64 = a64 @ b64
    if exact:
        assert np.array_equal(cg, c64.astype(np.float32))
        return 0.0, 0.0
    bound = a0.shape[1] * 2.0 ** -24 * (np.abs(a64) @ np.abs(b64))
    err = np.abs(cg.astype(np.float64) - c64)
    assert np.all(err <= bound)
    return float(err.max()), float(np.sqrt(np.mean(err ** 2)))


@pytest.mark.timeout(600)
@pytest.mark.parametrize("n,P", [(4096, 8), (1000, 3), (1024, 4)])
def test_matmul_fullsize(hd, n, P):
    """GEMM of Listings 2-3 with the row split of the matmul workload: first
    call gathers all of B to every device (P (P - 1) messages), later calls
    send nothing; C within the FP32 bound (random) and exact (ternary)."""
    for kind, (a0, b0) in (("random", matmul_inputs(n, 3)), ("ternary", ternary_matmul_inputs(n, 4))):
        say(f"case matmul {kind} n={n} P={P}")
        rt, orc = hd.Runtime(), O.Oracle(simulate_devices=False, eval_kernels=False)
        g = prog.gemm(rt, a0, b0, P)
        o = prog.gemm(orc, a0, b0, P)
        for it in range(2):
            rt.apply("gemm", g[3], list(g[:3]))
            orc.apply("gemm", o[3], list(o[:3]))
            mg, mo = rt.messages(), orc.messages()
            assert len(mo) == (P * (P - 1) if it == 0 else 0)
            assert np.array_equal(mg, mo), f"call {it}: message tables differ"
            assert np.array_equal(rt.pack(), orc.pack()), f"call {it}: pack buffers differ"
            _same_gdef(rt, orc, [(g[1], o[1]), (g[2], o[2])], f"call {it}")
        cg = rt.read(g[2], g[3])
        emax, erms = _check_product(cg, a0, b0, kind == "ternary")
        say(f"  {kind}: max |C - C64| = {emax:.3e}, rms {erms:.3e}")
        rt.close()
        orc.close()


@pytest.mark.timeout(900)
def test_batched_fullsize(hd):
    """The whole seed-4 batched instance (64 arrays, sides 512-4096, 2-32
    irregular row partitions, stencil and lower-triangular): two batched
    steps, each call's message table, the pack buffer, every array's values
    and GDEF against the oracle running the calls one by one."""
    inst = batched_instance(seed=4)
    say(f"case batched full instance: {len(inst)} arrays, "
        f"{sum(m['shape'][0] * m['shape'][1] for m in inst) / 1e6:.1f} M elements per array set")
    rt, orc = hd.Runtime(), O.Oracle(simulate_devices=False)
    ga = prog.batched_arrays(rt, inst)
    oa = prog.batched_arrays(orc, inst)
    b0, b1 = _record(rt, ga, True), _record(rt, ga, False)
    for step in range(2):
        even = step % 2 == 0
        assert rt.L.hdarray_batch_run(b0 if even else b1) == 0
        tables, packs = _oracle_step(orc, oa, even)
        _check_tables(rt.messages(), tables)
        assert np.array_equal(rt.pack(), np.concatenate(packs))
        say(f"  step {step}: {sum(len(t) for t in tables)} messages, tables and pack equal")
    for (gA, gB, gp, _), (oA, oB, op, _) in zip(ga, oa):
        assert np.array_equal(rt.read(gA, gp), orc.read(oA, op))
        assert np.array_equal(rt.read(gB, gp), orc.read(oB, op))
        _same_gdef(rt, orc, [(gA, oA), (gB, oB)], "after two steps")
    rt.close()
    orc.close()
