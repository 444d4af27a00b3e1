"""Batched step (one persistent, graph-replayed launch for many independent
ApplyKernel calls) against the oracle running the same calls one by one:
every array, its GDEF map and the per-call message tables bit-exact, for
every step, before and after the tile-shape autotuner."""
import sys

import numpy as np
import pytest

import oracle as O
from workloads import programs as prog
from workloads import batched_instance

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def hd():
    import paper_1809_05657_amd as hdm
    import torch

    assert torch.cuda.is_available()
    hdm.load()
    return hdm


def _record(rt, arrs, even):
    rt.L.hdarray_batch_begin()
    for i, (A, B, p, kind) in enumerate(arrs):
        if even:
            rt.apply(f"b{i}AB", p, [A, B])
        else:
            rt.apply(f"b{i}BA", p, [B, A])
    bid = rt.L.hdarray_batch_end()
    assert bid >= 0, bid
    return bid


def _oracle_step(orc, arrs, even):
    tables, packs = [], []
    for i, (A, B, p, kind) in enumerate(arrs):
        if even:
            orc.apply(f"b{i}AB", p, [A, B])
        else:
            orc.apply(f"b{i}BA", p, [B, A])
        tables.append(orc.messages())
        packs.append(orc.pack())
    return tables, packs


def _check_tables(gpu_tab, tables):
    """The batch table is the calls' tables in call order; offsets run on."""
    want = np.concatenate([t for t in tables if len(t)]) if any(len(t) for t in tables) else np.zeros((0, 12))
    assert gpu_tab.shape[0] == want.shape[0]
    if not len(want):
        return
    cols = [0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 11]
    assert np.array_equal(gpu_tab[:, cols], want[:, cols])
    ends = np.cumsum(gpu_tab[:, 11])
    assert np.array_equal(gpu_tab[1:, 10], ends[:-1]) and gpu_tab[0, 10] == 0


@pytest.mark.parametrize("scale,narr", [(0.04, 64), (0.1, 16)])
def test_batched_matches_oracle(hd, scale, narr):
    inst = batched_instance(seed=4, narrays=narr, scale=scale)
    say(f"case batched scale={scale} arrays={narr} sides={[m['shape'] for m in inst[:4]]}...")
    rt, orc = hd.Runtime(), O.Oracle()
    ga = prog.batched_arrays(rt, inst)
    oa = prog.batched_arrays(orc, inst)
    b0, b1 = _record(rt, ga, True), _record(rt, ga, False)
    for step in range(6):
        if step == 2:
            ids = (b0, b1)
            import ctypes
            arr = (ctypes.c_int * 2)(*ids)
            cfg = rt.L.hdarray_batch_autotune(arr, 2, 1)
            assert cfg > 0
            say(f"autotuned rows={(cfg >> 8) & 255} shape={cfg & 255} per_cu={cfg >> 16}")
            # the autotuner ran 21 candidates x (1 + reps) real pairs of steps
            for _ in range(42):
                _oracle_step(orc, oa, True)
                _oracle_step(orc, oa, False)
        even = step % 2 == 0
        rc = rt.L.hdarray_batch_run(b0 if even else b1)
        assert rc == 0
        tables, packs = _oracle_step(orc, oa, even)
        _check_tables(rt.messages(), tables)
        assert np.array_equal(rt.pack(), np.concatenate(packs))
    for (gA, gB, gp, _), (oA, oB, op, _) in zip(ga, oa):
        assert np.array_equal(rt.read(gA, gp), orc.read(oA, op))
        assert np.array_equal(rt.read(gB, gp), orc.read(oB, op))
        og, hg = rt.gdef(gB)
        oo, ho = orc.gdef(oB)
        assert np.array_equal(og, oo) and np.array_equal(hg, ho)


def _block_arrays(api, shapes, base):
    """Jacobi arrays on block partitions: a row crosses several devices, so
    its GDEF list and holder-adding runs outgrow the one-lane update and the
    batch's wave form takes it."""
    out = []
    for i, (n0, n1, nd) in enumerate(shapes):
        rng = np.random.default_rng(50 + i)
        A0 = rng.random((n0, n1), dtype=np.float32)
        B0 = rng.random((n0, n1), dtype=np.float32)
        A, B = api.create(A0), api.create(B0)
        p = api.partition(2, (n0, n1), ndev=nd)
        for k in (f"b{base + i}AB", f"b{base + i}BA"):
            api.kernel(k, prog.K_JACOBI2D)
            api.set_offsets(k, 1, 0, prog.J2D_OFFSETS)
            api.set_offsets(k, 0, 1, [(0, 0)])
        api.write(A, A0, p)
        api.write(B, B0, p)
        out.append((A, B, p, 0))
    return out


def test_batched_wide_rows(hd):
    """Block partitions (rows over 4-8 devices) beside row partitions in one
    batch: every step's tables, packs, values and GDEF against the oracle."""
    shapes = [(96, 700, 16), (130, 260, 6), (70, 2100, 8)]
    say(f"case batched wide rows {shapes}")
    rt, orc = hd.Runtime(), O.Oracle()
    inst = batched_instance(seed=4, narrays=6, scale=0.05)
    ga = prog.batched_arrays(rt, inst)
    oa = prog.batched_arrays(orc, inst)
    # kernels b<i>AB / b<i>BA, i = position in the batch
    ga += _block_arrays(rt, shapes, len(ga))
    oa += _block_arrays(orc, shapes, len(oa))
    b0, b1 = _record(rt, ga, True), _record(rt, ga, False)
    for step in range(5):
        even = step % 2 == 0
        assert rt.L.hdarray_batch_run(b0 if even else b1) == 0
        tables, packs = _oracle_step(orc, oa, even)
        _check_tables(rt.messages(), tables)
        assert np.array_equal(rt.pack(), np.concatenate(packs))
    for (gA, gB, gp, _), (oA, oB, op, _) in zip(ga, oa):
        assert np.array_equal(rt.read(gA, gp), orc.read(oA, op))
        og, hg = rt.gdef(gB)
        oo, ho = orc.gdef(oB)
        assert np.array_equal(og, oo) and np.array_equal(hg, ho)
