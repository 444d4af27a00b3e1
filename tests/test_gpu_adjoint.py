"""Differentiation through ApplyKernel steps (7-point stencil, 2 x 2 x 2
blocks, T = 64, checkpoints every 8) on a 32^3 copy of the stencil3d
workload: the forward is bit-exact against the FP32 oracle; the gradient
w.r.t. u0 and the 7 coefficients agrees with the FP64 CPU adjoint and with
FP64 finite differences to <= 1e-4 relative; recomputed checkpoint segments
are bit-exact; the reverse halo exchange uses exactly the use-region
messages of the cotangent array."""
import sys

import numpy as np
import pytest

import oracle as O
from workloads import programs as prog
from workloads import S3D_COEFFS, stencil3d_inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_1809_05657_amd as hdm
    from paper_1809_05657_amd import autograd as ag

    assert torch.cuda.is_available()
    hdm.load()
    return hdm, ag, torch


def _fp32_oracle_forward(u0, T, coef):
    o = O.Oracle(simulate_devices=False)
    U, V, p = prog.stencil3d(o, u0, 8)
    for t in range(T):
        if t % 2 == 0:
            o.apply("s3dUV", p, [U, V], coef)
        else:
            o.apply("s3dVU", p, [V, U], coef)
    return o.read(V if T % 2 == 0 else U, p)


def test_adjoint_matches_fp64_and_fd(env):
    hdm, ag, torch = env
    n, T, ck = 32, 64, 8
    say(f"case adjoint stencil3d {n}^3 T={T} ckpt={ck}")
    u0, w = stencil3d_inputs(n)
    coef = [float(c) for c in S3D_COEFFS]
    rt = hdm.Runtime()
    solver = ag.Stencil3D(rt, (n, n, n), ndev=8, T=T, ckpt=ck)
    dev = torch.device("cuda:0")
    u0_t = torch.from_numpy(u0).to(dev)
    uT = solver.forward(u0_t, coef).cpu().numpy()
    # forward: bit-exact against the FP32 oracle (same operation order)
    assert np.array_equal(uT, _fp32_oracle_forward(u0, T, coef))
    c64 = np.array(S3D_COEFFS, dtype=np.float64)
    uT64 = O.s3d_forward64(u0.astype(np.float64), c64, T)
    say(f"forward fp32 vs fp64: max abs {np.max(np.abs(uT - uT64)):.3e}")
    g0, cb = solver.backward(torch.from_numpy(w).to(dev))
    g0 = g0.cpu().numpy().astype(np.float64)
    cb = cb.cpu().numpy()
    g64, gc64 = O.s3d_adjoint64(u0.astype(np.float64), c64, T, w.astype(np.float64))
    rel = np.linalg.norm(g0 - g64) / np.linalg.norm(g64)
    relc = np.abs(cb - gc64) / np.abs(gc64)
    say(f"adjoint vs fp64 adjoint: rel L2 {rel:.3e}, coefficient rel {relc.max():.3e}")
    assert rel <= 1e-4
    assert np.all(relc <= 1e-4)
    # FP64 central differences: L is linear in u0, so they are exact
    rng = np.random.default_rng(55)

    def loss(u, cc):
        return float(np.sum(w.astype(np.float64) * O.s3d_forward64(u, cc, T)))

    for _ in range(2):
        v = rng.standard_normal(u0.shape)
        fd = (loss(u0 + v, c64) - loss(u0 - v, c64)) / 2
        assert abs(fd - np.sum(g0 * v)) <= 1e-4 * abs(fd)
    h = 1e-6
    for e in range(7):
        cp, cm = c64.copy(), c64.copy()
        cp[e] += h
        cm[e] -= h
        fd = (loss(u0.astype(np.float64), cp) - loss(u0.astype(np.float64), cm)) / (2 * h)
        assert abs(fd - cb[e]) <= 1e-4 * abs(fd), (e, fd, cb[e])
    # recomputed segments equal the stored checkpoints bit for bit
    for s in range(T // ck - 1):
        solver._segment(s)
        a = rt.read(solver.S[ck], solver.part)
        b = rt.read(solver.Ck[s + 1], solver.part)
        assert np.array_equal(a, b)


def test_autograd_function_and_dot_product(env):
    hdm, ag, torch = env
    n = 20
    say(f"case autograd {n}^3 T=8 ckpt=4 and FP32 dot-product test")
    u0, w = stencil3d_inputs(n, seed=7)
    rt = hdm.Runtime()
    solver = ag.Stencil3D(rt, (n, n, n), ndev=8, T=8, ckpt=4)
    dev = torch.device("cuda:0")
    u = torch.from_numpy(u0).to(dev).requires_grad_(True)
    c = torch.tensor(S3D_COEFFS, device=dev, requires_grad=True)
    out = ag.stencil3d(u, c, solver)
    loss = (out.double() * torch.from_numpy(w).to(dev).double()).sum()
    loss.backward()
    g64, gc64 = O.s3d_adjoint64(u0.astype(np.float64), np.array(S3D_COEFFS, np.float64), 8, w.astype(np.float64))
    g = u.grad.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(g - g64) / np.linalg.norm(g64) <= 1e-4
    assert np.all(np.abs(c.grad.cpu().numpy() - gc64) <= 1e-4 * np.abs(gc64))
    # one step: <S v, w> = <v, S^T w> in FP32 within 1e-5
    s1 = ag.Stencil3D(rt, (n, n, n), ndev=8, T=1, ckpt=1)
    v = np.random.default_rng(3).random((n, n, n), dtype=np.float32)
    sv = s1.forward(torch.from_numpy(v).to(dev), list(S3D_COEFFS)).cpu().numpy().astype(np.float64)
    stw, _ = s1.backward(torch.from_numpy(w).to(dev))
    lhs = float(np.sum(sv * w))
    rhs = float(np.sum(v.astype(np.float64) * stw.cpu().numpy()))
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


def test_reverse_messages_parity(env):
    """The reverse exchange of one adjoint step uses the use-region messages
    of the cotangent array (owner -> user), which the oracle derives for an
    array held only by its owners."""
    hdm, ag, torch = env
    shape = (12, 13, 30)
    say(f"case reverse messages {shape}")
    rng = np.random.default_rng(8)
    u0 = rng.random(shape, dtype=np.float32)
    rt = hdm.Runtime()
    gU, gV, gp = prog.stencil3d(rt, u0, 8)
    G0, G1 = rt.create(shape=shape), rt.create(shape=shape)
    rt.write(G0, np.zeros(shape, np.float32), gp)
    rt.write(G1, rng.random(shape, dtype=np.float32), gp)
    rt.apply("s3dUV", gp, [gU, gV], [float(x) for x in S3D_COEFFS])
    rt.apply_adjoint("s3dUV", gp, G0, G1, gV, [float(x) for x in S3D_COEFFS])
    mg = rt.messages()
    o = O.Oracle(simulate_devices=False, eval_kernels=False)
    oU, oV, op = prog.stencil3d(o, u0, 8)
    oG0, oG1 = o.create(shape=shape), o.create(shape=shape)
    o.write(oG0, np.zeros(shape, np.float32), op)
    o.kernel("use", prog.K_STENCIL3D7)
    o.set_offsets("use", 1, 0, prog.S3D_OFFSETS)
    o.apply("use", op, [oG1, oG0], [float(x) for x in S3D_COEFFS])
    mo = o.messages()
    assert len(mg) == len(mo) > 0
    cols = [2, 3, 4, 5, 6, 7, 8, 9, 10, 11]
    assert np.array_equal(mg[:, cols], mo[:, cols])


@pytest.mark.parametrize("shape", [(6, 6, 512), (5, 7, 600), (9, 33, 70)])
def test_adjoint_wide_rows(env, shape):
    """Boxes 256 columns wide (the extended column right of the box falls
    just past the last column tile), wider than one tile, and narrow boxes
    with unaligned starts: gradient and coefficient gradients against the
    FP64 CPU adjoint."""
    hdm, ag, torch = env
    T, ck = 4, 2
    say(f"case adjoint wide rows {shape} T={T}")
    rng = np.random.default_rng(sum(shape))
    u0 = rng.random(shape, dtype=np.float32)
    w = rng.random(shape, dtype=np.float32)
    coef = [float(c) for c in S3D_COEFFS]
    rt = hdm.Runtime()
    solver = ag.Stencil3D(rt, shape, ndev=8, T=T, ckpt=ck)
    dev = torch.device("cuda:0")
    solver.forward(torch.from_numpy(u0).to(dev), coef)
    g0, cb = solver.backward(torch.from_numpy(w).to(dev))
    g0 = g0.cpu().numpy().astype(np.float64)
    cb = cb.cpu().numpy()
    c64 = np.array(S3D_COEFFS, dtype=np.float64)
    g64, gc64 = O.s3d_adjoint64(u0.astype(np.float64), c64, T, w.astype(np.float64))
    assert np.linalg.norm(g0 - g64) / np.linalg.norm(g64) <= 1e-4
    assert np.all(np.abs(cb - gc64) <= 1e-4 * np.abs(gc64))


def test_plan_cache_pass_bit_identical(env):
    """A checkpointed forward + adjoint pass with the plan cache on (Sec.
    4.2: the forward and recomputation calls skip their derivation when the
    history decides) gives the same gradient and coefficient gradients, bit
    for bit, as the pass that derives every call."""
    hdm, ag, torch = env
    n = 20
    say(f"case plan cache pass {n}^3 T=8 ckpt=4")
    u0, w = stencil3d_inputs(n, seed=9)
    dev = torch.device("cuda:0")
    out = []
    for cache in (False, True):
        rt = hdm.Runtime()
        rt.set_plan_cache(cache)
        solver = ag.Stencil3D(rt, (n, n, n), ndev=8, T=8, ckpt=4)
        uT = solver.forward(torch.from_numpy(u0).to(dev), list(S3D_COEFFS)).cpu().numpy()
        g, cb = solver.backward(torch.from_numpy(w).to(dev))
        g, cb = g.cpu().numpy(), cb.cpu().numpy()
        # a second pass on the same solver (the cache now holds its plans)
        uT2 = solver.forward(torch.from_numpy(u0).to(dev), list(S3D_COEFFS)).cpu().numpy()
        g2, cb2 = solver.backward(torch.from_numpy(w).to(dev))
        out.append((uT, g, cb, uT2, g2.cpu().numpy(), cb2.cpu().numpy(), rt.stats()))
        rt.close()
    for a, b in zip(out[0][:6], out[1][:6]):
        assert np.array_equal(a, b)
    assert out[1][6]["cache_hits"] > 0
