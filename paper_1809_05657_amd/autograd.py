"""Differentiable 7-point stencil time stepping through the HDArray runtime.

``Stencil3D(rt, shape, ndev, T, ckpt)`` holds the HDArrays of a
checkpointed run of T ApplyKernel steps (7-point stencil, BLOCK partition,
use = own block +-1 along each axis, def = own block).  ``apply(u0, coef)``
is a ``torch.autograd.Function``: the forward runs the T steps and keeps a
checkpoint every ``ckpt`` steps; the backward recomputes each segment from
its checkpoint (the recomputed halos are exactly the ones the forward
exchanged) and runs the adjoint steps in reverse, whose reverse halo
exchange adds the cotangents of halo cells to their owners
(``hdarray_apply_adjoint``).  Every step runs in the library's kernels; this
module only orders the calls and moves tensors in and out through device
pointers.
"""
import torch

from . import BLOCK, K_COPY, K_STENCIL3D7

S3D_OFFSETS = [(0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]


def check_field(t, shape, what):
    """The library reads and writes fields through raw device pointers as
    dense fp32 of the solver's shape: anything else (a host tensor, another
    dtype or shape) is refused here, before any pointer reaches the GPU."""
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{what}: expected a torch.Tensor, got {type(t).__name__}")
    if t.dtype != torch.float32:
        raise ValueError(f"{what}: expected float32, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what}: expected shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_cuda:
        raise ValueError(f"{what}: expected a GPU tensor, got one on {t.device}")
    return t.contiguous()


class Stencil3D:
    def __init__(self, rt, shape, ndev=8, T=64, ckpt=8):
        assert T % ckpt == 0
        self.rt, self.shape, self.T, self.ckpt = rt, tuple(shape), T, ckpt
        self.part = rt.partition(BLOCK, self.shape, ndev=ndev)
        mk = lambda nm: rt.create(shape=self.shape, name=nm)
        self.S = [mk(f"seg{k}") for k in range(ckpt + 1)]      # states of one segment
        self.Ck = [mk(f"ckpt{k}") for k in range(T // ckpt)]  # u_0, u_ckpt, ...
        self.G = [mk("gA"), mk("gB")]                          # cotangents (ping-pong)
        if "s3d" not in rt.kernels:
            rt.kernel("s3d", K_STENCIL3D7)
            rt.set_offsets("s3d", 1, 0, S3D_OFFSETS)
            rt.set_offsets("s3d", 0, 1, [(0, 0, 0)])
            rt.kernel("s3dcp", K_COPY)
            rt.set_offsets("s3dcp", 1, 0, [(0, 0, 0)])
            rt.set_offsets("s3dcp", 0, 1, [(0, 0, 0)])
        self.coef = None

    def _segment(self, s):
        """S[0] <- checkpoint s, then ckpt steps S[k+1] = S(S[k])."""
        rt, p = self.rt, self.part
        rt.apply("s3dcp", p, [self.S[0], self.Ck[s]])
        for k in range(self.ckpt):
            rt.apply("s3d", p, [self.S[k + 1], self.S[k]], self.coef)

    def forward(self, u0, coef):
        rt, p = self.rt, self.part
        u0 = check_field(u0, self.shape, "u0")
        self.coef = [float(c) for c in coef]
        if len(self.coef) != 7:
            raise ValueError(f"coef: expected 7 weights, got {len(self.coef)}")
        rt.write_device(self.S[0], u0.data_ptr(), p)
        for s in range(self.T // self.ckpt):
            rt.apply("s3dcp", p, [self.Ck[s], self.S[0]])
            for k in range(self.ckpt):
                rt.apply("s3d", p, [self.S[k + 1], self.S[k]], self.coef)
            if s + 1 < self.T // self.ckpt:
                rt.apply("s3dcp", p, [self.S[0], self.S[self.ckpt]])
        out = torch.empty_like(u0)
        rt.read_device(self.S[self.ckpt], out.data_ptr(), p)
        rt.sync()
        return out

    def backward(self, gT):
        rt, p = self.rt, self.part
        gT = check_field(gT, self.shape, "grad of u_T")
        cbar = torch.zeros(8, dtype=torch.float64, device=gT.device)
        rt.write_device(self.G[0], gT.data_ptr(), p)
        cur = 0
        for s in reversed(range(self.T // self.ckpt)):
            self._segment(s)
            for k in reversed(range(self.ckpt)):
                rt.apply_adjoint("s3d", p, self.G[1 - cur], self.G[cur], self.S[k], self.coef, cbar.data_ptr())
                cur = 1 - cur
        g0 = torch.empty_like(gT)
        rt.read_device(self.G[cur], g0.data_ptr(), p)
        rt.sync()
        return g0, cbar[:7].clone()


class _Fn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, coef, solver):
        ctx.solver = solver
        return solver.forward(u0, coef.detach().cpu().tolist())

    @staticmethod
    def backward(ctx, gout):
        g0, gc = ctx.solver.backward(gout)
        return g0, gc.to(torch.float32), None


def stencil3d(u0, coef, solver):
    """u_T of T stencil steps from u0 (differentiable w.r.t. u0 and coef)."""
    return _Fn.apply(u0, coef, solver)
