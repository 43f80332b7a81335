"""torch.autograd.Function over K unrolled PDHG steps (hand-written adjoint).

The forward pass runs the library's fused primal/dual kernels K times with
fixed step sizes and the scaling factors of the last configure held fixed,
storing (x, y, A~x) every ``ckpt_every`` steps.  The backward pass replays
each segment from its checkpoint with the same deterministic kernels and runs
the transposed products and the projection-mask backward in reverse, giving
dL/dc, dL/db and dL/dA.values (A's CSR order).  The subgradient of the
projection max(l, v) is taken as 1[v > l] (0 at a tie).
"""
from __future__ import annotations

import torch

from . import _lib as L


class PDHGUnroll(torch.autograd.Function):
    """x_K = PDHGUnroll.apply(c, b, a_values, solver, K, ckpt_every, tau,
    sigma, precision).  c, b, a_values are float64 tensors (host or device);
    x_K is returned on the device of c."""

    @staticmethod
    def forward(ctx, c, b, a_values, solver, K: int, ckpt_every: int,
                tau: float, sigma: float, precision: int = L.FP64):
        solver.set_values(a_values)
        solver.set_rhs_obj(b, c)
        dev = c.is_cuda
        xK, tape = solver.unrolled_forward(K, ckpt_every, tau, sigma,
                                           precision=precision, device=dev)
        ctx.tape = tape
        ctx.dev = dev
        out = xK if dev else torch.from_numpy(xK)
        return out

    @staticmethod
    def backward(ctx, gx):
        g = gx.detach().to(torch.float64).contiguous()
        if not ctx.dev:
            g = g.cpu()
        gc, gb, gA = ctx.tape.backward(g if ctx.dev else g.numpy(), device=ctx.dev)
        ctx.tape.free()
        if not ctx.dev:
            gc, gb, gA = (torch.from_numpy(t) for t in (gc, gb, gA))
        return gc, gb, gA, None, None, None, None, None, None
