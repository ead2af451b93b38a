"""Reverse-mode differentiation of the forward simulation through the adjoint
state method (the paper's gradient method, section 3), as a torch op.

    data = fwi_forward(vel, op)          # [np][ns][nt][nr], differentiable in vel
    loss = f(data); loss.backward()      # vel.grad via one adjoint sweep

forward runs vip_forward_tape, which stores the wavefield state every
`ckpt_every` steps in a tape owned by the operator; backward runs
vip_adjoint_tape, which recomputes each segment from its checkpoint and
propagates grad_data backwards with the exact discrete adjoint of the scheme.
Memory: the tape holds 2 N floats per checkpoint per (particle, shot) pair
instead of the nt N floats of the whole history.
"""
from __future__ import annotations

import torch

from . import binding as vb


class FwiOperator:
    """Grid, acquisition and checkpoint interval of a differentiable forward."""

    def __init__(self, ctx: vb.Context, grid: vb.Grid, geom: vb.Geometry, ckpt_every: int = 50):
        self.ctx, self.grid, self.geom, self.ckpt_every = ctx, grid, geom, int(ckpt_every)
        self._tape = None
        self._ws = None

    def buffers(self, npart: int):
        tape_bytes, ws_bytes = vb.tape_sizes(self.grid, self.geom, npart, self.ckpt_every)
        if self._tape is None or self._tape.numel() < tape_bytes:
            self._tape = torch.empty(max(tape_bytes, 256), dtype=torch.uint8, device=self.ctx.device)
        if self._ws is None or self._ws.numel() < ws_bytes:
            self._ws = torch.zeros(max(ws_bytes, 256), dtype=torch.uint8, device=self.ctx.device)
        return self._tape, self._ws


class _VipFwi(torch.autograd.Function):
    @staticmethod
    def forward(fctx, vel: torch.Tensor, op: FwiOperator):
        vel = vel.contiguous()
        tape, ws = op.buffers(vel.shape[0])
        data = vb.vip_forward_tape(op.ctx, op.grid, op.geom, vel, op.ckpt_every, tape, ws)
        fctx.save_for_backward(vel)
        fctx.op = op
        return data

    @staticmethod
    def backward(fctx, grad_data: torch.Tensor):
        (vel,) = fctx.saved_tensors
        op = fctx.op
        tape, ws = op.buffers(vel.shape[0])
        grad_vel = vb.vip_adjoint_tape(op.ctx, op.grid, op.geom, vel, op.ckpt_every, tape,
                                       grad_data.contiguous().to(torch.float32), ws)
        return grad_vel, None


def fwi_forward(vel: torch.Tensor, op: FwiOperator) -> torch.Tensor:
    """Receiver data of every (particle, shot) pair; differentiable in vel.

    The operator's tape is overwritten by each call, so call backward before
    the next forward through the same operator."""
    return _VipFwi.apply(vel, op)
