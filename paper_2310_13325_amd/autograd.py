"""Reverse-mode differentiation of the forward simulation through the adjoint
state method (the paper's gradient method, section 3), as a torch op.

    data = fwi_forward(vel, op)          # [np][ns][nt][nr], differentiable in vel
    loss = f(data); loss.backward()      # vel.grad via one adjoint sweep

forward runs vip_forward_tape, which stores the wavefield state every
`ckpt_every` steps in a tape of its own (kept by the autograd graph until it
is freed); backward runs vip_adjoint_tape, which recomputes each segment from
its checkpoint and propagates grad_data backwards with the exact discrete
adjoint of the scheme.  Memory: a tape holds 2 N floats per checkpoint per
(particle, shot) pair instead of the nt N floats of the whole history.
"""
from __future__ import annotations

import torch

from . import binding as vb


class FwiOperator:
    """Grid, acquisition and checkpoint interval of a differentiable forward."""

    def __init__(self, ctx: vb.Context, grid: vb.Grid, geom: vb.Geometry, ckpt_every: int = 50):
        self.ctx, self.grid, self.geom, self.ckpt_every = ctx, grid, geom, int(ckpt_every)
        self._ws = None

    def workspace(self, npart: int) -> torch.Tensor:
        """Scratch shared by every call through this operator (stream-ordered;
        nothing in it outlives a call)."""
        _, ws_bytes = vb.tape_sizes(self.grid, self.geom, npart, self.ckpt_every)
        if self._ws is None or self._ws.numel() < ws_bytes:
            self._ws = torch.zeros(max(ws_bytes, 256), dtype=torch.uint8, device=self.ctx.device)
        return self._ws

    def new_tape(self, npart: int) -> torch.Tensor:
        tape_bytes, _ = vb.tape_sizes(self.grid, self.geom, npart, self.ckpt_every)
        return torch.empty(max(tape_bytes, 256), dtype=torch.uint8, device=self.ctx.device)


class _VipFwi(torch.autograd.Function):
    @staticmethod
    def forward(fctx, vel: torch.Tensor, op: FwiOperator):
        vel = vel.contiguous()
        tape = op.new_tape(vel.shape[0])
        data = vb.vip_forward_tape(op.ctx, op.grid, op.geom, vel, op.ckpt_every, tape,
                                   op.workspace(vel.shape[0]))
        fctx.save_for_backward(vel)
        fctx.op = op
        fctx.tape = tape   # this forward's checkpoints, alive as long as its graph
        return data

    @staticmethod
    def backward(fctx, grad_data: torch.Tensor):
        (vel,) = fctx.saved_tensors
        op = fctx.op
        grad_vel = vb.vip_adjoint_tape(op.ctx, op.grid, op.geom, vel, op.ckpt_every, fctx.tape,
                                       grad_data.contiguous().to(torch.float32),
                                       op.workspace(vel.shape[0]))
        return grad_vel, None


def fwi_forward(vel: torch.Tensor, op: FwiOperator) -> torch.Tensor:
    """Receiver data of every (particle, shot) pair; differentiable in vel.

    Each call records its own tape, so several forwards may precede their
    backwards (two calls in one loss, gradcheck's perturbed forwards)."""
    return _VipFwi.apply(vel, op)
