"""Differentiable rollout of the PIC step with the hand-written adjoint.

``PicRollout`` is a ``torch.autograd.Function`` whose forward advances
``steps`` full steps (push/deposit then field advance, HIP kernels of
libpic) from initial fields ``a0 * (E_unit, B_unit)`` and initial momenta
``u0``, and returns the final fields.  Its backward runs the transposes of the
two kernels (``pic_field_advance_adjoint``, ``pic_push_deposit_adjoint``)
step by step in reverse.  Memory is bounded by checkpointing: the forward
keeps the full state every ``checkpoint_every`` steps, the backward recomputes
each segment from its checkpoint, keeps that segment's per-step states and
walks back through them.

Particles are sorted by tile once, before the first step (later drift takes
the kernels' global-memory path), so every stored state and every adjoint
array shares one particle order; gradients are returned in the caller's
order through the permutation the sort applied to the ids.
"""
from __future__ import annotations

import numpy as np
import torch

from . import pic as P


class Runner:
    """Owns one context, the device state and the checkpoints of a rollout."""

    def __init__(self, w, real_bytes=4, steps=None, checkpoint_every=10, device="cuda"):
        self.w = w
        self.steps = w.steps if steps is None else steps
        self.every = checkpoint_every
        self.sim = P.Simulation(w.dims, w.n3, w.dx3, w.dt, w.order, real_bytes, w.bc3,
                                sort_every=1 << 30, q_const=w.q_const, device=device)
        self.real = self.sim.real
        self.device = self.sim.device

    def set_inputs(self, plasma, E_unit, B_unit):
        """Positions and charges of the plasma; fields per unit a0."""
        self.plasma = plasma
        self.sim.load(plasma, E_unit, B_unit, with_id=True)
        self.E_unit = self.sim.E.clone()
        self.B_unit = self.sim.B.clone()
        self.cell0 = self.sim.cell.clone()
        self.off0 = self.sim.off.clone()
        self.q0 = None if self.sim.q is None else self.sim.q.clone()
        self.id0 = self.sim.id.clone()

    # ---- state helpers
    def _state(self):
        s = self.sim
        return (s.cell.clone(), s.off.clone(), s.u.clone(), s.E.clone(), s.B.clone())

    def _restore(self, st):
        s = self.sim
        s.cell.copy_(st[0])
        s.off.copy_(st[1])
        s.u.copy_(st[2])
        s.E.copy_(st[3])
        s.B.copy_(st[4])

    def _step(self):
        self.sim.push_deposit()
        self.sim.field_advance()

    def forward(self, a0: torch.Tensor, u0: torch.Tensor):
        s = self.sim
        s.cell.copy_(self.cell0)
        s.off.copy_(self.off0)
        if self.q0 is not None:
            s.q.copy_(self.q0)
        s.id.copy_(self.id0)
        s.u.copy_(u0.to(self.real))
        a = a0.to(self.real)
        s.E.copy_(a * self.E_unit)
        s.B.copy_(a * self.B_unit)
        s.sort()  # once; fixes the particle order for the whole rollout
        self.perm = s.id[: s.np].long().clone()  # slot -> caller index (live particles)
        self.checkpoints = {}
        for n in range(self.steps):
            if n % self.every == 0:
                self.checkpoints[n] = self._state()
            self._step()
        return s.E.clone(), s.B.clone()

    def backward(self, gE: torch.Tensor, gB: torch.Tensor):
        s = self.sim
        lamE = gE.to(self.real).contiguous().clone()
        lamB = gB.to(self.real).contiguous().clone()
        lamJ = torch.zeros_like(lamE)
        lamX = torch.zeros_like(s.off)
        lamU = torch.zeros_like(s.u)
        lf = P.fields_struct(lamE, lamB, lamJ)
        lp = P.particles_struct(s.np, None, lamX, lamU)
        ws = s.ws.data_ptr()
        starts = sorted(self.checkpoints)
        for k, n0 in reversed(list(enumerate(starts))):
            n1 = starts[k + 1] if k + 1 < len(starts) else self.steps
            # recompute the segment, keeping each step's input state
            self._restore(self.checkpoints[n0])
            states = []
            for n in range(n0, n1):
                states.append(self._state())
                self._step()
            for n in reversed(range(n0, n1)):
                cell, off, u, E, B = states[n - n0]
                parts = P.particles_struct(s.np, cell, off, u, s.q)
                fields = P.fields_struct(E, B)
                P.pic_field_advance_adjoint(s.ctx, lf, ws, s.stream)
                P.pic_push_deposit_adjoint(s.ctx, parts, fields, lf, lp, ws, s.stream)
            del states
        g_a0 = (lamE * self.E_unit).sum(dtype=torch.float64) + (lamB * self.B_unit).sum(dtype=torch.float64)
        g_u0 = torch.zeros_like(lamU)
        g_u0[:, self.perm] = lamU[:, : s.np]
        return g_a0, g_u0


class PicRollout(torch.autograd.Function):
    """(a0, u0) -> (E^N, B^N) through the HIP step; backward = hand-written adjoint."""

    @staticmethod
    def forward(ctx, a0, u0, runner):
        ctx.runner = runner
        E, B = runner.forward(a0, u0)
        return E, B

    @staticmethod
    def backward(ctx, gE, gB):
        g_a0, g_u0 = ctx.runner.backward(gE, gB)
        return g_a0.to(torch.float64).reshape(()), g_u0, None


def window_energy(w, E, window=64):
    """L = 1/2 sum (E_x)^2 dV over the x-window of `window` cells that ends at
    the laser pulse's centre at the final time (full transverse extent)."""
    shape = (w.n3[2], w.n3[1], w.n3[0])
    Ex = E[0].reshape(shape).to(torch.float64)
    L = w.laser
    t_end = w.steps * w.dt
    ic = int(np.floor((L.x_center + t_end) / w.dx[0]))
    lo = max(ic - window, 0)
    dV = float(np.prod(w.dx[: w.dims]))
    return 0.5 * dV * (Ex[:, :, lo:ic] ** 2).sum(), (lo, ic)
