"""Differentiable K-step rollout of the PIC step (torch.autograd.Function).

The loss is the total field energy U_E + U_B after K steps (FP64, from the
library's diagnostics); the parameters are a per-cell source added to E_y at
step 0 and the initial momenta u^{-1/2} of one species.  Forward runs K steps
with the unfused pair (gather + push, deposit) and the Yee update, so the
particle order never changes, and keeps a checkpoint every N steps.  Backward
replays each segment from its checkpoint, keeping the state before every
step, and walks it back with the library's hand-written adjoint
(pic_energy_adjoint once, then per step pic_yee_adjoint and
pic_particle_adjoint).  Torch only provides device memory and copies.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L
from .sim import Simulation, _ptr, _stream


def _fields_struct(E, B, J) -> L.Fields:
    f = L.Fields()
    f.E = L._c3p(*[_ptr(t) for t in E])
    f.B = L._c3p(*[_ptr(t) for t in B])
    f.J = L._c3p(*[_ptr(t) for t in J])
    return f


def _species_struct(q, m, npart, cell, off, u, w) -> L.Species:
    s = L.Species()
    s.np = npart
    s.q = q
    s.m = m
    s.cell = _ptr(cell)
    s.off = L._c3p(*[_ptr(t) for t in off])
    s.u = L._c3p(*[_ptr(t) for t in u])
    s.w = _ptr(w)
    return s


class Rollout:
    """A periodic box with one species whose initial positions and weights are
    fixed; `loss(ey_src, u0)` is differentiable in both arguments.

    ey_src: (N,) tensor, N = n[0]*n[1]*n[2], added to E_y at step 0.
    u0: (3, np) tensor of initial momenta u^{-1/2}.
    """

    def __init__(self, dims, n, dx, dt, order, precision, species: dict, steps: int, checkpoint_every: int,
                 device="cuda"):
        # the rollout never sorts (particle order must match between forward and
        # backward), so the tile shape only has to be valid
        tile = tuple(next(t for t in (8, 4, 2, 1) if n[d] % t == 0) if d < dims else 1 for d in range(3))
        self.sim = Simulation(dims, n, dx, dt, order, precision, tile=tile, slack=0, sort_every=1 << 30,
                              max_particles=species["w"].shape[0], device=device)
        self.steps = int(steps)
        self.every = int(checkpoint_every)
        self.h = self.sim.add_species(species)
        cur = self.h.current()
        self.npart = self.h.np
        self.cell0 = cur["cell"][:self.npart].clone()
        self.off0 = [t[:self.npart].clone() for t in cur["off"]]
        self.w = cur["w"][:self.npart].clone()
        self.q, self.m = self.h.q, self.h.m
        self.dtype = self.sim.dtype
        self.dims = dims

    # ---- plumbing
    def _set_state(self, cell, off, u, E, B):
        cur = self.h.current()
        n = self.npart
        cur["cell"][:n].copy_(cell)
        for d in range(3):
            cur["off"][d][:n].copy_(off[d])
            cur["u"][d][:n].copy_(u[d])
        cur["w"][:n].copy_(self.w)
        for d in range(3):
            self.sim.fields["E"][d].copy_(E[d])
            self.sim.fields["B"][d].copy_(B[d])

    def _get_state(self):
        cur = self.h.current()
        n = self.npart
        return (cur["cell"][:n].clone(), [t[:n].clone() for t in cur["off"]], [t[:n].clone() for t in cur["u"]],
                [t.clone() for t in self.sim.fields["E"]], [t.clone() for t in self.sim.fields["B"]])

    def _step(self):
        s = self.sim
        s.zero_current()
        s.gather_push(self.h)
        s.deposit(self.h)
        s.yee_step()

    def _energy(self) -> float:
        d = self.sim.diagnostics([self.h])
        return d["UE"] + d["UB"]

    # ---- the differentiable map
    def forward(self, ey_src: torch.Tensor, u0: torch.Tensor):
        s = self.sim
        zeros = [torch.zeros(s.ncells, dtype=self.dtype, device=s.device) for _ in range(3)]
        E = [zeros[0], ey_src.detach().to(self.dtype).contiguous(), zeros[2]]
        B = [torch.zeros_like(zeros[0]) for _ in range(3)]
        u = [u0[d].detach().to(self.dtype).contiguous() for d in range(3)]
        self._set_state(self.cell0, self.off0, u, E, B)
        self.checkpoints = []
        for k in range(self.steps):
            if k % self.every == 0:
                self.checkpoints.append((k, self._get_state()))
            self._step()
        s.check()
        self.final_fields = ([t.clone() for t in s.fields["E"]], [t.clone() for t in s.fields["B"]])
        return self._energy()

    def backward(self, grad_loss: float):
        s = self.sim
        lib = s.lib
        st = ctypes.c_void_p(_stream())
        dev, dt = s.device, self.dtype
        lam = {k: [torch.zeros(s.ncells, dtype=dt, device=dev) for _ in range(3)] for k in ("E", "B", "J")}
        lam_f = _fields_struct(lam["E"], lam["B"], lam["J"])
        fin = _fields_struct(self.final_fields[0], self.final_fields[1], lam["J"])
        s._call(lib.pic_energy_adjoint(s.ctx, ctypes.byref(fin), ctypes.byref(lam_f), float(grad_loss), st),
                "pic_energy_adjoint")
        lx = [torch.zeros(self.npart, dtype=dt, device=dev) for _ in range(3)]
        lu = [torch.zeros(self.npart, dtype=dt, device=dev) for _ in range(3)]
        lsp = L.SpeciesAdjoint()
        lsp.x = L._c3p(*[_ptr(t) for t in lx])
        lsp.u = L._c3p(*[_ptr(t) for t in lu])
        scratch_j = [torch.zeros(s.ncells, dtype=dt, device=dev) for _ in range(3)]
        for seg in reversed(range(len(self.checkpoints))):
            k0, state = self.checkpoints[seg]
            k1 = self.checkpoints[seg + 1][0] if seg + 1 < len(self.checkpoints) else self.steps
            self._set_state(*state)
            saved = []
            for _ in range(k0, k1):
                saved.append(self._get_state())
                self._step()
            for cell, off, u, E, B in reversed(saved):
                s._call(lib.pic_yee_adjoint(s.ctx, ctypes.byref(lam_f), st), "pic_yee_adjoint")
                spn = _species_struct(self.q, self.m, self.npart, cell, off, u, self.w)
                fn = _fields_struct(E, B, scratch_j)
                s._call(lib.pic_particle_adjoint(s.ctx, ctypes.byref(spn), ctypes.byref(fn), ctypes.byref(lam_f),
                                                 ctypes.byref(lsp), st), "pic_particle_adjoint")
        s.check()
        return lam["E"][1].clone(), torch.stack(lu)


class _RolloutFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, ey_src, u0, roll):
        ctx.roll = roll
        val = roll.forward(ey_src, u0)
        return torch.tensor(val, dtype=torch.float64, device=ey_src.device)

    @staticmethod
    def backward(ctx, g):
        gs, gu = ctx.roll.backward(float(g.item()))
        return gs.to(torch.float64), gu.to(torch.float64), None


def rollout_loss(roll: Rollout, ey_src: torch.Tensor, u0: torch.Tensor) -> torch.Tensor:
    """Total field energy after the rollout; differentiable in ey_src and u0."""
    return _RolloutFn.apply(ey_src, u0, roll)
