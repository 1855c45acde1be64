"""Differentiable K-step rollout of the PIC step (torch.autograd.Function).

The loss is the total field energy U_E + U_B after K steps (FP64, from the
library's diagnostics); the parameters are a per-cell source added to E_y at
step 0 and the initial momenta u^{-1/2} of one species.  The species is sorted
by tile once, when the rollout is built (the permutation is recorded, and
parameters and gradients are mapped through it); forward then runs K fused
steps (pic_step with sort_every = 0, so the particle order never changes;
particles that drift out of their tile take the library's straggler path)
and keeps a checkpoint every N steps.  Backward
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
        # the fused kernel's tile shapes (16x16 in 2D, 8x8x8 / 8x8x4 in 3D) where they divide the box
        want = (16, 16, 1) if dims == 2 else ((8, 8, 8) if precision == "fp32" else (8, 8, 4))
        tile = tuple(next(t for t in (want[d], 8, 4, 2, 1) if n[d] % t == 0) if d < dims else 1 for d in range(3))
        # slack 2: the particles drift from the tiles of the one sort for the whole rollout
        self.sim = Simulation(dims, n, dx, dt, order, precision, tile=tile, slack=2, sort_every=0,
                              max_particles=species["w"].shape[0], device=device)
        self.steps = int(steps)
        self.every = int(checkpoint_every)
        npart = int(species["w"].shape[0])
        assert precision == "fp64" or npart < (1 << 24), "particle indices must be exact in the weight array"
        # sort once with each particle's index + 1 in place of its weight: the
        # sorted weights are then the permutation
        tagged = dict(species)
        tagged["w"] = np.arange(1, npart + 1, dtype=np.float64)
        self.h = self.sim.add_species(tagged)
        self.sim.sort(self.h)
        cur = self.h.current()
        self.npart = self.h.np
        assert self.npart == npart
        self.perm = (cur["w"][:npart].double().round().long() - 1)  # sorted slot -> original index
        w0 = torch.as_tensor(np.asarray(species["w"], np.float64), device=self.sim.device)
        cur["w"][:npart].copy_(w0[self.perm].to(self.sim.dtype))
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
        self.sim.step(1, [self.h])

    def _energy(self) -> float:
        d = self.sim.diagnostics([self.h])
        return d["UE"] + d["UB"]

    # ---- the differentiable map
    def forward(self, ey_src: torch.Tensor, u0: torch.Tensor):
        s = self.sim
        zeros = [torch.zeros(s.ncells, dtype=self.dtype, device=s.device) for _ in range(3)]
        E = [zeros[0], ey_src.detach().to(self.dtype).contiguous(), zeros[2]]
        B = [torch.zeros_like(zeros[0]) for _ in range(3)]
        u = [u0[d].detach()[self.perm].to(self.dtype).contiguous() for d in range(3)]
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
                spn.tile_start = self.h.struct.tile_start  # same particle order: the tiled reverse step
                fn = _fields_struct(E, B, scratch_j)
                s._call(lib.pic_particle_adjoint(s.ctx, ctypes.byref(spn), ctypes.byref(fn), ctypes.byref(lam_f),
                                                 ctypes.byref(lsp), st), "pic_particle_adjoint")
        s.check()
        gu = torch.empty((3, self.npart), dtype=dt, device=dev)
        gu[:, self.perm] = torch.stack(lu)  # back to the caller's particle order
        return lam["E"][1].clone(), gu


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
