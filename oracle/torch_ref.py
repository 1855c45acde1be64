"""Second, independent FP64 implementation of the PIC step in plain PyTorch
(CPU), differentiable with torch.autograd.  TEST INFRASTRUCTURE ONLY: the
reference gradient for the hand-written adjoint of the HIP library, and a
forward cross-check of the C oracle.

It follows the same method (paper Sec. 2: shape-weighted gather, eq. 3 with
leap-frog and the relativistic Boris rotation, eq. 4 in Esirkepov's
charge-conserving form, the two curl equations on the Yee lattice) but is
written separately: positions are continuous coordinates in cell units
(x = cell + offset), windows are vectorised over particles, fields are
(3, nz, ny, nx) tensors and the curls use torch.roll.  The integer parts of
positions are constants for autograd, so gradients flow through offsets,
momenta, weights and fields.
"""
from __future__ import annotations

import math

import torch

TD = torch.float64
# stagger of Ex Ey Ez Bx By Bz (cell units, x y z)
STAGGER = ((0.5, 0, 0), (0, 0.5, 0), (0, 0, 0.5), (0, 0.5, 0.5), (0.5, 0, 0.5), (0.5, 0.5, 0))


def shape(order: int, r: torch.Tensor) -> torch.Tensor:
    """B-spline of order 1 (hat) or 2 (quadratic) at distance r (cell units)."""
    a = r.abs()
    if order == 1:
        return torch.clamp(1.0 - a, min=0.0)
    inner = 0.75 - r * r
    outer = 0.5 * (1.5 - a) ** 2
    return torch.where(a <= 0.5, inner, torch.where(a < 1.5, outer, torch.zeros_like(r)))


class Grid:
    def __init__(self, dims, n, dx, dt, order):
        self.dims, self.n, self.dx, self.dt, self.order = dims, tuple(n), tuple(dx), float(dt), order
        self.dV = math.prod(dx[:dims])

    @property
    def shape3(self):
        return (self.n[2], self.n[1], self.n[0])


def _flat(g: Grid, i, j, k):
    return (i % g.n[0]) + g.n[0] * ((j % g.n[1]) + g.n[1] * (k % g.n[2]))


def gather(g: Grid, E: torch.Tensor, B: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
    """(6, np): every component averaged over its own staggered grid with the
    particle shape, a 4-node window per dimension from floor(xi) - 1."""
    F = torch.cat([E.reshape(3, -1), B.reshape(3, -1)])
    ar = torch.arange(4, dtype=torch.int64)
    out = []
    for c in range(6):
        nodes_d = []
        for d in range(3):
            if d < g.dims:
                base = torch.floor((x[d] - STAGGER[c][d]).detach()).to(torch.int64) - 1
                nodes_d.append(base[:, None] + ar[None, :])
            else:
                nodes_d.append(torch.zeros((x.shape[1], 1), dtype=torch.int64))
        flat = _flat(g, nodes_d[0][:, :, None, None], nodes_d[1][:, None, :, None], nodes_d[2][:, None, None, :])
        vals = F[c][flat.reshape(-1)].reshape(flat.shape)
        out.append((vals * _weights(g, x, c)).sum(dim=(1, 2, 3)))
    return torch.stack(out)


def _weights(g: Grid, x: torch.Tensor, c: int) -> torch.Tensor:
    ar = torch.arange(4, dtype=torch.int64)
    ws = []
    for d in range(3):
        if d < g.dims:
            xi = x[d] - STAGGER[c][d]
            base = torch.floor(xi.detach()).to(torch.int64) - 1
            nodes = base[:, None] + ar[None, :]
            ws.append(shape(g.order, xi[:, None] - nodes.to(TD)))
        else:
            ws.append(torch.ones((x.shape[1], 1), dtype=TD))
    return ws[0][:, :, None, None] * ws[1][:, None, :, None] * ws[2][:, None, None, :]


def boris(q: float, m: float, dt: float, eb: torch.Tensor, u: torch.Tensor) -> torch.Tensor:
    """Relativistic Boris rotation u^{n-1/2} -> u^{n+1/2}."""
    h = q * dt / (2.0 * m)
    E, B = eb[:3], eb[3:]
    um = u + h * E
    gm = torch.sqrt(1.0 + (um * um).sum(0))
    t = h * B / gm
    s = 2.0 * t / (1.0 + (t * t).sum(0))
    up = um + torch.linalg.cross(um, t, dim=0)
    upl = um + torch.linalg.cross(up, s, dim=0)
    return upl + h * E


def deposit(g: Grid, q: float, x0: torch.Tensor, x1: torch.Tensor, u: torch.Tensor, w: torch.Tensor) -> torch.Tensor:
    """Esirkepov current (3, N) of particles moving x0 -> x1 (unwrapped)."""
    N = g.n[0] * g.n[1] * g.n[2]
    npart = x0.shape[1]
    J = torch.zeros((3, N), dtype=TD)
    W = 6
    ar = torch.arange(W, dtype=torch.int64)
    S0, DS, nodes = [], [], []
    for d in range(3):
        if d < g.dims:
            base = torch.floor(x0[d].detach()).to(torch.int64) - 2
            nd = base[:, None] + ar[None, :]
            s0 = shape(g.order, x0[d][:, None] - nd.to(TD))
            s1 = shape(g.order, x1[d][:, None] - nd.to(TD))
        else:
            nd = torch.zeros((npart, 1), dtype=torch.int64)
            s0 = torch.ones((npart, 1), dtype=TD)
            s1 = torch.ones((npart, 1), dtype=TD)
        S0.append(s0)
        DS.append(s1 - s0)
        nodes.append(nd)
    qw = q * w / g.dV
    I = nodes[0][:, :, None, None]
    Jn = nodes[1][:, None, :, None]
    K = nodes[2][:, None, None, :]
    flat = _flat(g, I, Jn, K).expand(npart, nodes[0].shape[1], nodes[1].shape[1], nodes[2].shape[1])

    def outer(a, b, c):
        return a[:, :, None, None] * b[:, None, :, None] * c[:, None, None, :]

    if g.dims == 3:
        for comp, (a, b, c) in enumerate(((0, 1, 2), (1, 0, 2), (2, 0, 1))):
            Sb0, Sc0, Db, Dc = S0[b], S0[c], DS[b], DS[c]
            trans = (Sb0[:, :, None] * Sc0[:, None, :] + 0.5 * Db[:, :, None] * Sc0[:, None, :]
                     + 0.5 * Sb0[:, :, None] * Dc[:, None, :] + Db[:, :, None] * Dc[:, None, :] / 3.0)
            # W_a[i_a, i_b, i_c] = DS_a * trans ; arrange to [i, j, k]
            if a == 0:
                Wc = DS[0][:, :, None, None] * trans[:, None, :, :]
            elif a == 1:
                Wc = DS[1][:, None, :, None] * trans[:, :, None, :]
            else:
                Wc = DS[2][:, None, None, :] * trans[:, :, :, None]
            acc = torch.cumsum(Wc, dim=1 + a)
            contrib = (-qw * g.dx[a] / g.dt)[:, None, None, None] * acc
            J[comp] = J[comp].index_add(0, flat.reshape(-1), contrib.reshape(-1))
    else:
        for comp, (a, b) in enumerate(((0, 1), (1, 0))):
            trans = S0[b] + 0.5 * DS[b]
            if a == 0:
                Wc = DS[0][:, :, None] * trans[:, None, :]
            else:
                Wc = trans[:, :, None] * DS[1][:, None, :]
            acc = torch.cumsum(Wc, dim=1 + a)
            contrib = (-qw * g.dx[a] / g.dt)[:, None, None] * acc
            J[comp] = J[comp].index_add(0, flat.reshape(-1), contrib[..., None].reshape(-1))
        gam = torch.sqrt(1.0 + (u * u).sum(0))
        vz = u[2] / gam
        Wz = (S0[0][:, :, None] * S0[1][:, None, :] + 0.5 * DS[0][:, :, None] * S0[1][:, None, :]
              + 0.5 * S0[0][:, :, None] * DS[1][:, None, :] + DS[0][:, :, None] * DS[1][:, None, :] / 3.0)
        contrib = (qw * vz)[:, None, None] * Wz
        J[2] = J[2].index_add(0, flat.reshape(-1), contrib[..., None].reshape(-1))
    return J


def _roll(F, shift, axis, g):
    # F: (nz, ny, nx); axis 0 = x, 1 = y, 2 = z
    return torch.roll(F, shifts=shift, dims=2 - axis)


def curl_e(g: Grid, E: torch.Tensor) -> torch.Tensor:
    """Curl of E at the B points (forward differences)."""
    Ex, Ey, Ez = (E[c].reshape(g.shape3) for c in range(3))

    def dfwd(F, ax):
        if ax >= g.dims:
            return torch.zeros_like(F)
        return (_roll(F, -1, ax, g) - F) / g.dx[ax]

    return torch.stack([(dfwd(Ez, 1) - dfwd(Ey, 2)).reshape(-1), (dfwd(Ex, 2) - dfwd(Ez, 0)).reshape(-1),
                        (dfwd(Ey, 0) - dfwd(Ex, 1)).reshape(-1)])


def curl_b(g: Grid, B: torch.Tensor) -> torch.Tensor:
    """Curl of B at the E points (backward differences)."""
    Bx, By, Bz = (B[c].reshape(g.shape3) for c in range(3))

    def dbwd(F, ax):
        if ax >= g.dims:
            return torch.zeros_like(F)
        return (F - _roll(F, 1, ax, g)) / g.dx[ax]

    return torch.stack([(dbwd(Bz, 1) - dbwd(By, 2)).reshape(-1), (dbwd(Bx, 2) - dbwd(Bz, 0)).reshape(-1),
                        (dbwd(By, 0) - dbwd(Bx, 1)).reshape(-1)])


def step(g: Grid, E, B, species):
    """One step; species = list of dicts {q, m, x (3,np), u (3,np), w (np)} with
    x continuous in cell units.  Returns (E, B, J, new species)."""
    N = g.n[0] * g.n[1] * g.n[2]
    J = torch.zeros((3, N), dtype=TD)
    out = []
    for sp in species:
        eb = gather(g, E, B, sp["x"])
        u = boris(sp["q"], sp["m"], g.dt, eb, sp["u"])
        gam = torch.sqrt(1.0 + (u * u).sum(0))
        disp = torch.stack([g.dt * u[d] / gam / g.dx[d] if d < g.dims else torch.zeros_like(u[d]) for d in range(3)])
        x1 = sp["x"] + disp
        J = J + deposit(g, sp["q"], sp["x"], x1, u, sp["w"])
        n = torch.tensor([g.n[0], g.n[1], g.n[2]], dtype=TD)[:, None]
        xw = torch.remainder(x1, n)
        out.append(dict(sp, x=xw, u=u))
    B = B - 0.5 * g.dt * curl_e(g, E)
    E = E + g.dt * (curl_b(g, B) - J)
    B = B - 0.5 * g.dt * curl_e(g, E)
    return E, B, J, out


def field_energy(g: Grid, E, B):
    return 0.5 * g.dV * ((E * E).sum() + (B * B).sum())


def rollout_loss(g: Grid, E0, B0, species, steps: int):
    E, B = E0, B0
    sp = species
    for _ in range(steps):
        E, B, _, sp = step(g, E, B, sp)
    return field_energy(g, E, B)
