"""Seeded synthetic inputs shared by the HIP path and the oracle.

This module holds random draws and data placement only: none of the PIC
method's arithmetic.  It produces particle states as plain numpy arrays in the
per-dimension (cell index, offset) form, plus random field arrays.

* Positions: exactly ``ppc`` particles per cell, offsets uniform in [0,1)^D.
* Momenta u = p/(m c): each component drawn from N(0, sigma^2), no mean removed.
* Weights: a constant supplied by the caller.

Two counter-streaming beams (the two-stream workload): ``two_beams`` places
``ppc`` particles per cell per beam at uniform random offsets with mean
momenta +-u0 along x; ``quiet_beams`` places them on a regular sub-lattice of
every cell (the same points for both beams) with u_x = +-u0 + eps sin(k x).

``round_f32`` snaps a state onto float32-representable values (offsets stay
strictly below 1) so the FP32 path and the FP64 oracle start from the same
numbers.
"""
from __future__ import annotations

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_plasma(n: tuple, dims: int, ppc: int, u_sigma: float, weight: float, seed: int,
                   q: float = -1.0, m: float = 1.0, u_mean: tuple = (0.0, 0.0, 0.0)) -> dict:
    """``ppc`` particles in every cell of an n[0] x n[1] x n[2] box (n[2] = 1 in 2D),
    ordered cell by cell (x fastest), offsets uniform, momenta Gaussian."""
    g = rng(seed)
    ncell = int(n[0] * n[1] * n[2])
    npart = ncell * ppc
    lin = np.repeat(np.arange(ncell, dtype=np.int64), ppc)
    cell = np.zeros((3, npart), np.int32)
    cell[0] = lin % n[0]
    cell[1] = (lin // n[0]) % n[1]
    cell[2] = lin // (n[0] * n[1])
    off = np.zeros((3, npart), np.float64)
    off[:dims] = g.random((dims, npart))
    u = g.normal(0.0, u_sigma, (3, npart)) if u_sigma > 0 else np.zeros((3, npart))
    u = u + np.asarray(u_mean, np.float64)[:, None]
    w = np.full(npart, weight, np.float64)
    return {"q": float(q), "m": float(m), "cell": cell, "off": off, "u": np.ascontiguousarray(u), "w": w}


def foil(n: tuple, dims: int, x0: int, x1: int, ppc: int, u_sigma: float, weight: float, seed: int,
         q: float = -1.0, m: float = 1.0) -> dict:
    """A slab: ``ppc`` particles in every cell with x cell in [x0, x1) over the
    whole y (and z) extent, ordered cell by cell, offsets uniform, momenta
    Gaussian (sigma 0: cold)."""
    g = rng(seed)
    nx = x1 - x0
    ncell = int(nx * n[1] * n[2])
    npart = ncell * ppc
    lin = np.repeat(np.arange(ncell, dtype=np.int64), ppc)
    cell = np.zeros((3, npart), np.int32)
    cell[0] = x0 + lin % nx
    cell[1] = (lin // nx) % n[1]
    cell[2] = lin // (nx * n[1])
    off = np.zeros((3, npart), np.float64)
    off[:dims] = g.random((dims, npart))
    u = g.normal(0.0, u_sigma, (3, npart)) if u_sigma > 0 else np.zeros((3, npart))
    w = np.full(npart, weight, np.float64)
    return {"q": float(q), "m": float(m), "cell": cell, "off": off, "u": np.ascontiguousarray(u), "w": w}


def co_located(sp: dict, q: float, m: float, u_sigma: float, seed: int) -> dict:
    """A second species at exactly the positions of ``sp`` (so the initial
    charge density of the pair vanishes), with its own Gaussian momenta."""
    g = rng(seed)
    npart = sp["w"].shape[0]
    u = g.normal(0.0, u_sigma, (3, npart)) if u_sigma > 0 else np.zeros((3, npart))
    return {"q": float(q), "m": float(m), "cell": sp["cell"].copy(), "off": sp["off"].copy(),
            "u": np.ascontiguousarray(u), "w": sp["w"].copy()}


def shuffle(sp: dict, seed: int) -> dict:
    """Random permutation of the particles (order carries no physics)."""
    perm = rng(seed).permutation(sp["w"].shape[0])
    out = dict(sp)
    for k in ("cell", "off", "u"):
        out[k] = np.ascontiguousarray(sp[k][:, perm])
    out["w"] = np.ascontiguousarray(sp["w"][perm])
    return out


def random_particles(n: tuple, dims: int, npart: int, u_sigma: float, weight_range: tuple, seed: int,
                     q: float = -1.0, m: float = 1.0) -> dict:
    """``npart`` particles at uniform random cells and offsets, random weights."""
    g = rng(seed)
    cell = np.zeros((3, npart), np.int32)
    for d in range(dims):
        cell[d] = g.integers(0, n[d], npart)
    off = np.zeros((3, npart), np.float64)
    off[:dims] = g.random((dims, npart))
    u = np.ascontiguousarray(g.normal(0.0, u_sigma, (3, npart)))
    w = g.uniform(weight_range[0], weight_range[1], npart)
    return {"q": float(q), "m": float(m), "cell": cell, "off": off, "u": u, "w": w}


def random_fields(ncells: int, scale: float, seed: int) -> dict:
    """E and B with N(0, scale^2) entries, J zero; arrays (3, ncells)."""
    g = rng(seed)
    return {"E": g.normal(0.0, scale, (3, ncells)), "B": g.normal(0.0, scale, (3, ncells)),
            "J": np.zeros((3, ncells))}


def round_f32(sp: dict) -> dict:
    """Snap offsets, momenta and weights to float32 values (kept as float64).
    Offsets that would round up to 1.0 are set to the largest float32 below 1."""
    out = dict(sp)
    off = sp["off"].astype(np.float32)
    off = np.where(off >= np.float32(1.0), np.nextafter(np.float32(1.0), np.float32(0.0)), off)
    out["off"] = np.ascontiguousarray(off.astype(np.float64))
    out["u"] = np.ascontiguousarray(sp["u"].astype(np.float32).astype(np.float64))
    out["w"] = np.ascontiguousarray(sp["w"].astype(np.float32).astype(np.float64))
    out["cell"] = np.ascontiguousarray(sp["cell"].copy())
    return out


def round_fields_f32(f: dict) -> dict:
    return {k: np.ascontiguousarray(v.astype(np.float32).astype(np.float64)) for k, v in f.items()}


def two_beams(n: tuple, dims: int, ppc: int, u0: float, u_sigma: float, weight: float, seed: int,
              q: float = -1.0, m: float = 1.0) -> tuple:
    """Two beams of ``ppc`` particles per cell each, offsets uniform, momenta
    Gaussian (spread u_sigma) about (+u0, 0, 0) and (-u0, 0, 0)."""
    a = uniform_plasma(n, dims, ppc, u_sigma, weight, seed, q=q, m=m, u_mean=(u0, 0.0, 0.0))
    b = uniform_plasma(n, dims, ppc, u_sigma, weight, seed + 1, q=q, m=m, u_mean=(-u0, 0.0, 0.0))
    return a, b


def quiet_beams(n: tuple, dims: int, sub: tuple, u0: float, eps: float, k: float, dx: float, weight: float,
                q: float = -1.0, m: float = 1.0) -> tuple:
    """Two cold beams on the same regular sub-lattice of sub[0] x sub[1] (x sub[2])
    points per cell (offsets (i + 1/2)/sub), with u_x = +-u0 + eps sin(k x) at
    x = (cell + offset) dx: a quiet start with one seeded mode."""
    ncell = int(n[0] * n[1] * n[2])
    per = int(np.prod(sub[:dims]))
    lin = np.repeat(np.arange(ncell, dtype=np.int64), per)
    npart = ncell * per
    cell = np.zeros((3, npart), np.int32)
    cell[0] = lin % n[0]
    cell[1] = (lin // n[0]) % n[1]
    cell[2] = lin // (n[0] * n[1])
    grids = np.meshgrid(*[(np.arange(sub[d]) + 0.5) / sub[d] for d in range(dims)], indexing="ij")
    off = np.zeros((3, npart), np.float64)
    for d in range(dims):
        off[d] = np.tile(grids[d].ravel(), ncell)
    x = (cell[0] + off[0]) * dx
    out = []
    for sign in (1.0, -1.0):
        u = np.zeros((3, npart))
        u[0] = sign * u0 + eps * np.sin(k * x)
        out.append({"q": float(q), "m": float(m), "cell": cell.copy(), "off": off.copy(), "u": u,
                    "w": np.full(npart, weight, np.float64)})
    return tuple(out)


def uniform_plasma_device(arrays: dict, n: tuple, dims: int, bits: tuple, ppc: int, u_mean: tuple, u_sigma: float,
                          weight: float, seed: int, chunk: int = 1 << 26) -> None:
    """Fill device arrays (cell: packed int32, off[3], u[3], w; torch tensors)
    in place with ``ppc`` particles per cell, cell by cell, offsets uniform in
    [0,1), momenta Gaussian about u_mean, from torch's seeded device
    generator, in chunks of ``chunk`` particles (for boxes too large to draw
    on the host).  The draws differ from the numpy generators'; the layout is
    the same."""
    import torch
    cell = arrays["cell"]
    dev = cell.device
    npart = int(n[0] * n[1] * n[2]) * ppc
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(seed))
    for lo in range(0, npart, chunk):
        hi = min(lo + chunk, npart)
        lin = torch.arange(lo, hi, device=dev, dtype=torch.int64) // ppc
        ix = lin % n[0]
        iy = (lin // n[0]) % n[1]
        iz = lin // (n[0] * n[1])
        packed = ix | (iy << bits[0]) | (iz << (bits[0] + bits[1]))
        cell[lo:hi] = packed.to(torch.int32)
        del lin, ix, iy, iz, packed
        for d in range(3):
            off = arrays["off"][d]
            if d < dims:
                off[lo:hi] = torch.rand(hi - lo, generator=gen, device=dev, dtype=off.dtype)
            u = arrays["u"][d]
            u[lo:hi] = torch.randn(hi - lo, generator=gen, device=dev, dtype=u.dtype) * u_sigma + u_mean[d]
        arrays["w"][lo:hi] = weight
