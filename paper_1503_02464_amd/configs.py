"""The synthetic workloads, in normalised units (c = eps0 = 1, charge in e,
mass in m_e, lengths in c/omega_p for plasma boxes, c/omega_L for laser boxes).

Readings where the workload text is silent (each is listed with its reason in
the design notes):
* "CFL limit" is the Yee limit dt_max = 1/sqrt(sum 1/dx_d^2), stricter than the
  dx >= c dt statement of Sec. 2.
* the uniform thermal 3D box and the differentiable 2D box give no cell size:
  dx = 0.05 c/omega_p as in the small 2D box, dt = 0.7 of the limit.
* macro weight w = n dV / ppc, so omega_p = 1 at n = 1 (paper eq. 2, the
  normalisation A absorbed into w; Sec. 3.3 per-particle weight).
* laser boxes: lengths in c/omega_L (lambda = 2 pi, n_c = 1, a0 = peak E in
  m_e c omega_L / e); open x faces with the particle region `absorb` cells in
  from each face and the laser sheet on the node plane `laser_plane`; waist =
  1/e field radius, duration = FWHM of the intensity, envelope centre
  t0 = 1.5 tau; the beam waist sits on the sheet (its Rayleigh length, at
  least 28 lambda, dwarfs the distance to the foil, so the foil sees the same
  spot size within 2 %); foil front at 10 lambda (2D) and 5 lambda (3D);
  ions (Z = 1, m = 1836 m_e) at the electrons' positions; the 3D box's
  thermal spread 0.001 m_e c is a momentum spread for both species.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field


def yee_dt_max(dims: int, dx: tuple) -> float:
    return 1.0 / math.sqrt(sum(1.0 / dx[d] ** 2 for d in range(dims)))


@dataclass
class Workload:
    name: str
    dims: int
    n: tuple
    dx: tuple
    cfl: float
    order: int
    ppc: int
    u_sigma: float
    steps: int
    density: float = 1.0
    seed: int = 1000
    tile: tuple = (8, 8, 1)
    note: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def dt(self) -> float:
        return self.cfl * yee_dt_max(self.dims, self.dx)

    @property
    def ncells(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    @property
    def nparticles(self) -> int:
        return self.ncells * self.ppc

    @property
    def cell_volume(self) -> float:
        v = 1.0
        for d in range(self.dims):
            v *= self.dx[d]
        return v

    @property
    def weight(self) -> float:
        return self.density * self.cell_volume / self.ppc


def uniform_2d_small() -> Workload:
    """2D3V periodic uniform plasma, 64x64, dx = 0.05, 0.7 CFL, 4 ppc, sigma 0.01,
    linear shape, 100 steps, FP64."""
    return Workload("uniform-2d3v-64x64-4ppc-linear", 2, (64, 64, 1), (0.05, 0.05, 1.0), 0.7, 1, 4, 0.01, 100,
                    seed=1000, tile=(8, 8, 1))


def thermal_3d(scale: int = 1) -> Workload:
    """3D3V periodic uniform thermal plasma, 256^3 (divided by ``scale`` per dim),
    8 ppc, sigma 0.05, quadratic shape, 200 steps; the bandwidth benchmark."""
    n = 256 // scale
    return Workload(f"thermal-3d3v-{n}^3-8ppc-quadratic", 3, (n, n, n), (0.05, 0.05, 0.05), 0.7, 2, 8, 0.05, 200,
                    seed=1002, tile=(8, 8, 8))


def diff_2d(n: int = 512) -> Workload:
    """Differentiable 2D3V rollout: 512^2, 16 ppc, sigma 0.02, linear shape, 200 steps."""
    return Workload(f"diff-2d3v-{n}x{n}-16ppc-linear", 2, (n, n, 1), (0.05, 0.05, 1.0), 0.7, 1, 16, 0.02, 200,
                    seed=1004, tile=(16, 16, 1), extra={"checkpoint_every": 20, "src_sigma": 0.01})


@dataclass
class LaserFoil:
    """A foil of electrons and ions hit by a laser injected near the low x face."""

    name: str
    dims: int
    n: tuple
    dx: tuple
    cfl: float
    order: int
    steps: int
    foil_x: tuple      # x cells [x0, x1) of the foil
    density: float     # in n_c
    ppc: int           # per species
    u_sigma_e: float   # electron momentum spread (u = p / m_e c)
    u_sigma_i: float   # ion momentum spread (u = p / m_i c)
    a0: float
    waist: float       # 1/e field radius
    tau: float         # intensity FWHM
    absorb: int = 8
    laser_plane: int = 4
    tile: tuple = (16, 16, 1)
    seed: int = 1001
    m_ion: float = 1836.0
    sort_levels: int = 32  # about twice the particles per cell of a species

    @property
    def dt(self) -> float:
        return self.cfl * yee_dt_max(self.dims, self.dx)

    @property
    def ncells(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    @property
    def cell_volume(self) -> float:
        v = 1.0
        for d in range(self.dims):
            v *= self.dx[d]
        return v

    @property
    def weight(self) -> float:
        return self.density * self.cell_volume / self.ppc

    @property
    def t0(self) -> float:
        return 1.5 * self.tau

    def laser(self) -> dict:
        yc = 0.5 * self.n[1] * self.dx[1]
        zc = 0.5 * self.n[2] * self.dx[2] if self.dims == 3 else 0.0
        return {"plane": self.laser_plane, "e0": self.a0, "omega": 1.0, "w0": self.waist, "tau": self.tau,
                "t0": self.t0, "yc": yc, "zc": zc, "pol": 1}

    def species(self):
        """(electrons, ions) as numpy particle dicts, ions co-located."""
        from . import inputs
        e = inputs.foil(self.n, self.dims, self.foil_x[0], self.foil_x[1], self.ppc, self.u_sigma_e, self.weight,
                        self.seed)
        i = inputs.co_located(e, 1.0, self.m_ion, self.u_sigma_i, self.seed + 1)
        return e, i


def laser_foil_2d(scale: int = 1) -> LaserFoil:
    """2D3V laser on a thin foil: 2048x1024 cells, dx = lambda/40, 0.98 CFL,
    open x, periodic y; foil 0.5 lambda at 50 n_c, 64 ppc per species, cold;
    a0 = 5, waist 4 lambda, 10 cycles; quadratic shape, 2000 steps; 8x8
    tiles (the foil is 20 cells thick: 16x16 tiles left a quarter of the
    CUs busy) and 64 sort levels (128, twice the particles per cell, only
    lengthen the sort's scans over tiles x levels).  ``scale`` divides the
    box, the foil position and thickness and the spot."""
    lam = 2 * math.pi
    dx = lam / 40
    x0 = 400 // scale
    return LaserFoil(f"laser-foil-2d3v-{2048 // scale}x{1024 // scale}-64ppc-quadratic", 2,
                     (2048 // scale, 1024 // scale, 1), (dx, dx, 1.0), 0.98, 2, 2000, (x0, x0 + max(20 // scale, 2)),
                     50.0, 64, 0.0, 0.0, 5.0, 4 * lam / scale, 10 * lam, tile=(8, 8, 1), seed=1001,
                     sort_levels=64)


def laser_foil_3d(scale: int = 1) -> LaserFoil:
    """3D3V laser on a foil, one GPU's subdomain: 512x256x256 cells, dx =
    lambda/20, 0.98 CFL, open x; foil 1 lambda at 30 n_c, 16 ppc per species,
    momentum spread 0.001 m_e c; a0 = 10, waist 3 lambda, 10 cycles;
    quadratic shape, FP32, 500 steps."""
    lam = 2 * math.pi
    dx = lam / 20
    x0 = 100 // scale
    return LaserFoil(f"laser-foil-3d3v-{512 // scale}x{256 // scale}x{256 // scale}-16ppc-quadratic", 3,
                     (512 // scale, 256 // scale, 256 // scale), (dx, dx, dx), 0.98, 2, 500,
                     (x0, x0 + max(20 // scale, 2)), 30.0, 16, 0.001, 0.001 / 1836.0, 10.0, 3 * lam / scale,
                     10 * lam, tile=(8, 8, 8), seed=1003, sort_levels=32)


def two_stream_3d(scale: int = 1) -> Workload:
    """The paper's scaling workload (Sec. 4): two counter-streaming beams filling
    a periodic 512x512x128 box (divided by ``scale`` per dimension), 54
    particles per cell.  Readings where the paper is silent: electrons only
    over a fixed neutralising background, 27 particles per cell per beam at
    uniform random offsets, beam momenta +-0.1 m_e c along x with a spread of
    0.001 m_e c, density 1 (0.5 per beam), dx = 0.05 c/omega_p (the most
    unstable wavelength, about 1 c/omega_p, spans 20 cells), dt = 0.7 of the Yee
    limit, quadratic shape, FP32."""
    n = (512 // scale, 512 // scale, 128 // scale)
    return Workload(f"two-stream-3d3v-{n[0]}x{n[1]}x{n[2]}-54ppc-quadratic", 3, n, (0.05, 0.05, 0.05), 0.7, 2, 54,
                    0.001, 200, seed=1005, tile=(8, 8, 8), extra={"u0": 0.1, "beams": 2, "sort_levels": 64})


WORKLOADS = {"uniform-2d-64": uniform_2d_small, "laser-foil-2d": laser_foil_2d, "thermal-3d-256": thermal_3d,
             "laser-foil-3d": laser_foil_3d, "diff-2d-512": diff_2d, "two-stream-3d": two_stream_3d}


# Launch configuration of the fused step for the 3D benchmark workload, per
# precision: cells per tile, guard slack, sort cadence.  The FP64 tile is
# halved in z so fields + current + the wide-window list fit 160 KB of LDS.
BENCH_LAUNCH = {"fp32": {"tile": (8, 8, 8), "slack": 1, "sort_every": 12},
                "fp64": {"tile": (8, 8, 4), "slack": 1, "sort_every": 12}}
