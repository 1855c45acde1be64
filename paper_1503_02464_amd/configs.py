"""The five synthetic workloads, in normalised units (c = eps0 = 1, charge in e,
mass in m_e, lengths in c/omega_p for plasma boxes, c/omega_L for laser boxes).

Readings where the workload text is silent (each is listed with its reason in
the design notes):
* "CFL limit" is the Yee limit dt_max = 1/sqrt(sum 1/dx_d^2), stricter than the
  dx >= c dt statement of Sec. 2.
* the uniform thermal 3D box and the differentiable 2D box give no cell size:
  dx = 0.05 c/omega_p as in the small 2D box, dt = 0.7 of the limit.
* macro weight w = n dV / ppc, so omega_p = 1 at n = 1 (paper eq. 2, the
  normalisation A absorbed into w; Sec. 3.3 per-particle weight).
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


WORKLOADS = {"uniform-2d-64": uniform_2d_small, "thermal-3d-256": thermal_3d, "diff-2d-512": diff_2d}


# Launch configuration of the fused step for the 3D benchmark workload, per
# precision: cells per tile, guard slack, sort cadence.  The FP64 tile is
# halved in z so fields + current + the wide-window list fit 160 KB of LDS.
BENCH_LAUNCH = {"fp32": {"tile": (8, 8, 8), "slack": 1, "sort_every": 4},
                "fp64": {"tile": (8, 8, 4), "slack": 1, "sort_every": 4}}
