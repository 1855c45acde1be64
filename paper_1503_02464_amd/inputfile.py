"""JSON input files: a run described without code (the paper's Sec. 3.2: a
simulation initialised by reading a user-friendly JSON input file, so that
typical setups need no code editing).

A file holds one object; units are normalised (c = eps0 = 1, charge in e,
mass in m_e, lengths in c/omega_p for plasma boxes, c/omega_L for laser boxes):

    {
      "name": "...",
      "grid": {"dims": 3, "cells": [nx, ny, nz], "dx": [dx, dy, dz],
               "cfl": 0.7},                     # or "dt": value
      "shape_order": 2,                         # 1 linear, 2 quadratic
      "precision": "fp32",                      # or "fp64"
      "steps": 200,
      "launch": {"tile": [8, 8, 8], "slack": 1, "sort_every": 12,
                 "sort_levels": 0, "current_accum": "auto"},
      "boundaries": {"x": "periodic"}           # or {"x": "open", "absorb": 8}
      "laser": {"plane": 4, "a0": 5.0, "omega": 1.0, "waist": ...,
                "duration_fwhm": ..., "t0": ..., "axis": [yc, zc],
                "polarisation": "y"},           # open x only; optional
      "species": [
        {"name": "electrons", "charge": -1.0, "mass": 1.0,
         "profile": {"kind": "uniform"},        # or {"kind": "slab", "x_cells": [x0, x1]}
         "density": 1.0, "ppc": 8,
         "momentum": {"spread": 0.05, "mean": [0, 0, 0]},
         "seed": 1002},
        {"name": "ions", "charge": 1.0, "mass": 1836.0,
         "co_located_with": "electrons",        # same positions as that species
         "momentum": {"spread": 0.0}, "seed": 1004}
      ],
      "extra": {...}                            # workload-specific values
    }

``load`` validates a file and returns a ``RunSpec``; ``RunSpec.workload()``
gives the same workload objects as ``configs`` (so a file and the code path
describe identical runs), ``RunSpec.species()`` draws the particles with the
seeded generators of ``inputs``, and ``RunSpec.simulation()`` builds the
``Simulation`` with its laser and species.  ``python -m
paper_1503_02464_amd.run FILE`` runs one.
"""
from __future__ import annotations

import json
import math
from dataclasses import dataclass, field

from . import configs, inputs

_PRECISIONS = ("fp32", "fp64")
_ACCUM = ("auto", "fix64", "fp64", "fp32")


class InputError(ValueError):
    """A JSON input file that does not describe a valid run."""


def _need(obj: dict, key: str, where: str):
    if key not in obj:
        raise InputError(f"{where}: missing '{key}'")
    return obj[key]


def _vec(v, n: int, where: str, kind=float) -> tuple:
    if not isinstance(v, (list, tuple)) or len(v) != n:
        raise InputError(f"{where}: expected a list of {n} values, got {v!r}")
    try:
        return tuple(kind(x) for x in v)
    except (TypeError, ValueError) as e:
        raise InputError(f"{where}: {e}") from None


@dataclass
class SpeciesSpec:
    name: str
    charge: float
    mass: float
    density: float = 0.0
    ppc: int = 0
    profile: dict = field(default_factory=lambda: {"kind": "uniform"})
    spread: float = 0.0
    mean: tuple = (0.0, 0.0, 0.0)
    seed: int = 0
    co_located_with: str | None = None


@dataclass
class RunSpec:
    name: str
    dims: int
    n: tuple
    dx: tuple
    dt: float
    cfl: float | None
    order: int
    precision: str
    steps: int
    tile: tuple
    slack: int
    sort_every: int
    sort_levels: int
    current_accum: str
    open_x: bool
    absorb: int
    laser: dict | None
    species_specs: list
    extra: dict

    # -- what the file describes ------------------------------------------
    def workload(self):
        """The run as the workload objects of ``configs``: a ``LaserFoil`` for
        an open box with a slab of electrons and co-located ions, else a
        ``Workload`` (one species, or two counter-streaming beams)."""
        sp = self.species_specs
        if self.open_x:
            e = sp[0]
            ions = [s for s in sp if s.co_located_with == e.name]
            if len(sp) != 2 or not ions or e.profile.get("kind") != "slab" or self.laser is None:
                raise InputError("an open box maps onto a laser-foil workload: a slab species, co-located ions "
                                 "and a laser")
            i = ions[0]
            x0, x1 = e.profile["x_cells"]
            L = self.laser
            return configs.LaserFoil(self.name, self.dims, self.n, self.dx, self.cfl, self.order, self.steps,
                                     (int(x0), int(x1)), e.density, e.ppc, e.spread, i.spread, L["a0"], L["waist"],
                                     L["duration_fwhm"], absorb=self.absorb, laser_plane=L["plane"], tile=self.tile,
                                     seed=e.seed, m_ion=i.mass, sort_levels=self.sort_levels)
        first = sp[0]
        density = sum(s.density for s in sp)
        ppc = sum(s.ppc for s in sp)
        extra = dict(self.extra)
        return configs.Workload(self.name, self.dims, self.n, self.dx, self.cfl, self.order, ppc, first.spread,
                                self.steps, density=density, seed=first.seed, tile=self.tile, extra=extra)

    def species(self) -> list:
        """The particles of every species (numpy dicts in the per-dimension
        cell + offset form), drawn with ``inputs``' seeded generators."""
        out, by_name = [], {}
        for s in self.species_specs:
            if s.co_located_with is not None:
                if s.co_located_with not in by_name:
                    raise InputError(f"species {s.name}: co_located_with names no earlier species")
                base = by_name[s.co_located_with]
                d = inputs.co_located(base, s.charge, s.mass, s.spread, s.seed)
            else:
                cell_volume = math.prod(self.dx[:self.dims])
                w = s.density * cell_volume / s.ppc
                kind = s.profile.get("kind")
                if kind == "uniform":
                    d = inputs.uniform_plasma(self.n, self.dims, s.ppc, s.spread, w, s.seed, q=s.charge, m=s.mass,
                                              u_mean=s.mean)
                elif kind == "slab":
                    x0, x1 = s.profile["x_cells"]
                    d = inputs.foil(self.n, self.dims, int(x0), int(x1), s.ppc, s.spread, w, s.seed, q=s.charge,
                                    m=s.mass)
                else:
                    raise InputError(f"species {s.name}: unknown profile kind {kind!r}")
            by_name[s.name] = d
            out.append(d)
        return out

    def simulation(self, device: str = "cuda"):
        """A ``Simulation`` of this run with its laser and species added
        (returns the simulation and the species handles)."""
        from .sim import Simulation
        sp = self.species()
        sim = Simulation(self.dims, self.n, self.dx, self.dt, self.order, self.precision, tile=self.tile,
                         slack=self.slack, sort_every=self.sort_every,
                         max_particles=max((d["w"].shape[0] for d in sp), default=1),
                         current_accum=self.current_accum, open_x=self.open_x, absorb=self.absorb,
                         sort_levels=self.sort_levels, device=device)
        if self.laser is not None:
            L = self.laser
            sim.set_laser(L["plane"], L["a0"], L["omega"], L["waist"], L["duration_fwhm"], L["t0"], L["axis"][0],
                          L["axis"][1], 1 if L["polarisation"] == "y" else 2)
        handles = [sim.add_species(d) for d in sp]
        return sim, handles


def parse(doc: dict) -> RunSpec:
    """Validate one input document (the parsed JSON object)."""
    if not isinstance(doc, dict):
        raise InputError("the input file must hold one JSON object")
    name = str(doc.get("name", "run"))
    g = _need(doc, "grid", "file")
    dims = int(_need(g, "dims", "grid"))
    if dims not in (2, 3):
        raise InputError("grid.dims must be 2 or 3")
    n = _vec(_need(g, "cells", "grid"), dims, "grid.cells", int) + (1,) * (3 - dims)
    dx = _vec(_need(g, "dx", "grid"), dims, "grid.dx") + (1.0,) * (3 - dims)
    if min(n) < 1 or min(dx[:dims]) <= 0:
        raise InputError("grid: cells and dx must be positive")
    limit = configs.yee_dt_max(dims, dx)
    cfl = None
    if "dt" in g:
        dt = float(g["dt"])
    else:
        cfl = float(_need(g, "cfl", "grid"))
        dt = cfl * limit
    if not (0 < dt < limit):
        raise InputError(f"grid: dt = {dt} must lie in (0, {limit}) (the Yee limit)")
    order = int(doc.get("shape_order", 2))
    if order not in (1, 2):
        raise InputError("shape_order must be 1 or 2")
    prec = str(doc.get("precision", "fp32"))
    if prec not in _PRECISIONS:
        raise InputError(f"precision must be one of {_PRECISIONS}")
    steps = int(doc.get("steps", 1))
    ln = doc.get("launch", {})
    tile = _vec(ln.get("tile", [8, 8, 8][:dims]), dims, "launch.tile", int) + (1,) * (3 - dims)
    for d in range(dims):
        if n[d] % tile[d]:
            raise InputError(f"launch.tile[{d}] = {tile[d]} does not divide grid.cells[{d}] = {n[d]}")
    accum = str(ln.get("current_accum", "auto"))
    if accum not in _ACCUM:
        raise InputError(f"launch.current_accum must be one of {_ACCUM}")
    bc = doc.get("boundaries", {"x": "periodic"})
    bx = bc.get("x", "periodic")
    if bx not in ("periodic", "open"):
        raise InputError("boundaries.x must be 'periodic' or 'open'")
    open_x = bx == "open"
    absorb = int(bc.get("absorb", 0)) if open_x else 0
    laser = None
    if "laser" in doc:
        if not open_x:
            raise InputError("a laser needs open x faces (boundaries.x = 'open')")
        L = doc["laser"]
        laser = {"plane": int(_need(L, "plane", "laser")), "a0": float(_need(L, "a0", "laser")),
                 "omega": float(L.get("omega", 1.0)), "waist": float(_need(L, "waist", "laser")),
                 "duration_fwhm": float(_need(L, "duration_fwhm", "laser")),
                 "polarisation": str(L.get("polarisation", "y"))}
        laser["t0"] = float(L.get("t0", 1.5 * laser["duration_fwhm"]))
        axis = L.get("axis", [0.5 * n[1] * dx[1], 0.5 * n[2] * dx[2] if dims == 3 else 0.0])
        laser["axis"] = _vec(axis, 2, "laser.axis")
        if laser["polarisation"] not in ("y", "z") or (laser["polarisation"] == "z" and dims == 2):
            raise InputError("laser.polarisation must be 'y' (or 'z' in 3D)")
    specs = []
    for k, s in enumerate(_need(doc, "species", "file")):
        where = f"species[{k}]"
        mom = s.get("momentum", {})
        sp = SpeciesSpec(name=str(_need(s, "name", where)), charge=float(_need(s, "charge", where)),
                         mass=float(_need(s, "mass", where)), spread=float(mom.get("spread", 0.0)),
                         mean=_vec(mom.get("mean", [0.0, 0.0, 0.0]), 3, where + ".momentum.mean"),
                         seed=int(s.get("seed", 1000 + k)), co_located_with=s.get("co_located_with"))
        if sp.mass <= 0:
            raise InputError(f"{where}: mass must be positive")
        if sp.co_located_with is None:
            sp.density = float(_need(s, "density", where))
            sp.ppc = int(_need(s, "ppc", where))
            sp.profile = dict(s.get("profile", {"kind": "uniform"}))
            if sp.ppc < 1:
                raise InputError(f"{where}: ppc must be at least 1")
            if sp.profile.get("kind") == "slab":
                x0, x1 = _vec(_need(sp.profile, "x_cells", where + ".profile"), 2, where + ".profile.x_cells", int)
                if not (0 <= x0 < x1 <= n[0]):
                    raise InputError(f"{where}: slab x_cells must satisfy 0 <= x0 < x1 <= cells[0]")
        specs.append(sp)
    if not specs:
        raise InputError("at least one species")
    return RunSpec(name=name, dims=dims, n=n, dx=dx, dt=dt, cfl=cfl, order=order, precision=prec, steps=steps,
                   tile=tile, slack=int(ln.get("slack", 1)), sort_every=int(ln.get("sort_every", 8)),
                   sort_levels=int(ln.get("sort_levels", 0)), current_accum=accum, open_x=open_x, absorb=absorb,
                   laser=laser, species_specs=specs, extra=dict(doc.get("extra", {})))


def load(path: str) -> RunSpec:
    """Read and validate a JSON input file."""
    with open(path) as f:
        try:
            doc = json.load(f)
        except json.JSONDecodeError as e:
            raise InputError(f"{path}: {e}") from None
    return parse(doc)
