"""Output manager (paper Sec. 3.1): reduced-dimension outputs (a plane of a
3D box, a line of a 2D one) and subdomain outputs (a box inside the grid) of
the fields and charge densities, and phase-space dumps of the particles, each
within a temporal window and at a chosen frequency.

The selection runs on the GPU, right after the step, on the stream the step
ran on (pic_extract_grid packs the box's points, pic_extract_particles
compacts the selected particles in storage order).  The packed result is
copied to pinned host memory on a side stream and saved by a writer thread, so
the following steps run while the copy and the write proceed.  Each request
has two staging slots (device buffer + pinned host buffer) used in turn; a
slot is reused once its previous write has finished.

Requests, one JSON object each (a list of them is the ``--outputs`` file of
``run``):

  {"name": "ey_mid", "kind": "fields", "components": ["Ey", "Bz"],
   "box": {"lo": [0, 0, 64], "hi": [256, 256, 65], "stride": [1, 1, 1]},
   "every": 10, "from": 0, "to": 1000}
  {"name": "rho_e", "kind": "density", "species": [0], "box": {...}, "every": 50}
  {"name": "electrons", "kind": "particles", "species": 0,
   "cells": {"lo": [...], "hi": [...]}, "subsample": 4, "every": 100}

``components`` takes Ex .. Jz or the groups E, B, J; ``box`` is in grid
points (default: the whole grid, stride 1), ``cells`` in cells; ``from`` and
``to`` bound the window (inclusive; default 0 and no end); an output fires at
the steps from, from + every, ... within it.  ``subsample`` keeps every k-th
particle of the storage order; ``capacity`` (records per dump) defaults to
ceil(np / subsample) at the first dump.

Files under the output directory: ``outputs.json`` (the requests as resolved:
components with their Yee positions, boxes, dtypes, record layout), and per
request ``<name>/<step>.npy`` (fields and densities: shape (components, m_z,
m_y, m_x); particles: (count, dims + 4) rows x_0 .. x_{dims-1}, u_0, u_1,
u_2, w) and ``<name>/index.jsonl`` (one line per file: step, time, file,
shape; for particles the count selected and whether the capacity cut it).
"""
from __future__ import annotations

import json
import math
import os
import threading
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

COMPONENTS = {"Ex": ("E", 0), "Ey": ("E", 1), "Ez": ("E", 2), "Bx": ("B", 0), "By": ("B", 1), "Bz": ("B", 2),
              "Jx": ("J", 0), "Jy": ("J", 1), "Jz": ("J", 2)}
# Position of each component's value (i, j, k) on the Yee lattice, in cells from node (i, j, k).
YEE_POSITION = {"Ex": (0.5, 0, 0), "Ey": (0, 0.5, 0), "Ez": (0, 0, 0.5), "Bx": (0, 0.5, 0.5), "By": (0.5, 0, 0.5),
                "Bz": (0.5, 0.5, 0), "Jx": (0.5, 0, 0), "Jy": (0, 0.5, 0), "Jz": (0, 0, 0.5), "rho": (0, 0, 0)}
KINDS = ("fields", "density", "particles")


class OutputError(ValueError):
    """A malformed output request."""


@dataclass
class Request:
    name: str
    kind: str
    lo: tuple
    hi: tuple
    stride: tuple
    every: int
    start: int
    stop: int | None
    components: list = field(default_factory=list)
    species: list = field(default_factory=list)
    subsample: int = 1
    capacity: int | None = None

    def fires(self, step: int) -> bool:
        """Whether this output is written after the given step."""
        if step < self.start or (self.stop is not None and step > self.stop):
            return False
        return (step - self.start) % self.every == 0

    def points(self) -> tuple:
        """Points (or, for particles, cells) per axis of the box, (m_x, m_y, m_z)."""
        return tuple(max(0, -(-(self.hi[d] - self.lo[d]) // self.stride[d])) for d in range(3))


def _ints(v, what: str, name: str) -> tuple:
    if not isinstance(v, (list, tuple)) or not all(isinstance(x, int) and not isinstance(x, bool) for x in v):
        raise OutputError(f"{name}: {what} must be a list of integers")
    return tuple(v)


def _box(spec: dict | None, dims: int, n: tuple, name: str, strided: bool) -> tuple:
    spec = spec or {}
    lo = _ints(spec.get("lo", [0] * dims), "lo", name)
    hi = _ints(spec.get("hi", list(n[:dims])), "hi", name)
    st = _ints(spec.get("stride", [1] * dims), "stride", name) if strided else (1,) * dims
    if not (len(lo) == len(hi) == len(st) == dims):
        raise OutputError(f"{name}: lo, hi and stride need {dims} entries")
    lo, hi, st = lo + (0,) * (3 - dims), hi + (1,) * (3 - dims), st + (1,) * (3 - dims)
    for d in range(3):
        if not (0 <= lo[d] <= hi[d] <= n[d]):
            raise OutputError(f"{name}: need 0 <= lo <= hi <= {n[d]} along axis {d}")
        if st[d] < 1:
            raise OutputError(f"{name}: stride must be >= 1")
    return lo, hi, st


def parse_requests(reqs: list, dims: int, n: tuple, nspecies: int) -> list:
    """Validate output requests against a grid of n cells (dims 2 or 3) with
    nspecies species and resolve their defaults."""
    if not isinstance(reqs, list):
        raise OutputError("the outputs are a list of requests")
    n = tuple(n) + (1,) * (3 - len(n))
    out, names = [], set()
    for r in reqs:
        if not isinstance(r, dict):
            raise OutputError("each output request is an object")
        name = r.get("name")
        if not isinstance(name, str) or not name or "/" in name or name.startswith("."):
            raise OutputError(f"bad output name {name!r}")
        if name in names:
            raise OutputError(f"{name}: duplicate output name")
        names.add(name)
        kind = r.get("kind")
        if kind not in KINDS:
            raise OutputError(f"{name}: kind must be one of {KINDS}")
        every, start, stop = r.get("every", 1), r.get("from", 0), r.get("to")
        if not isinstance(every, int) or every < 1:
            raise OutputError(f"{name}: every must be an integer >= 1")
        if not isinstance(start, int) or start < 0 or (stop is not None and (not isinstance(stop, int) or stop < start)):
            raise OutputError(f"{name}: need 0 <= from <= to")
        req = Request(name, kind, (0, 0, 0), (1, 1, 1), (1, 1, 1), every, start, stop)
        if kind in ("fields", "density"):
            req.lo, req.hi, req.stride = _box(r.get("box"), dims, n, name, True)
        else:
            req.lo, req.hi, req.stride = _box(r.get("cells"), dims, n, name, False)
        if kind == "fields":
            comps = r.get("components", ["E", "B"])
            if not isinstance(comps, list) or not comps:
                raise OutputError(f"{name}: components must be a non-empty list")
            for c in comps:
                if c in ("E", "B", "J"):
                    req.components += [c + a for a in "xyz"]
                elif c in COMPONENTS:
                    req.components.append(c)
                else:
                    raise OutputError(f"{name}: unknown component {c!r}")
            if len(req.components) > 16:
                raise OutputError(f"{name}: at most 16 components")
        elif kind == "density":
            sp = r.get("species", list(range(nspecies)))
            if not isinstance(sp, list) or not sp or not all(isinstance(i, int) and 0 <= i < nspecies for i in sp):
                raise OutputError(f"{name}: species must list indices below {nspecies}")
            req.species, req.components = sp, ["rho"]
        else:
            sp = r.get("species")
            if not isinstance(sp, int) or not 0 <= sp < nspecies:
                raise OutputError(f"{name}: species must be an index below {nspecies}")
            req.species = [sp]
            sub, cap = r.get("subsample", 1), r.get("capacity")
            if not isinstance(sub, int) or sub < 1:
                raise OutputError(f"{name}: subsample must be an integer >= 1")
            if cap is not None and (not isinstance(cap, int) or cap < 1):
                raise OutputError(f"{name}: capacity must be an integer >= 1")
            req.subsample, req.capacity = sub, cap
        out.append(req)
    return out


class _Slot:
    """A device staging buffer, its pinned host twin and the pending write."""

    def __init__(self, shape: tuple, dtype, device):
        import torch
        self.dev = torch.empty(shape, dtype=dtype, device=device)
        self.host = torch.empty(shape, dtype=dtype, pin_memory=True)
        self.count_dev = torch.zeros(1, dtype=torch.int64, device=device)
        self.count_host = torch.zeros(1, dtype=torch.int64, pin_memory=True)
        self.done = None


class OutputManager:
    """Writes the requested outputs of a Simulation after the steps they
    name.  Call after_step() after every step (or chunk of steps; only the
    step it is called at is considered) and close() at the end."""

    def __init__(self, sim, requests: list, out_dir: str, writers: int = 2):
        import torch
        self.sim = sim
        self.reqs = parse_requests(requests, sim.dims, sim.n, len(sim.species))
        self.out = out_dir
        self.copy_stream = torch.cuda.Stream(device=sim.device)
        self.read_stream = torch.cuda.Stream(device=sim.device)
        self.pool = ThreadPoolExecutor(max_workers=writers)
        self.lock = threading.Lock()
        self.slots = {r.name: [None, None] for r in self.reqs}
        self.turn = {r.name: 0 for r in self.reqs}
        self.rho = {}
        self.files = 0
        self.marks = []  # event pairs around each extraction on the step's stream
        os.makedirs(out_dir, exist_ok=True)
        for r in self.reqs:
            os.makedirs(os.path.join(out_dir, r.name), exist_ok=True)
        self._describe()

    def _dtype(self, r: Request):
        import torch
        return torch.float64 if r.kind == "density" else self.sim.dtype

    def _describe(self) -> None:
        s = self.sim
        desc = {"cells": list(s.n[:s.dims]), "dx": list(s.dx[:s.dims]), "dt": s.dt, "outputs": []}
        for r in self.reqs:
            d = {"name": r.name, "kind": r.kind, "every": r.every, "from": r.start, "to": r.stop,
                 "dtype": str(self._dtype(r)).replace("torch.", "")}
            if r.kind == "particles":
                d.update(species=r.species[0], cells={"lo": list(r.lo[:s.dims]), "hi": list(r.hi[:s.dims])},
                         subsample=r.subsample, record=[f"x{a}" for a in range(s.dims)] + ["u0", "u1", "u2", "w"])
            else:
                d.update(box={"lo": list(r.lo[:s.dims]), "hi": list(r.hi[:s.dims]), "stride": list(r.stride[:s.dims])},
                         components=r.components, positions={c: YEE_POSITION[c][:s.dims] for c in r.components},
                         layout="(component, z, y, x)" if s.dims == 3 else "(component, 1, y, x)")
                if r.kind == "density":
                    d["species"] = r.species
            desc["outputs"].append(d)
        with open(os.path.join(self.out, "outputs.json"), "w") as f:
            json.dump(desc, f, indent=1)

    def _slot(self, r: Request) -> _Slot:
        k = self.turn[r.name] % 2
        self.turn[r.name] += 1
        slot = self.slots[r.name][k]
        if slot is not None and slot.done is not None:
            slot.done.result()  # its previous write is finished (and re-raises its errors)
            slot.done = None
        if slot is None:
            if r.kind == "particles":
                cap = r.capacity or max(1, math.ceil(self.sim.species[r.species[0]].np / r.subsample))
                shape = (cap, self.sim.dims + 4)
            else:
                mx, my, mz = r.points()
                shape = (len(r.components), mz, my, mx)
            slot = _Slot(shape, self._dtype(r), self.sim.device)
            self.slots[r.name][k] = slot
        return slot

    def after_step(self, step: int | None = None) -> int:
        """Extract and queue every output that fires at this step (default: the
        simulation's step count).  Returns the number queued."""
        step = self.sim.step_count if step is None else int(step)
        fired = [r for r in self.reqs if r.fires(step)]
        for r in fired:
            self._emit(r, step)
        return len(fired)

    def _emit(self, r: Request, step: int) -> None:
        import torch
        s = self.sim
        slot = self._slot(r)
        b = s.box(r.lo, r.hi, r.stride)
        begin = torch.cuda.Event(enable_timing=True)
        begin.record(torch.cuda.current_stream(s.device))
        if r.kind == "fields":
            s.extract_grid([s.fields[COMPONENTS[c][0]][COMPONENTS[c][1]] for c in r.components], b, out=slot.dev)
        elif r.kind == "density":
            rho = self.rho.get(r.name)
            if rho is None:
                rho = self.rho[r.name] = torch.empty(s.ncells, dtype=torch.float64, device=s.device)
            s.charge_density_into(rho, [s.species[i] for i in r.species])
            s.extract_grid([rho], b, out=slot.dev)
        else:
            s.extract_particles(s.species[r.species[0]], b, r.subsample, slot.dev, slot.count_dev)
        ready = torch.cuda.Event(enable_timing=True)
        ready.record(torch.cuda.current_stream(s.device))
        self.marks.append((begin, ready))
        self.copy_stream.wait_event(ready)
        with torch.cuda.stream(self.copy_stream):
            if r.kind == "particles":
                slot.count_host.copy_(slot.count_dev, non_blocking=True)
            else:
                slot.host.copy_(slot.dev, non_blocking=True)
            copied = torch.cuda.Event()
            copied.record(self.copy_stream)
        slot.done = self.pool.submit(self._write, r, slot, step, copied)

    def _write(self, r: Request, slot: _Slot, step: int, copied) -> None:
        import torch
        copied.synchronize()
        line = {"step": step, "time": step * self.sim.dt}
        if r.kind == "particles":
            n = int(slot.count_host[0])
            k = min(n, slot.dev.shape[0])
            if k:  # the selection finished before its count was copied; fetch the k records
                with torch.cuda.stream(self.read_stream):
                    slot.host[:k].copy_(slot.dev[:k], non_blocking=True)
                    fetched = torch.cuda.Event()
                    fetched.record(self.read_stream)
                fetched.synchronize()
            arr = slot.host[:k].numpy()
            line.update(count=n, truncated=n > k)
        else:
            arr = slot.host.numpy()
        rel = f"{step:08d}.npy"
        np.save(os.path.join(self.out, r.name, rel), arr)
        line.update(file=rel, shape=list(arr.shape))
        with self.lock:
            with open(os.path.join(self.out, r.name, "index.jsonl"), "a") as f:
                f.write(json.dumps(line) + "\n")
            self.files += 1

    def flush(self) -> None:
        """Wait until every queued output is on disk."""
        for pair in self.slots.values():
            for slot in pair:
                if slot is not None and slot.done is not None:
                    slot.done.result()
                    slot.done = None

    def extraction_ms(self) -> tuple:
        """Milliseconds the extractions took on the step's stream (density
        deposits included) and their count, since the last call
        (synchronising)."""
        total = 0.0
        for a, b in self.marks:
            b.synchronize()
            total += a.elapsed_time(b)
        n = len(self.marks)
        self.marks = []
        return total, n

    def close(self) -> None:
        self.flush()
        self.pool.shutdown(wait=True)
