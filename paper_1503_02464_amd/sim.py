"""Python face of the PIC library: torch tensors own the device memory, the
library does every step of the computation.  This module only marshals
arguments (pointers, sizes, the current HIP stream) and converts the
per-dimension (cell, offset) particle form to the packed cell index."""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L


def _ptr(t: torch.Tensor) -> int:
    return t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def pack_cells(cell: np.ndarray, bits: tuple) -> np.ndarray:
    """Per-dimension cell indices (3, np) -> packed int32: ix | iy << bx | iz << (bx + by)."""
    c = np.asarray(cell, np.int64)
    packed = c[0] | (c[1] << bits[0]) | (c[2] << (bits[0] + bits[1]))
    return packed.astype(np.uint32).view(np.int32)


def unpack_cells(packed: np.ndarray, bits: tuple) -> np.ndarray:
    p = np.asarray(packed).view(np.uint32).astype(np.int64)
    b0, b1, b2 = bits
    out = np.zeros((3, p.shape[0]), np.int32)
    out[0] = p & ((1 << b0) - 1)
    out[1] = (p >> b0) & ((1 << b1) - 1)
    out[2] = (p >> (b0 + b1)) & ((1 << b2) - 1)
    return out


def cell_bits(n: tuple, dims: int) -> tuple:
    """Bits per dimension of the packed cell index: ceil(log2(n_d))."""
    return tuple(int(np.ceil(np.log2(n[d]))) if d < dims and n[d] > 1 else 0 for d in range(3))


@dataclass
class SpeciesState:
    """Device arrays of one species (two sets for the out-of-place sort)."""

    q: float
    m: float
    np: int
    sets: list  # two dicts: cell (int32), off (3 tensors), u (3 tensors), w
    tile_start: torch.Tensor
    struct: L.Species

    def current(self) -> dict:
        """The set the struct's primary pointers name (after sorts swapped them)."""
        for s in self.sets:
            if _ptr(s["cell"]) == self.struct.cell:
                return s
        raise RuntimeError("species pointers out of sync")


class Simulation:
    """One periodic box: grid parameters, E/B/J, workspace and species.

    dims 2 or 3; n cells per dim (n[2] = 1 in 2D); dx spacings; dt step;
    order 1 (linear) or 2 (quadratic); precision "fp32" or "fp64"; tile cells
    per sort tile; slack guard cells; sort_every steps between sorts;
    current_accum the LDS current accumulation type ("auto": fix64 for an
    fp32 state, fp64 for an fp64 state; "fp64", "fix64", "fp32"); open_x
    opens the x faces (Mur fields, particles removed outside
    [absorb, n0 - absorb) cells); sort_levels the levels per tile of the sort
    (0: the library's default)."""

    def __init__(self, dims: int, n: tuple, dx: tuple, dt: float, order: int, precision: str = "fp32",
                 tile: tuple = (8, 8, 8), slack: int = 1, sort_every: int = 4, max_particles: int = 0,
                 current_accum: str = "auto", open_x: bool = False, absorb: int = 0, sort_levels: int = 0,
                 device: str = "cuda", field_sets: int = 2):
        self.lib = L.load()
        self.dims = dims
        self.n = tuple(int(v) for v in n) + (1,) * (3 - len(n))
        self.dx = tuple(float(v) for v in dx) + (1.0,) * (3 - len(dx))
        self.dt = float(dt)
        self.order = order
        self.precision = precision
        self.dtype = torch.float32 if precision == "fp32" else torch.float64
        self.device = torch.device(device)
        tile = tuple(tile) + (1,) * (3 - len(tile))
        if dims == 2:
            tile = (tile[0], tile[1], 1)
        p = L.Params()
        p.dims = dims
        p.n = L._c3i(*self.n)
        p.dx = L._c3d(*self.dx)
        p.dt = self.dt
        p.shape_order = order
        p.precision = L.PIC_FP32 if precision == "fp32" else L.PIC_FP64
        p.tile = L._c3i(*tile)
        p.slack = slack
        p.sort_every = sort_every
        self.sort_every = int(sort_every)
        p.max_particles = int(max_particles)
        p.current_accum = {"auto": L.PIC_ACC_AUTO, "fp32": L.PIC_ACC_FP32, "fp64": L.PIC_ACC_FP64,
                           "fix64": L.PIC_ACC_FIX64}[current_accum]
        p.open_x = 1 if open_x else 0
        p.absorb = int(absorb)
        p.sort_levels = int(sort_levels)
        self.open_x = bool(open_x)
        self.absorb = int(absorb)
        self.params = p
        ctx = ctypes.c_void_p()
        st = self.lib.pic_init(ctypes.byref(p), ctypes.byref(ctx))
        L.check(self.lib, None, st, "pic_init")
        self.ctx = ctx
        nbytes = self.lib.pic_workspace_bytes(ctx)
        # 256-byte aligned workspace carved from a torch allocation
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = _ptr(self._ws)
        aligned = (base + 255) & ~255
        self._call(self.lib.pic_set_workspace(ctx, ctypes.c_void_p(aligned), nbytes), "pic_set_workspace")
        self.ncells = self.n[0] * self.n[1] * self.n[2]
        self.fields = {k: [torch.zeros(self.ncells, dtype=self.dtype, device=self.device) for _ in range(3)]
                       for k in ("E", "B", "J")}
        self.fstruct = L.Fields()
        for k in ("E", "B", "J"):
            setattr(self.fstruct, k, L._c3p(*[_ptr(t) for t in self.fields[k]]))
        # a second E, B set lets the library run the Yee step in one pass and swap the sets
        self._field_pool = {}
        if field_sets == 2:
            self.fields_alt = {k: [torch.zeros(self.ncells, dtype=self.dtype, device=self.device) for _ in range(3)]
                               for k in ("E", "B")}
            for k in ("E", "B"):
                setattr(self.fstruct, k + "_alt", L._c3p(*[_ptr(t) for t in self.fields_alt[k]]))
            for k in ("E", "B"):
                for t in self.fields[k] + self.fields_alt[k]:
                    self._field_pool[_ptr(t)] = t
        bits = (ctypes.c_int32 * 3)()
        self.lib.pic_cell_bits(ctx, bits)
        self.bits = tuple(bits)
        self.ntiles = int(self.lib.pic_num_tiles(ctx))
        self.species: list = []

    # -- plumbing ---------------------------------------------------------
    def _call(self, status: int, what: str) -> None:
        L.check(self.lib, self.ctx, status, what)

    def _sync_fields(self) -> None:
        """Follow the library's swaps of the two E, B sets: self.fields names
        the tensors the struct's current pointers name."""
        if not self._field_pool:
            return
        for k in ("E", "B"):
            cur = [self._field_pool[p] for p in getattr(self.fstruct, k)]
            alt = [self._field_pool[p] for p in getattr(self.fstruct, k + "_alt")]
            self.fields[k], self.fields_alt[k] = cur, alt

    def close(self) -> None:
        if getattr(self, "ctx", None):
            torch.cuda.synchronize()
            self.lib.pic_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- data in / out ----------------------------------------------------
    def pack_cells(self, cell: np.ndarray) -> np.ndarray:
        return pack_cells(cell, self.bits)

    def unpack_cells(self, packed: np.ndarray) -> np.ndarray:
        return unpack_cells(packed, self.bits)

    def set_fields(self, E=None, B=None, J=None) -> None:
        for k, v in (("E", E), ("B", B), ("J", J)):
            if v is None:
                continue
            for d in range(3):
                self.fields[k][d].copy_(torch.as_tensor(np.asarray(v[d]), dtype=self.dtype))

    def get_fields(self) -> dict:
        torch.cuda.synchronize()
        return {k: np.stack([t.double().cpu().numpy() for t in v]) for k, v in self.fields.items()}

    def add_species(self, sp: dict, capacity: int | None = None) -> SpeciesState:
        """Upload a species given as numpy arrays (per-dimension cells, offsets,
        momenta, weights; see paper_1503_02464_amd.inputs)."""
        npart = int(sp["w"].shape[0])
        cap = max(npart, capacity or 0, 1)
        dev, dt = self.device, self.dtype
        sets = []
        for _ in range(2):
            sets.append({
                "cell": torch.zeros(cap, dtype=torch.int32, device=dev),
                "off": [torch.zeros(cap, dtype=dt, device=dev) for _ in range(3)],
                "u": [torch.zeros(cap, dtype=dt, device=dev) for _ in range(3)],
                "w": torch.zeros(cap, dtype=dt, device=dev),
            })
        s0 = sets[0]
        if npart:
            s0["cell"][:npart].copy_(torch.from_numpy(self.pack_cells(sp["cell"])))
            for d in range(3):
                s0["off"][d][:npart].copy_(torch.as_tensor(sp["off"][d], dtype=dt))
                s0["u"][d][:npart].copy_(torch.as_tensor(sp["u"][d], dtype=dt))
            s0["w"][:npart].copy_(torch.as_tensor(sp["w"], dtype=dt))
        tile_start = torch.zeros(self.ntiles + 1, dtype=torch.int32, device=dev)
        st = L.Species()
        st.np = npart
        st.q = float(sp["q"])
        st.m = float(sp["m"])
        self._fill_struct(st, sets[0], sets[1])
        st.tile_start = _ptr(tile_start)
        st.sorted = 0
        state = SpeciesState(float(sp["q"]), float(sp["m"]), npart, sets, tile_start, st)
        self.species.append(state)
        return state

    def new_species(self, q: float, m: float, npart: int) -> SpeciesState:
        """A species of npart particles whose device arrays (state.sets[0], in
        the packed-cell form) the caller fills, e.g. with a device-side
        generator; the second set receives the sorts."""
        dev, dt = self.device, self.dtype
        cap = max(int(npart), 1)
        sets = [{"cell": torch.zeros(cap, dtype=torch.int32, device=dev),
                 "off": [torch.zeros(cap, dtype=dt, device=dev) for _ in range(3)],
                 "u": [torch.zeros(cap, dtype=dt, device=dev) for _ in range(3)],
                 "w": torch.zeros(cap, dtype=dt, device=dev)} for _ in range(2)]
        tile_start = torch.zeros(self.ntiles + 1, dtype=torch.int32, device=dev)
        st = L.Species()
        st.np = int(npart)
        st.q = float(q)
        st.m = float(m)
        self._fill_struct(st, sets[0], sets[1])
        st.tile_start = _ptr(tile_start)
        st.sorted = 0
        state = SpeciesState(float(q), float(m), int(npart), sets, tile_start, st)
        self.species.append(state)
        return state

    @staticmethod
    def _fill_struct(st: L.Species, a: dict, b: dict) -> None:
        st.cell = _ptr(a["cell"])
        st.off = L._c3p(*[_ptr(t) for t in a["off"]])
        st.u = L._c3p(*[_ptr(t) for t in a["u"]])
        st.w = _ptr(a["w"])
        st.cell_alt = _ptr(b["cell"])
        st.off_alt = L._c3p(*[_ptr(t) for t in b["off"]])
        st.u_alt = L._c3p(*[_ptr(t) for t in b["u"]])
        st.w_alt = _ptr(b["w"])

    def get_species(self, s: SpeciesState) -> dict:
        torch.cuda.synchronize()
        cur = s.current()
        n = s.np
        out = {"q": s.q, "m": s.m,
               "cell": self.unpack_cells(cur["cell"][:n].cpu().numpy()),
               "off": np.stack([t[:n].double().cpu().numpy() for t in cur["off"]]),
               "u": np.stack([t[:n].double().cpu().numpy() for t in cur["u"]]),
               "w": cur["w"][:n].double().cpu().numpy()}
        if self.dims == 2:
            out["off"][2] = 0.0
        return out

    def tile_start(self, s: SpeciesState) -> np.ndarray:
        torch.cuda.synchronize()
        return s.tile_start.cpu().numpy().astype(np.int64)

    # -- the hot path -----------------------------------------------------
    def gather_push(self, s: SpeciesState) -> None:
        self._call(self.lib.pic_gather_push(self.ctx, ctypes.byref(s.struct), ctypes.byref(self.fstruct),
                                            ctypes.c_void_p(_stream())), "pic_gather_push")

    def deposit(self, s: SpeciesState) -> None:
        self._call(self.lib.pic_deposit(self.ctx, ctypes.byref(s.struct), ctypes.byref(self.fstruct),
                                        ctypes.c_void_p(_stream())), "pic_deposit")

    def zero_current(self) -> None:
        self._call(self.lib.pic_zero_current(self.ctx, ctypes.byref(self.fstruct), ctypes.c_void_p(_stream())),
                   "pic_zero_current")

    def yee_step(self) -> None:
        try:
            self._call(self.lib.pic_yee_step(self.ctx, ctypes.byref(self.fstruct), ctypes.c_void_p(_stream())),
                       "pic_yee_step")
        finally:
            self._sync_fields()

    def set_laser(self, plane: int, e0: float, omega: float = 1.0, w0: float = 1e30, tau: float = 1e30,
                  t0: float = 0.0, yc: float = 0.0, zc: float = 0.0, pol: int = 1) -> None:
        """Register the laser current sheet that every step adds (open x only)."""
        las = L.Laser(plane=int(plane), pol=int(pol), e0=float(e0), omega=float(omega), w0=float(w0), tau=float(tau),
                      t0=float(t0), yc=float(yc), zc=float(zc))
        self._call(self.lib.pic_set_laser(self.ctx, ctypes.byref(las)), "pic_set_laser")

    def laser_current(self, t: float) -> None:
        """J += the registered laser sheet at time t."""
        self._call(self.lib.pic_laser_current(self.ctx, ctypes.byref(self.fstruct), float(t),
                                              ctypes.c_void_p(_stream())), "pic_laser_current")

    def live(self, s: SpeciesState) -> torch.Tensor:
        """Mask of the particles not removed at an open face (weight != 0)."""
        return s.current()["w"][:s.np] != 0

    def sort(self, s: SpeciesState) -> None:
        try:
            self._call(self.lib.pic_sort(self.ctx, ctypes.byref(s.struct), ctypes.c_void_p(_stream())), "pic_sort")
        finally:  # with open x faces the sort drops the removed particles
            s.np = int(s.struct.np)

    def step(self, nsteps: int = 1, species: list | None = None) -> None:
        sp = species if species is not None else self.species
        arr = (L.Species * max(len(sp), 1))()
        for i, s in enumerate(sp):
            arr[i] = s.struct
        try:
            self._call(self.lib.pic_step(self.ctx, arr, len(sp), ctypes.byref(self.fstruct), int(nsteps),
                                         ctypes.c_void_p(_stream())), "pic_step")
        finally:  # also after a failure: the library may have swapped sets, dropped removed
            for i, s in enumerate(sp):  # particles or cleared sorted
                s.struct = arr[i]
                s.np = int(arr[i].np)
            self._sync_fields()

    def diagnostics(self, species: list | None = None) -> dict:
        sp = species if species is not None else self.species
        arr = (L.Species * max(len(sp), 1))()
        for i, s in enumerate(sp):
            arr[i] = s.struct
        out = (ctypes.c_double * L.PIC_NDIAG)()
        self._call(self.lib.pic_diagnostics(self.ctx, arr, len(sp), ctypes.byref(self.fstruct), out,
                                            ctypes.c_void_p(_stream())), "pic_diagnostics")
        keys = ("UE", "UB", "K", "Q", "rho_max", "gauss_max", "gauss_change", "continuity")
        return dict(zip(keys, list(out)))

    def charge_density(self, species: list | None = None, gauss: bool = False):
        """The FP64 charge density on the nodes (and div E - rho when gauss),
        computed by the library into device grids; returns numpy arrays."""
        sp = species if species is not None else self.species
        arr = (L.Species * max(len(sp), 1))()
        for i, s in enumerate(sp):
            arr[i] = s.struct
        rho = torch.empty(self.ncells, dtype=torch.float64, device=self.device)
        g = torch.empty(self.ncells, dtype=torch.float64, device=self.device) if gauss else None
        self._call(self.lib.pic_charge_density(self.ctx, arr, len(sp), ctypes.byref(self.fstruct),
                                               ctypes.c_void_p(_ptr(rho)),
                                               ctypes.c_void_p(_ptr(g) if g is not None else None),
                                               ctypes.c_void_p(_stream())), "pic_charge_density")
        torch.cuda.synchronize()
        return (rho.cpu().numpy(), g.cpu().numpy()) if gauss else rho.cpu().numpy()

    # -- outputs: device-side extraction (pic_extract_grid / _particles) ----
    def box(self, lo=None, hi=None, stride=None) -> L.Box:
        """A pic_box over this grid (defaults: the whole grid, stride 1)."""
        lo = tuple(int(v) for v in lo) + (0, 0, 0)[len(lo):] if lo is not None else (0, 0, 0)
        hi = tuple(int(v) for v in hi) + (1, 1, 1)[len(hi):] if hi is not None else self.n
        stride = tuple(int(v) for v in stride) + (1, 1, 1)[len(stride):] if stride is not None else (1, 1, 1)
        if self.dims == 2:
            lo, hi = (lo[0], lo[1], 0), (hi[0], hi[1], 1)
        return L.Box(lo=L._c3i(*lo), hi=L._c3i(*hi), stride=L._c3i(*stride))

    @staticmethod
    def box_shape(b: L.Box) -> tuple:
        """Points per axis of a box, (m_x, m_y, m_z)."""
        return tuple(max(0, -(-(b.hi[d] - b.lo[d]) // b.stride[d])) for d in range(3))

    def extract_grid(self, grids: list, b: L.Box, out: torch.Tensor | None = None) -> torch.Tensor:
        """The values of device grids (tensors of ncells elements, one dtype)
        at the box's points, packed as (len(grids), m_z, m_y, m_x) into a device
        tensor; enqueued on the current stream, not synchronised."""
        mx, my, mz = self.box_shape(b)
        shape = (len(grids), mz, my, mx)
        dtype = grids[0].dtype
        for t in grids:  # the library reads n0 n1 n2 elements of one size from each pointer
            if t.dtype != dtype or t.numel() != self.ncells or not t.is_contiguous() or not t.is_cuda:
                raise ValueError("grids must be contiguous device tensors of ncells elements of one dtype")
        if out is not None and (out.dtype != dtype or out.numel() < len(grids) * mx * my * mz or not out.is_contiguous()):
            raise ValueError("out must be a contiguous tensor of the grids' dtype holding every extracted value")
        if out is None:
            out = torch.empty(shape, dtype=dtype, device=self.device)
        arr = (ctypes.c_void_p * len(grids))(*[_ptr(g) for g in grids])
        self._call(self.lib.pic_extract_grid(self.ctx, arr, len(grids), grids[0].element_size(), ctypes.byref(b),
                                             ctypes.c_void_p(_ptr(out)), ctypes.c_void_p(_stream())),
                   "pic_extract_grid")
        return out

    def extract_particles(self, s: SpeciesState, cells: L.Box, every: int, out: torch.Tensor,
                          count: torch.Tensor) -> None:
        """Phase-space records (dims + 4 values each) of the species' particles
        in the cell box, every every-th in storage order, into out (a device
        tensor of capacity x (dims + 4) values of the state's dtype); the
        number selected goes to count (a device int64 tensor of one element).
        Enqueued on the current stream, not synchronised."""
        rec = self.dims + 4
        if out.dtype != self.dtype or out.numel() % rec != 0 or not out.is_contiguous() or not out.is_cuda:
            raise ValueError(f"out must be a contiguous device tensor of records of {rec} {self.dtype} values")
        if count.dtype != torch.int64 or count.numel() < 1 or not count.is_cuda:
            raise ValueError("count must be a device int64 tensor")
        self._call(self.lib.pic_extract_particles(self.ctx, ctypes.byref(s.struct), ctypes.byref(cells), int(every),
                                                  ctypes.c_void_p(_ptr(out)), out.numel() // rec,
                                                  ctypes.c_void_p(_ptr(count)), ctypes.c_void_p(_stream())),
                   "pic_extract_particles")

    def charge_density_into(self, rho: torch.Tensor, species: list | None = None) -> None:
        """The FP64 charge density of the given species into the device grid
        rho (pic_charge_density), enqueued on the current stream."""
        sp = species if species is not None else self.species
        arr = (L.Species * max(len(sp), 1))()
        for i, s in enumerate(sp):
            arr[i] = s.struct
        self._call(self.lib.pic_charge_density(self.ctx, arr, len(sp), ctypes.byref(self.fstruct),
                                               ctypes.c_void_p(_ptr(rho)), ctypes.c_void_p(None),
                                               ctypes.c_void_p(_stream())), "pic_charge_density")

    def check(self) -> None:
        self._call(self.lib.pic_check(self.ctx, ctypes.c_void_p(_stream())), "pic_check")

    def set_timing(self, on: bool) -> None:
        self._call(self.lib.pic_set_timing(self.ctx, 1 if on else 0), "pic_set_timing")

    def get_timing(self) -> dict:
        ms = (ctypes.c_double * L.PIC_NPHASE)()
        cnt = (ctypes.c_int64 * L.PIC_NPHASE)()
        self._call(self.lib.pic_get_timing(self.ctx, ms, cnt, L.PIC_NPHASE), "pic_get_timing")
        return {name: (ms[i], cnt[i]) for i, name in enumerate(L.PHASES)}

    def straggler_count(self) -> int:
        """Particles the last fused launch sent to the HBM path (synchronises)."""
        n = ctypes.c_int64()
        self._call(self.lib.pic_straggler_count(self.ctx, ctypes.byref(n), ctypes.c_void_p(_stream())),
                   "pic_straggler_count")
        return int(n.value)

    @property
    def step_count(self) -> int:
        return int(self.lib.pic_step_count(self.ctx))
