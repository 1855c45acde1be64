"""FP64 CPU oracle of the explicit electromagnetic PIC step (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and its
Python binding) never imports, links or calls it.

The arithmetic lives in ``oracle.c`` (plain C, FP64, ``-O2 -ffp-contract=off``);
this module compiles it with gcc on first use and wraps it with ctypes.  Layouts:

* fields: dict with ``E``, ``B``, ``J`` -> float64 arrays of shape (3, N),
  N = n[0]*n[1]*n[2], x fastest; component positions on the Yee lattice as in
  the C header comment (paper Sec. 2, "FDTD scheme on the Yee lattice").
* species: dict with ``q``, ``m`` (floats), ``cell`` int32 (3, np) per-dimension
  cell indices, ``off`` float64 (3, np) offsets in [0,1), ``u`` float64 (3, np)
  momenta p/(m c) at n-1/2, ``w`` float64 (np,) macro-particle weights
  (paper Sec. 3.3: seven values per particle, x y z px py pz w).

Every function cites the passage of the paper it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fPIC", "-shared"]


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (no GPU involved)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_OMP_SRC = os.path.join(_HERE, "oracle_omp.c")
_OMP_LIB = os.path.join(_HERE, "liboracle_omp.so")
_omp_lib = None


def build_timing(force: bool = False) -> str:
    """Compile the all-core timing build (oracle_omp.c, which includes oracle.c
    unchanged) with OpenMP; used only to time the oracle on every host core."""
    newest = max(os.path.getmtime(_SRC), os.path.getmtime(_OMP_SRC))
    if force or not os.path.exists(_OMP_LIB) or os.path.getmtime(_OMP_LIB) < newest:
        tmp = _OMP_LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", *CFLAGS, "-fopenmp", "-o", tmp, _OMP_SRC, "-lm"])
        os.replace(tmp, _OMP_LIB)
    return _OMP_LIB


class _Grid(ctypes.Structure):
    _fields_ = [
        ("dims", ctypes.c_int32),
        ("n", ctypes.c_int32 * 3),
        ("dx", ctypes.c_double * 3),
        ("dt", ctypes.c_double),
        ("order", ctypes.c_int32),
    ]


_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int32)


def _bind(path: str):
    """Load a compiled oracle library and declare its C signatures."""
    lib = ctypes.CDLL(path)
    g = ctypes.POINTER(_Grid)
    lib.or_shape.argtypes = [ctypes.c_int32, ctypes.c_double]
    lib.or_shape.restype = ctypes.c_double
    lib.or_gather.argtypes = [g] + [_D] * 6 + [ctypes.c_int64] + [_I] * 3 + [_D] * 3 + [_D]
    lib.or_gather_bruteforce.argtypes = lib.or_gather.argtypes
    lib.or_boris.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_double, _D, _D, _D, _D]
    lib.or_move.argtypes = [g, ctypes.c_int64, _D, _D, _D, _I, _I, _I, _D, _D, _D, _I]
    lib.or_move.restype = ctypes.c_int64
    lib.or_deposit.argtypes = ([g, ctypes.c_double, ctypes.c_int64] + [_I] * 3 + [_D] * 3 + [_I]
                               + [_D] * 3 + [_D] * 3 + [_D] + [_D] * 3)
    lib.or_push_deposit.argtypes = ([g, ctypes.c_double, ctypes.c_double, ctypes.c_int64] + [_D] * 6
                                    + [_I] * 3 + [_D] * 3 + [_D] * 3 + [_D] + [_D] * 3)
    lib.or_push_deposit.restype = ctypes.c_int64
    lib.or_yee_b.argtypes = [g, ctypes.c_double] + [_D] * 6
    lib.or_yee_e.argtypes = [g] + [_D] * 9
    lib.or_yee_step.argtypes = [g] + [_D] * 9
    lib.or_yee_step_open.argtypes = [g] + [_D] * 9
    lib.or_laser_j0.argtypes = [g, ctypes.c_double, ctypes.c_double]
    lib.or_laser_j0.restype = ctypes.c_double
    lib.or_laser_add.argtypes = [g, _D, _D, ctypes.c_int32, ctypes.c_int32] + [ctypes.c_double] * 8
    lib.or_absorb.argtypes = [ctypes.c_int64, _I, ctypes.c_int32, ctypes.c_int32, _D]
    lib.or_absorb.restype = ctypes.c_int64
    lib.or_rho.argtypes = [g, ctypes.c_double, ctypes.c_int64] + [_I] * 3 + [_D] * 3 + [_D, _D]
    lib.or_div.argtypes = [g] + [_D] * 4
    lib.or_field_energy.argtypes = [g] + [_D] * 3
    lib.or_field_energy.restype = ctypes.c_double
    lib.or_kinetic_energy.argtypes = [ctypes.c_double, ctypes.c_int64] + [_D] * 4
    lib.or_kinetic_energy.restype = ctypes.c_double
    return lib


def _load():
    global _lib
    with _lock:
        if _lib is None:
            _lib = _bind(build())
    return _lib


class use_library:
    """Context manager: route every oracle call through another compiled copy
    of the oracle (used to check that the pins catch planted mistakes)."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib
        _load()
        self.saved = _lib
        _lib = _bind(self.path)
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


@dataclass(frozen=True)
class Grid:
    """Grid of the periodic box: ``dims`` in {2,3}, ``n`` cells, ``dx`` spacings,
    ``dt`` step and shape ``order`` (1 linear, 2 quadratic)."""

    dims: int
    n: tuple
    dx: tuple
    dt: float
    order: int

    @property
    def ncells(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    def c(self) -> _Grid:
        return _Grid(self.dims, (ctypes.c_int32 * 3)(*self.n), (ctypes.c_double * 3)(*self.dx), self.dt, self.order)


def _d(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous, (a.dtype, a.flags)
    return a.ctypes.data_as(_D)


def _i(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(_I)


def shape(order: int, xi: float) -> float:
    """B-spline shape S_m(xi) in cell units (paper Sec. 2: compact, positive g)."""
    return _load().or_shape(order, float(xi))


def new_fields(grid: Grid) -> dict:
    n = grid.ncells
    return {k: np.zeros((3, n), np.float64) for k in ("E", "B", "J")}


def copy_species(sp: dict) -> dict:
    out = dict(sp)
    for k in ("cell", "off", "u", "w"):
        out[k] = np.ascontiguousarray(np.array(sp[k], copy=True))
    return out


def gather(grid: Grid, E: np.ndarray, B: np.ndarray, cell: np.ndarray, off: np.ndarray, brute: bool = False):
    """E and B at each particle: shape-weighted average of the grid fields
    (paper Sec. 2, 'spatial average of the EM fields weighted with g').
    Returns (6, np) in the order Ex Ey Ez Bx By Bz."""
    lib = _load()
    np_ = cell.shape[1]
    out = np.zeros((6, np_), np.float64)
    E = np.ascontiguousarray(E, np.float64)
    B = np.ascontiguousarray(B, np.float64)
    cell = np.ascontiguousarray(cell, np.int32)
    off = np.ascontiguousarray(off, np.float64)
    fn = lib.or_gather_bruteforce if brute else lib.or_gather
    g = grid.c()
    fn(ctypes.byref(g), _d(E[0]), _d(E[1]), _d(E[2]), _d(B[0]), _d(B[1]), _d(B[2]), np_,
       _i(cell[0]), _i(cell[1]), _i(cell[2]), _d(off[0]), _d(off[1]), _d(off[2]), _d(out))
    return out


def boris(q: float, m: float, dt: float, EB: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Relativistic Boris rotation u^{n-1/2} -> u^{n+1/2} (paper Sec. 2, eq. 3
    advanced with leap-frog and the Boris pusher, ref. [8])."""
    lib = _load()
    u = np.ascontiguousarray(np.array(u, np.float64, copy=True))
    EB = np.ascontiguousarray(EB, np.float64)
    lib.or_boris(u.shape[1], q, m, dt, _d(EB), _d(u[0]), _d(u[1]), _d(u[2]))
    return u


def move(grid: Grid, u: np.ndarray, cell: np.ndarray, off: np.ndarray):
    """x^{n+1} = x^n + dt v^{n+1/2} (paper eq. 3, dr/dt = v), renormalised to
    cell + offset.  Returns (cell, off, dcell, n_bad)."""
    lib = _load()
    cell = np.ascontiguousarray(np.array(cell, np.int32, copy=True))
    off = np.ascontiguousarray(np.array(off, np.float64, copy=True))
    u = np.ascontiguousarray(u, np.float64)
    np_ = cell.shape[1]
    dc = np.zeros((3, np_), np.int32)
    g = grid.c()
    bad = lib.or_move(ctypes.byref(g), np_, _d(u[0]), _d(u[1]), _d(u[2]), _i(cell[0]), _i(cell[1]), _i(cell[2]),
                      _d(off[0]), _d(off[1]), _d(off[2]), _i(dc))
    return cell, off, dc, int(bad)


def deposit(grid: Grid, q: float, cell0, off0, dcell, off1, u, w, J: np.ndarray) -> None:
    """Charge-conserving current J^{n+1/2} += Esirkepov(x^n -> x^{n+1})
    (paper eq. 4 and Sec. 2 'enforcing the continuity equation'; method of
    Esirkepov, CPC 135 (2001) 144).  J is updated in place."""
    lib = _load()
    c0 = np.ascontiguousarray(cell0, np.int32)
    o0 = np.ascontiguousarray(off0, np.float64)
    dc = np.ascontiguousarray(dcell, np.int32)
    o1 = np.ascontiguousarray(off1, np.float64)
    u = np.ascontiguousarray(u, np.float64)
    w = np.ascontiguousarray(w, np.float64)
    assert J.dtype == np.float64 and J.flags.c_contiguous
    g = grid.c()
    lib.or_deposit(ctypes.byref(g), q, c0.shape[1], _i(c0[0]), _i(c0[1]), _i(c0[2]), _d(o0[0]), _d(o0[1]),
                   _d(o0[2]), _i(dc), _d(o1[0]), _d(o1[1]), _d(o1[2]), _d(u[0]), _d(u[1]), _d(u[2]), _d(w),
                   _d(J[0]), _d(J[1]), _d(J[2]))


def push_deposit(grid: Grid, fields: dict, sp: dict) -> int:
    """Gather, Boris, move and deposit for one species, in place (paper Sec. 2)."""
    lib = _load()
    E, B, J = fields["E"], fields["B"], fields["J"]
    c, o, u, w = sp["cell"], sp["off"], sp["u"], sp["w"]
    g = grid.c()
    bad = lib.or_push_deposit(ctypes.byref(g), sp["q"], sp["m"], c.shape[1], _d(E[0]), _d(E[1]), _d(E[2]),
                              _d(B[0]), _d(B[1]), _d(B[2]), _i(c[0]), _i(c[1]), _i(c[2]), _d(o[0]), _d(o[1]),
                              _d(o[2]), _d(u[0]), _d(u[1]), _d(u[2]), _d(w), _d(J[0]), _d(J[1]), _d(J[2]))
    return int(bad)


def push_deposit_threads(grid: Grid, fields: dict, sp: dict, threads: int) -> int:
    """push_deposit on `threads` OpenMP threads (the all-core timing build):
    contiguous particle chunks per thread, private current grids added in thread
    order.  For timing the oracle on every host core, not for parity."""
    global _omp_lib
    with _lock:
        if _omp_lib is None:
            _omp_lib = _bind(build_timing())
            _omp_lib.or_push_deposit_omp.argtypes = _omp_lib.or_push_deposit.argtypes + [ctypes.c_int32]
            _omp_lib.or_push_deposit_omp.restype = ctypes.c_int64
    E, B, J = fields["E"], fields["B"], fields["J"]
    c, o, u, w = sp["cell"], sp["off"], sp["u"], sp["w"]
    g = grid.c()
    bad = _omp_lib.or_push_deposit_omp(ctypes.byref(g), sp["q"], sp["m"], c.shape[1], _d(E[0]), _d(E[1]), _d(E[2]),
                                       _d(B[0]), _d(B[1]), _d(B[2]), _i(c[0]), _i(c[1]), _i(c[2]), _d(o[0]),
                                       _d(o[1]), _d(o[2]), _d(u[0]), _d(u[1]), _d(u[2]), _d(w), _d(J[0]), _d(J[1]),
                                       _d(J[2]), int(threads))
    if bad < 0:
        raise MemoryError("oracle timing build: no memory for the per-thread current grids")
    return int(bad)


def step_threads(grid: Grid, fields: dict, species: list, threads: int) -> int:
    """step() with the particles on `threads` threads (Yee stays serial: it is
    under one percent of the oracle's step)."""
    fields["J"][...] = 0.0
    bad = 0
    for sp in species:
        bad += push_deposit_threads(grid, fields, sp, threads)
    yee_step(grid, fields)
    return bad


def yee_b(grid: Grid, f: float, E: np.ndarray, B: np.ndarray) -> None:
    """B -= f dt curl E (paper Sec. 2, dB/dt = -curl E, Yee lattice [9])."""
    g = grid.c()
    _load().or_yee_b(ctypes.byref(g), f, _d(E[0]), _d(E[1]), _d(E[2]), _d(B[0]), _d(B[1]), _d(B[2]))


def yee_e(grid: Grid, B: np.ndarray, J: np.ndarray, E: np.ndarray) -> None:
    """E += dt (curl B - J) (paper Sec. 2, dE/dt = curl B - J)."""
    g = grid.c()
    _load().or_yee_e(ctypes.byref(g), _d(B[0]), _d(B[1]), _d(B[2]), _d(J[0]), _d(J[1]), _d(J[2]),
                     _d(E[0]), _d(E[1]), _d(E[2]))


def yee_step(grid: Grid, fields: dict) -> None:
    """B^{n+1/2}, E^{n+1}, B^{n+1} from E^n, B^n, J^{n+1/2}."""
    yee_b(grid, 0.5, fields["E"], fields["B"])
    yee_e(grid, fields["B"], fields["J"], fields["E"])
    yee_b(grid, 0.5, fields["E"], fields["B"])


def yee_step_open(grid: Grid, fields: dict) -> None:
    """The Yee step with open (first-order Mur) x faces, periodic y and z."""
    E, B, J = fields["E"], fields["B"], fields["J"]
    _load().or_yee_step_open(grid.c(), _d(E[0]), _d(E[1]), _d(E[2]), _d(B[0]), _d(B[1]), _d(B[2]),
                             _d(J[0]), _d(J[1]), _d(J[2]))


@dataclass
class Laser:
    """A laser current sheet on the node plane x = plane * dx (readings: see
    or_laser_add).  pol 1 = E_y, 2 = E_z; w0 is the 1/e field radius, tau the
    FWHM of the intensity envelope, t0 its centre, (yc, zc) the axis."""

    plane: int
    e0: float
    omega: float = 1.0
    w0: float = 1e30
    tau: float = 1e30
    t0: float = 0.0
    yc: float = 0.0
    zc: float = 0.0
    pol: int = 1


def laser_j0(grid: Grid, e0: float, omega: float) -> float:
    return _load().or_laser_j0(grid.c(), e0, omega)


def laser_add(grid: Grid, J: np.ndarray, laser: Laser, t: float) -> None:
    _load().or_laser_add(grid.c(), _d(J[1]), _d(J[2]), laser.plane, laser.pol, laser.e0, laser.omega, laser.w0,
                         laser.tau, laser.t0, laser.yc, laser.zc, t)


def absorb(sp: dict, lo: int, hi: int) -> int:
    """Mark particles whose x cell left [lo, hi) as removed (w = 0)."""
    ix = np.ascontiguousarray(sp["cell"][0], np.int32)
    return _load().or_absorb(sp["w"].shape[0], _i(ix), lo, hi, _d(sp["w"]))


def compact(sp: dict) -> dict:
    """Drop removed (w == 0) particles."""
    keep = sp["w"] != 0.0
    return {"q": sp["q"], "m": sp["m"], "cell": sp["cell"][:, keep].copy(), "off": sp["off"][:, keep].copy(),
            "u": sp["u"][:, keep].copy(), "w": sp["w"][keep].copy()}


def step_open(grid: Grid, fields: dict, species: list, lo: int, hi: int, laser: Laser | None = None,
              n: int = 0) -> tuple:
    """One step of a box with open x faces (step number n, J at t = (n + 1/2) dt):
    J = 0; every species pushed and deposited; the laser sheet added; particles
    whose x cell left [lo, hi) removed; the Yee step with Mur faces.  Returns
    (species with the removed particles dropped, count of moves > 1 cell,
    removed count)."""
    fields["J"][...] = 0.0
    bad = 0
    for sp in species:
        bad += push_deposit(grid, fields, sp)
    if laser is not None:
        laser_add(grid, fields["J"], laser, (n + 0.5) * grid.dt)
    removed = 0
    out = []
    for sp in species:
        removed += absorb(sp, lo, hi)
        out.append(compact(sp))
    yee_step_open(grid, fields)
    return out, bad, removed


def step(grid: Grid, fields: dict, species: list) -> int:
    """One full PIC step in place: J = 0, then for every species gather, Boris,
    move and deposit; then the Yee update.  Returns the count of particles that
    moved more than one cell (must be zero under the stability condition)."""
    fields["J"][...] = 0.0
    bad = 0
    for sp in species:
        bad += push_deposit(grid, fields, sp)
    yee_step(grid, fields)
    return bad


def rho(grid: Grid, species: list) -> np.ndarray:
    """Charge density on nodes, sum over particles of q w/dV S(x - node)."""
    out = np.zeros(grid.ncells, np.float64)
    g = grid.c()
    for sp in species:
        c = np.ascontiguousarray(sp["cell"], np.int32)
        o = np.ascontiguousarray(sp["off"], np.float64)
        w = np.ascontiguousarray(sp["w"], np.float64)
        _load().or_rho(ctypes.byref(g), sp["q"], c.shape[1], _i(c[0]), _i(c[1]), _i(c[2]), _d(o[0]), _d(o[1]),
                       _d(o[2]), _d(w), _d(out))
    return out


def div(grid: Grid, F: np.ndarray) -> np.ndarray:
    """Backward-difference divergence of an E-staggered field, on nodes."""
    out = np.zeros(grid.ncells, np.float64)
    g = grid.c()
    F = np.ascontiguousarray(F, np.float64)
    _load().or_div(ctypes.byref(g), _d(F[0]), _d(F[1]), _d(F[2]), _d(out))
    return out


def field_energy(grid: Grid, F: np.ndarray) -> float:
    g = grid.c()
    F = np.ascontiguousarray(F, np.float64)
    return float(_load().or_field_energy(ctypes.byref(g), _d(F[0]), _d(F[1]), _d(F[2])))


def kinetic_energy(sp: dict) -> float:
    u = np.ascontiguousarray(sp["u"], np.float64)
    w = np.ascontiguousarray(sp["w"], np.float64)
    return float(_load().or_kinetic_energy(sp["m"], u.shape[1], _d(u[0]), _d(u[1]), _d(u[2]), _d(w)))


def diagnostics(grid: Grid, fields: dict, species: list) -> dict:
    """FP64 energies and charge: U_E, U_B, K, Q, rho, Gauss residual div E - rho."""
    r = rho(grid, species)
    return {
        "UE": field_energy(grid, fields["E"]),
        "UB": field_energy(grid, fields["B"]),
        "K": sum(kinetic_energy(sp) for sp in species),
        "Q": float(sum(sp["q"] * np.sum(sp["w"]) for sp in species)),
        "rho": r,
        "gauss": div(grid, fields["E"]) - r,
    }


def tile_keys(grid: Grid, tile: tuple, cell: np.ndarray) -> np.ndarray:
    """Tile index of each particle's cell, tiles numbered x fastest."""
    ntx = grid.n[0] // tile[0]
    nty = grid.n[1] // tile[1]
    tz = cell[2] // tile[2] if grid.dims == 3 else np.zeros_like(cell[0])
    return (cell[0] // tile[0] + ntx * (cell[1] // tile[1] + nty * tz)).astype(np.int64)


def tile_sort(grid: Grid, tile: tuple, sp: dict) -> tuple:
    """Stable counting sort of a species by tile key.  Returns the sorted species
    and the tile start offsets (length ntiles + 1)."""
    keys = tile_keys(grid, tile, sp["cell"])
    ntiles = (grid.n[0] // tile[0]) * (grid.n[1] // tile[1]) * (grid.n[2] // tile[2])
    order = np.argsort(keys, kind="stable")
    out = dict(sp)
    for k in ("cell", "off", "u"):
        out[k] = np.ascontiguousarray(sp[k][:, order])
    out["w"] = np.ascontiguousarray(sp["w"][order])
    counts = np.bincount(keys, minlength=ntiles)
    start = np.zeros(ntiles + 1, np.int64)
    start[1:] = np.cumsum(counts)
    return out, start


# ---- Outputs (paper Sec. 3.1: reduced-dimension outputs, e.g. a plane of a
# 3D box or a line of a 2D one, and subdomain outputs, e.g. a small box in a
# large one).  Plain definitions by indexing, for the output extraction.

def box_axes(lo, hi, stride) -> list:
    """Selected indices per dimension: lo[d], lo[d] + stride[d], ... below hi[d]."""
    return [np.arange(lo[d], hi[d], stride[d], dtype=np.int64) for d in range(3)]


def extract_box(grid: Grid, grids: list, lo, hi, stride) -> np.ndarray:
    """Values of each flat grid (x fastest) at the points of the box, as an
    array of shape (len(grids), m_z, m_y, m_x): entry [g, c, b, a] is grid g
    at the a-th selected x index, b-th y index and c-th z index."""
    ix, iy, iz = box_axes(lo, hi, stride)
    n0, n1 = grid.n[0], grid.n[1]
    out = np.empty((len(grids), iz.size, iy.size, ix.size), dtype=np.asarray(grids[0]).dtype)
    for g, F in enumerate(grids):
        for c, k in enumerate(iz):
            for b, j in enumerate(iy):
                out[g, c, b, :] = np.asarray(F)[ix + n0 * (j + n1 * k)]
    return out


def phase_space(grid: Grid, sp: dict, lo, hi, every: int = 1, skip_weightless: bool = False) -> np.ndarray:
    """Phase-space records (Sec. 3.3: positions, momenta, weight) of the
    particles, in storage order, whose storage index is a multiple of every and
    whose cell lies in [lo, hi) along each dimension (and, with
    skip_weightless, whose weight is not 0): rows x_0 .. x_{dims-1}, u_0, u_1,
    u_2, w with x_d = (cell_d + off_d) dx_d in FP64."""
    dims = grid.dims
    rows = []
    for i in range(0, sp["w"].shape[0], every):
        inside = all(lo[d] <= sp["cell"][d, i] < hi[d] for d in range(dims))
        if not inside or (skip_weightless and sp["w"][i] == 0.0):
            continue
        x = [(float(sp["cell"][d, i]) + float(sp["off"][d, i])) * grid.dx[d] for d in range(dims)]
        rows.append(x + [float(sp["u"][0, i]), float(sp["u"][1, i]), float(sp["u"][2, i]), float(sp["w"][i])])
    return np.array(rows, dtype=np.float64).reshape(len(rows), dims + 4)
