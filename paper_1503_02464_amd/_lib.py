"""ctypes binding of libpic.so (the C ABI in include/pic.h): structs and
function signatures only.  Loading fails loudly when the library is missing;
there is no fallback implementation."""
from __future__ import annotations

import ctypes
import os
import re

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libpic.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "pic.h")

PIC_OK, PIC_EINVAL, PIC_ECFL, PIC_EHIP, PIC_ENOMEM, PIC_ECROSS, PIC_ENAN, PIC_ESTATE = 0, -1, -2, -3, -4, -5, -6, -7
PIC_FP32, PIC_FP64 = 0, 1
PIC_ACC_AUTO, PIC_ACC_FP32, PIC_ACC_FP64, PIC_ACC_FIX64 = 0, 1, 2, 3
PIC_NDIAG = 8
PIC_NOALLOC_MAX_CELLS = 1 << 22
PIC_NPHASE = 4
PIC_MAX_EXTRACT_GRIDS = 16
PHASES = ("sort", "zero_current", "push_deposit", "yee")

_c3i = ctypes.c_int32 * 3
_c3d = ctypes.c_double * 3
_c3p = ctypes.c_void_p * 3


class Params(ctypes.Structure):
    _fields_ = [
        ("dims", ctypes.c_int32),
        ("n", _c3i),
        ("dx", _c3d),
        ("dt", ctypes.c_double),
        ("shape_order", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("tile", _c3i),
        ("slack", ctypes.c_int32),
        ("sort_every", ctypes.c_int32),
        ("max_particles", ctypes.c_int64),
        ("current_accum", ctypes.c_int32),
        ("open_x", ctypes.c_int32),
        ("absorb", ctypes.c_int32),
        ("sort_levels", ctypes.c_int32),
    ]


class Laser(ctypes.Structure):
    _fields_ = [
        ("plane", ctypes.c_int32),
        ("pol", ctypes.c_int32),
        ("e0", ctypes.c_double),
        ("omega", ctypes.c_double),
        ("w0", ctypes.c_double),
        ("tau", ctypes.c_double),
        ("t0", ctypes.c_double),
        ("yc", ctypes.c_double),
        ("zc", ctypes.c_double),
    ]


class Fields(ctypes.Structure):
    _fields_ = [("E", _c3p), ("B", _c3p), ("J", _c3p), ("E_alt", _c3p), ("B_alt", _c3p)]


class Species(ctypes.Structure):
    _fields_ = [
        ("np", ctypes.c_int64),
        ("q", ctypes.c_double),
        ("m", ctypes.c_double),
        ("cell", ctypes.c_void_p),
        ("off", _c3p),
        ("u", _c3p),
        ("w", ctypes.c_void_p),
        ("cell_alt", ctypes.c_void_p),
        ("off_alt", _c3p),
        ("u_alt", _c3p),
        ("w_alt", ctypes.c_void_p),
        ("tile_start", ctypes.c_void_p),
        ("sorted", ctypes.c_int32),
    ]


class Box(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_int32 * 3), ("hi", ctypes.c_int32 * 3), ("stride", ctypes.c_int32 * 3)]


class SpeciesAdjoint(ctypes.Structure):
    _fields_ = [("x", _c3p), ("u", _c3p)]


class PicError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"pic status {status}: {msg}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load libpic.so and declare the ABI.  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not found: build it with `python -m paper_1503_02464_amd.build` "
                           "(the HIP library is required; there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    ctx = ctypes.c_void_p
    st = ctypes.c_int
    sig = {
        "pic_init": (st, [P(Params), P(ctx)]),
        "pic_destroy": (None, [ctx]),
        "pic_workspace_bytes": (ctypes.c_size_t, [ctx]),
        "pic_set_workspace": (st, [ctx, ctypes.c_void_p, ctypes.c_size_t]),
        "pic_num_tiles": (ctypes.c_int64, [ctx]),
        "pic_cell_bits": (None, [ctx, P(ctypes.c_int32)]),
        "pic_tile_lds_bytes": (ctypes.c_size_t, [ctx]),
        "pic_gather_push": (st, [ctx, P(Species), P(Fields), ctypes.c_void_p]),
        "pic_deposit": (st, [ctx, P(Species), P(Fields), ctypes.c_void_p]),
        "pic_zero_current": (st, [ctx, P(Fields), ctypes.c_void_p]),
        "pic_yee_step": (st, [ctx, P(Fields), ctypes.c_void_p]),
        "pic_set_laser": (st, [ctx, P(Laser)]),
        "pic_laser_current": (st, [ctx, P(Fields), ctypes.c_double, ctypes.c_void_p]),
        "pic_sort": (st, [ctx, P(Species), ctypes.c_void_p]),
        "pic_step": (st, [ctx, P(Species), ctypes.c_int32, P(Fields), ctypes.c_int32, ctypes.c_void_p]),
        "pic_diagnostics": (st, [ctx, P(Species), ctypes.c_int32, P(Fields), P(ctypes.c_double), ctypes.c_void_p]),
        "pic_charge_density": (st, [ctx, P(Species), ctypes.c_int32, P(Fields), ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p]),
        "pic_diagnostics_noalloc": (st, [ctx, P(Species), ctypes.c_int32, P(Fields), P(ctypes.c_double),
                                         ctypes.c_void_p]),
        "pic_extract_grid": (st, [ctx, P(ctypes.c_void_p), ctypes.c_int32, ctypes.c_int32, P(Box), ctypes.c_void_p,
                                  ctypes.c_void_p]),
        "pic_extract_particles": (st, [ctx, P(Species), P(Box), ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                       ctypes.c_void_p, ctypes.c_void_p]),
        "pic_check": (st, [ctx, ctypes.c_void_p]),
        "pic_set_timing": (st, [ctx, ctypes.c_int32]),
        "pic_get_timing": (st, [ctx, P(ctypes.c_double), P(ctypes.c_int64), ctypes.c_int32]),
        "pic_step_count": (ctypes.c_int64, [ctx]),
        "pic_straggler_count": (st, [ctx, P(ctypes.c_int64), ctypes.c_void_p]),
        "pic_energy_adjoint": (st, [ctx, P(Fields), P(Fields), ctypes.c_double, ctypes.c_void_p]),
        "pic_yee_adjoint": (st, [ctx, P(Fields), ctypes.c_void_p]),
        "pic_particle_adjoint": (st, [ctx, P(Species), P(Fields), P(Fields), P(SpeciesAdjoint), ctypes.c_void_p]),
        "pic_last_error": (ctypes.c_char_p, [ctx]),
        "pic_status_string": (ctypes.c_char_p, [st]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def header_functions(path: str = HEADER) -> list:
    """Names of the functions include/pic.h declares."""
    text = open(path).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(pic_[a-z_0-9]+)\s*\(", text, re.M)))


def check(lib, ctx, status: int, what: str) -> None:
    if status != PIC_OK:
        msg = lib.pic_last_error(ctx) if ctx else lib.pic_status_string(status)
        raise PicError(status, f"{what}: {msg.decode() if msg else ''}")
