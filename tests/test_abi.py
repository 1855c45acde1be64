"""The C ABI without a GPU: the library loads, exports every function the
header declares, and validates parameters on the host (no kernel runs)."""
import ctypes
import math
import subprocess

import numpy as np
import pytest

from paper_1503_02464_amd import _lib as L
from paper_1503_02464_amd import sim


@pytest.fixture(scope="module")
def lib():
    return L.load()


def params(dims=3, n=(16, 16, 16), dx=(0.05, 0.05, 0.05), cfl=0.7, order=2, prec=L.PIC_FP32, tile=(8, 8, 8),
           slack=1, sort_every=4, maxp=1000, acc=L.PIC_ACC_AUTO, open_x=0, absorb=0, sort_levels=0):
    p = L.Params()
    p.dims = dims
    p.n = L._c3i(*n)
    p.dx = L._c3d(*dx)
    p.dt = cfl / math.sqrt(sum(1.0 / dx[d] ** 2 for d in range(min(dims, 3)) if dx[d] > 0))
    p.shape_order = order
    p.precision = prec
    p.tile = L._c3i(*tile)
    p.slack = slack
    p.sort_every = sort_every
    p.max_particles = maxp
    p.current_accum = acc
    p.open_x = open_x
    p.absorb = absorb
    p.sort_levels = sort_levels
    return p


def init(lib, p):
    ctx = ctypes.c_void_p()
    st = lib.pic_init(ctypes.byref(p), ctypes.byref(ctx))
    return st, ctx


def test_exports_every_declared_function(lib):
    names = L.header_functions()
    assert len(names) >= 20, names
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert hasattr(lib, n)


def test_valid_init_and_queries(lib):
    st, ctx = init(lib, params())
    assert st == L.PIC_OK
    assert lib.pic_num_tiles(ctx) == 8
    assert lib.pic_workspace_bytes(ctx) > 0
    bits = (ctypes.c_int32 * 3)()
    lib.pic_cell_bits(ctx, bits)
    assert tuple(bits) == (4, 4, 4)
    # LDS: fields (8+1+2+2)^3 * 6 in FP32, rows padded from 13 to 14 (even, for pair reads) +
    # current (8+2+3+2)^3 * 3 accumulated in 64 bits, its planes padded from 15 * 15 = 225 to
    # 231 elements (the next value that is 7 mod 16) + a list of 512 wide-window particles
    # (8 FP32 values + one int each) and its length
    assert lib.pic_tile_lds_bytes(ctx) == 14 * 13 * 13 * 6 * 4 + 231 * 15 * 3 * 8 + 512 * 36 + 16
    # FP64 8x8x4 tiles: fields 14 x 13 x 9 doubles, current planes 231 x 11, 256 list entries of
    # 8 doubles + an int; FP32 4^3 tiles: rows 9 -> 10, current planes 11 * 11 = 121 -> 135
    for prec, tile, want in ((L.PIC_FP64, (8, 8, 4), 14 * 13 * 9 * 6 * 8 + 231 * 11 * 3 * 8 + 256 * 68 + 16),
                             (L.PIC_FP32, (4, 4, 4), 10 * 9 * 9 * 6 * 4 + 135 * 11 * 3 * 8 + 512 * 36 + 16)):
        st2, c2 = init(lib, params(prec=prec, tile=tile))
        assert st2 == L.PIC_OK
        assert lib.pic_tile_lds_bytes(c2) == want, (prec, tile)
        lib.pic_destroy(c2)
    # 2D 8x8 tiles (dense foils): fields 14 x 13, current 15 x 15, both under 16 KB, so the
    # wide-window list is twice as long (1024 entries)
    st2, c2 = init(lib, params(dims=2, n=(64, 64, 1), dx=(0.05, 0.05, 0.0), tile=(8, 8, 1)))
    assert st2 == L.PIC_OK
    assert lib.pic_tile_lds_bytes(c2) == 14 * 13 * 6 * 4 + 15 * 15 * 3 * 8 + 1024 * 36 + 16
    lib.pic_destroy(c2)
    assert lib.pic_step_count(ctx) == 0
    lib.pic_destroy(ctx)


def test_sort_every_zero_is_valid(lib):
    st, ctx = init(lib, params(sort_every=0))  # sort only species whose sorted flag is 0
    assert st == L.PIC_OK
    lib.pic_destroy(ctx)


@pytest.mark.parametrize("cfl,want", [(0.999, L.PIC_OK), (1.0, L.PIC_ECFL), (1.2, L.PIC_ECFL)])
def test_cfl_limit(lib, cfl, want):
    st, ctx = init(lib, params(cfl=cfl))
    assert st == want
    if st == L.PIC_OK:
        lib.pic_destroy(ctx)


@pytest.mark.parametrize("kw", [
    dict(dims=4), dict(order=3), dict(prec=7), dict(tile=(5, 8, 8)), dict(tile=(8, 8, 0)),
    dict(n=(16, 16, 2)), dict(dims=2, n=(16, 16, 4), tile=(8, 8, 1)), dict(dims=2, n=(16, 16, 1), tile=(8, 8, 2)),
    dict(sort_every=-1), dict(slack=5), dict(maxp=-1), dict(dx=(0.05, 0.0, 0.05)),
    dict(n=(64, 64, 64), tile=(32, 8, 8)),  # local cells must fit the packed 6-bit range
    dict(prec=L.PIC_FP64, tile=(16, 16, 16), n=(32, 32, 32)),  # LDS tile beyond 160 KB
    dict(acc=4), dict(prec=L.PIC_FP64, acc=L.PIC_ACC_FP32), dict(prec=L.PIC_FP64, acc=L.PIC_ACC_FIX64),
    dict(open_x=2), dict(open_x=1, absorb=5),  # absorb below 2 * order + 2
    dict(open_x=1, absorb=8),  # n[0] < 2 * absorb + 2
    dict(sort_levels=1), dict(sort_levels=129),
])
def test_invalid_params(lib, kw):
    st, ctx = init(lib, params(**kw))
    assert st == L.PIC_EINVAL, kw


def test_calls_without_workspace_fail_cleanly(lib):
    st, ctx = init(lib, params())
    assert st == L.PIC_OK
    sp = L.Species()
    f = L.Fields()
    assert lib.pic_gather_push(ctx, ctypes.byref(sp), ctypes.byref(f), None) == L.PIC_ENOMEM
    assert lib.pic_step(ctx, ctypes.byref(sp), 1, ctypes.byref(f), 1, None) == L.PIC_ENOMEM
    assert b"workspace" in lib.pic_last_error(ctx)
    lib.pic_destroy(ctx)


def test_header_and_binding_agree():
    text = open(L.HEADER).read()
    for name in ("PIC_OK = 0", "PIC_EINVAL = -1", "PIC_ECFL = -2", "PIC_EHIP = -3", "PIC_ENOMEM = -4",
                 "PIC_ECROSS = -5", "PIC_ENAN = -6", "PIC_ESTATE = -7"):
        assert name in text
    assert "#define PIC_NDIAG 8" in text and "#define PIC_NPHASE 4" in text
    assert f"#define PIC_MAX_EXTRACT_GRIDS {L.PIC_MAX_EXTRACT_GRIDS}" in text


def test_struct_layout_matches_header(tmp_path):
    """Offsets of every field of the ABI structs, from gcc on pic.h, equal the ctypes mirror."""
    structs = {"pic_params": L.Params, "pic_fields": L.Fields, "pic_species": L.Species, "pic_laser": L.Laser,
               "pic_box": L.Box}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pic.h"', "int main(void){"]
    for cname, cls in structs.items():
        lines.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    inc = L.HEADER.rsplit("/", 1)[0]
    subprocess.check_call(["gcc", f"-I{inc}", "-o", str(exe), str(src)])
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {(a, b): int(c) for a, b, c in (l.split() for l in out if l.strip())}
    for cname, cls in structs.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)


def test_cell_packing_roundtrip():
    r = np.random.default_rng(0)
    for n, dims in (((256, 256, 256), 3), ((2048, 1024, 1), 2), ((512, 256, 256), 3), ((13, 7, 5), 3)):
        bits = sim.cell_bits(n, dims)
        assert sum(bits) <= 31
        cell = np.zeros((3, 1000), np.int32)
        for d in range(dims):
            cell[d] = r.integers(0, n[d], 1000)
        packed = sim.pack_cells(cell, bits)
        assert packed.dtype == np.int32
        assert np.array_equal(sim.unpack_cells(packed, bits), cell)


def laser(**kw):
    las = L.Laser(plane=3, pol=1, e0=1.0, omega=2.0, w0=0.3, tau=1.0, t0=0.5, yc=0.4, zc=0.4)
    for k, v in kw.items():
        setattr(las, k, v)
    return las


def test_laser_validation(lib):
    st, ctx = init(lib, params(open_x=1, absorb=6))
    assert st == L.PIC_OK
    assert lib.pic_set_laser(ctx, ctypes.byref(laser())) == L.PIC_OK
    assert lib.pic_set_laser(ctx, None) == L.PIC_OK  # none
    for kw in (dict(plane=0), dict(plane=15), dict(pol=3), dict(e0=0.0), dict(w0=-1.0), dict(tau=0.0),
               dict(omega=1e4), dict(t0=float("nan"))):
        assert lib.pic_set_laser(ctx, ctypes.byref(laser(**kw))) == L.PIC_EINVAL, kw
    f = L.Fields()
    assert lib.pic_laser_current(ctx, ctypes.byref(f), 0.0, None) == L.PIC_EINVAL  # null field pointers
    lib.pic_destroy(ctx)
    st, ctx = init(lib, params())  # periodic: no laser, no adjoint restrictions
    assert lib.pic_set_laser(ctx, ctypes.byref(laser())) == L.PIC_EINVAL
    lib.pic_destroy(ctx)


def test_adjoint_refuses_open_faces(lib):
    st, ctx = init(lib, params(open_x=1, absorb=6))
    f = L.Fields()
    assert lib.pic_yee_adjoint(ctx, ctypes.byref(f), None) == L.PIC_EINVAL
    assert lib.pic_energy_adjoint(ctx, ctypes.byref(f), ctypes.byref(f), 1.0, None) == L.PIC_EINVAL
    lib.pic_destroy(ctx)


def box(lo, hi, stride=(1, 1, 1)):
    return L.Box(lo=(ctypes.c_int32 * 3)(*lo), hi=(ctypes.c_int32 * 3)(*hi), stride=(ctypes.c_int32 * 3)(*stride))


BAD_BOXES = [((-1, 0, 0), (4, 4, 4), (1, 1, 1)), ((0, 0, 0), (17, 4, 4), (1, 1, 1)), ((5, 0, 0), (4, 4, 4), (1, 1, 1)),
             ((0, 0, 0), (4, 4, 4), (0, 1, 1)), ((0, 0, 0), (4, 4, 16 + 1), (1, 1, 1))]


@pytest.mark.parametrize("lo,hi,stride", BAD_BOXES)
def test_extract_grid_refuses_bad_boxes(lib, lo, hi, stride):
    st, ctx = init(lib, params())
    grids = (ctypes.c_void_p * 1)(0x1000)
    b = box(lo, hi, stride)
    assert lib.pic_extract_grid(ctx, grids, 1, 4, ctypes.byref(b), ctypes.c_void_p(0x2000), None) == L.PIC_EINVAL
    assert b"box" in lib.pic_last_error(ctx)
    lib.pic_destroy(ctx)


def test_extract_grid_argument_checks(lib):
    st, ctx = init(lib, params())
    b = box((0, 0, 0), (16, 16, 1))
    grids = (ctypes.c_void_p * 17)(*([0x1000] * 17))
    dst = ctypes.c_void_p(0x2000)
    assert lib.pic_extract_grid(ctx, grids, 0, 4, ctypes.byref(b), dst, None) == L.PIC_EINVAL
    assert lib.pic_extract_grid(ctx, grids, 17, 4, ctypes.byref(b), dst, None) == L.PIC_EINVAL
    assert lib.pic_extract_grid(ctx, grids, 1, 2, ctypes.byref(b), dst, None) == L.PIC_EINVAL
    assert lib.pic_extract_grid(ctx, grids, 1, 4, None, dst, None) == L.PIC_EINVAL
    assert lib.pic_extract_grid(ctx, grids, 1, 4, ctypes.byref(b), None, None) == L.PIC_EINVAL
    nul = (ctypes.c_void_p * 2)(0x1000, None)
    assert lib.pic_extract_grid(ctx, nul, 2, 4, ctypes.byref(b), dst, None) == L.PIC_EINVAL
    lib.pic_destroy(ctx)


def test_extract_particles_argument_checks(lib):
    st, ctx = init(lib, params())
    sp = L.Species()
    cells = box((0, 0, 0), (16, 16, 16), (0, 0, 0))  # the stride of a cell box is not used
    cnt = ctypes.c_void_p(0x3000)
    # no workspace yet
    assert lib.pic_extract_particles(ctx, ctypes.byref(sp), ctypes.byref(cells), 1, None, 0, cnt, None) == L.PIC_ENOMEM
    lib.pic_destroy(ctx)
