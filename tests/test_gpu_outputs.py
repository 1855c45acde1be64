"""Outputs on the GPU (paper Sec. 3.1: reduced-dimension and subdomain outputs
of the grid data, the particles' phase space; Sec. 3.3: seven values per
particle).  pic_extract_grid against the oracle's indexing definition, bit for
bit: planes, lines, strided sub-boxes, the whole grid, an empty box, FP64
density grids, and a grid large enough for 64-bit indexing (sampled).
pic_extract_particles against the oracle's selection in storage order, bit for
bit: several chunks and a ragged tail, subsampling, a full capacity, an empty
species and removed particles at open faces.  The output manager's files
against the state at the steps it wrote them."""
import ctypes
import json
import math
import os

import numpy as np
import pytest
import torch

import oracle as O
from gpu_helpers import grid
from paper_1503_02464_amd import _lib as L
from paper_1503_02464_amd import inputs
from paper_1503_02464_amd.outputs import OutputManager
from paper_1503_02464_amd.sim import Simulation

pytestmark = pytest.mark.gpu

N = {3: (24, 16, 12), 2: (40, 24)}
TILE = {3: (8, 8, 4), 2: (8, 8)}
BOXES = {
    3: [((0, 0, 5), (24, 16, 6), (1, 1, 1)),   # a z plane
        ((0, 7, 3), (24, 8, 4), (1, 1, 1)),    # an x line
        ((3, 2, 1), (21, 15, 10), (4, 3, 2)),  # a strided sub-box
        ((0, 0, 0), (24, 16, 12), (1, 1, 1)),  # the whole grid
        ((23, 15, 11), (24, 16, 12), (1, 1, 1)),  # the last point
        ((5, 5, 5), (5, 9, 9), (1, 1, 1))],    # empty
    2: [((0, 11), (40, 12), (1, 1)),           # an x line
        ((17, 0), (18, 24), (1, 1)),           # a y line
        ((1, 2), (39, 23), (5, 4)),            # a strided sub-box
        ((0, 0), (40, 24), (1, 1))],           # the whole grid
}


def bits(a: np.ndarray) -> np.ndarray:
    return a.view(np.uint32 if a.itemsize == 4 else np.uint64)


def sim_for(dims, prec, npart=1, **kw):
    g = grid(dims, N[dims])
    return g, Simulation(dims, g.n, g.dx, g.dt, 2, prec, tile=TILE[dims], max_particles=max(npart, 1), **kw)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("dims", [2, 3])
def test_extract_grid_is_the_box_of_the_grid(dims, prec):
    g, s = sim_for(dims, prec)
    f = inputs.random_fields(g.ncells, 1.0, seed=900 + dims)
    f["J"] = inputs.random_fields(g.ncells, 1.0, seed=910 + dims)["E"]
    s.set_fields(f["E"], f["B"], f["J"])
    host = {k: [t.cpu().numpy() for t in s.fields[k]] for k in "EBJ"}
    comps = [("E", 1), ("B", 2), ("J", 0), ("E", 0)]
    for lo, hi, st in BOXES[dims]:
        b = s.box(lo, hi, st)
        got = s.extract_grid([s.fields[k][d] for k, d in comps], b).cpu().numpy()
        want = O.extract_box(g, [host[k][d] for k, d in comps], tuple(b.lo), tuple(b.hi), tuple(b.stride))
        assert got.shape == want.shape, (lo, hi, st)
        assert np.array_equal(bits(got), bits(want)), (lo, hi, st)
    s.close()


def test_extract_density_grid_fp64_from_fp32_state():
    """The FP64 charge-density grid (8-byte elements) out of an FP32 state."""
    g, s = sim_for(3, "fp32", 4000)
    sp = inputs.round_f32(inputs.random_particles(g.n, 3, 4000, 0.1, (0.5, 1.5), seed=920))
    s.add_species(sp)
    rho = torch.empty(s.ncells, dtype=torch.float64, device="cuda")
    s.charge_density_into(rho)
    b = s.box((2, 0, 3), (22, 16, 4), (2, 3, 1))
    got = s.extract_grid([rho], b).cpu().numpy()
    want = O.extract_box(g, [rho.cpu().numpy()], tuple(b.lo), tuple(b.hi), tuple(b.stride))
    assert np.array_equal(bits(got), bits(want))
    assert np.abs(got).max() > 0
    s.close()


def test_extract_grid_with_64bit_indices():
    """Two 1024^3 grids (2^31 output values, past 32-bit indexing): sampled
    output entries hold the flat index of their source point.  The grid is
    int32 (the copy moves 4-byte elements whatever they hold)."""
    lib = L.load()
    p = L.Params()
    p.dims, p.n, p.dx = 3, L._c3i(1024, 1024, 1024), L._c3d(1.0, 1.0, 1.0)
    p.dt, p.shape_order, p.precision = 0.5, 1, L.PIC_FP32
    p.tile, p.slack, p.sort_every, p.max_particles = L._c3i(8, 8, 8), 1, 4, 1
    p.sort_levels = 2  # keeps the sort's bucket count within its scan (no sort runs here)
    ctx = ctypes.c_void_p()
    assert lib.pic_init(ctypes.byref(p), ctypes.byref(ctx)) == L.PIC_OK
    src = torch.arange(1 << 30, dtype=torch.int32, device="cuda")
    out = torch.empty(1 << 31, dtype=torch.int32, device="cuda")
    b = L.Box(lo=L._c3i(0, 0, 0), hi=L._c3i(1024, 1024, 1024), stride=L._c3i(1, 1, 1))
    arr = (ctypes.c_void_p * 2)(src.data_ptr(), src.data_ptr())
    st = lib.pic_extract_grid(ctx, arr, 2, 4, ctypes.byref(b), ctypes.c_void_p(out.data_ptr()),
                              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == L.PIC_OK
    idx = torch.cat([torch.arange(0, 4096, device="cuda"), (1 << 31) - 1 - torch.arange(0, 4096, device="cuda"),
                     torch.randint(0, 1 << 31, (1 << 16,), device="cuda", generator=torch.Generator("cuda").manual_seed(5))])
    got = out[idx].long()
    assert torch.equal(got, idx % (1 << 30))
    lib.pic_destroy(ctx)
    del src, out
    torch.cuda.empty_cache()


def particle_state(dims, prec, npart, seed, **kw):
    g, s = sim_for(dims, prec, npart, **kw)
    sp = inputs.random_particles(g.n, dims, npart, 0.2, (0.5, 1.5), seed=seed)
    if prec == "fp32":
        sp = inputs.round_f32(sp)
    h = s.add_species(sp)
    return g, s, h


def extract(s, h, lo, hi, every, cap):
    out = torch.full((max(cap, 1), s.dims + 4), float("nan"), dtype=s.dtype, device="cuda")
    cnt = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    s.extract_particles(h, s.box(lo, hi), every, out[:cap] if cap else out[:0], cnt)
    torch.cuda.synchronize()
    return out.cpu().numpy(), int(cnt.item())


def as_state(prec, rec):
    """The oracle's FP64 records in the state's precision: positions rounded
    once, momenta and weights exact (they are FP32 values in an FP32 state)."""
    return rec.astype(np.float32) if prec == "fp32" else rec


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("dims", [2, 3])
def test_extract_particles_matches_the_selection(dims, prec):
    """50,003 particles (six full chunks of 8192 and a ragged one), after two
    steps and a sort so the storage order is the library's: boxes, strides
    of the storage order, and every record bit for bit in order."""
    npart = 50_003
    g, s, h = particle_state(dims, prec, npart, seed=930 + dims)
    s.step(2)
    ref = s.get_species(h)
    n = N[dims]
    cases = [((0,) * dims, n, 1), ((0,) * dims, n, 7), ((3, 2, 1)[:dims], (21, 15, 10)[:dims], 1),
             ((5, 0, 0)[:dims], (6, n[1], n[2] if dims == 3 else 1)[:dims], 3), ((4, 4, 4)[:dims], (4, 9, 9)[:dims], 1)]
    for lo, hi, every in cases:
        b = s.box(lo, hi)
        want = as_state(prec, O.phase_space(g, ref, tuple(b.lo), tuple(b.hi), every))
        got, k = extract(s, h, lo, hi, every, npart)
        assert k == want.shape[0], (lo, hi, every)
        assert np.array_equal(bits(got[:k]), bits(want)), (lo, hi, every)
        assert np.isnan(got[k:]).all()  # nothing written past the count
    s.close()


def test_extract_particles_capacity_and_empty_species():
    g, s, h = particle_state(3, "fp32", 20_000, seed=940)
    ref = s.get_species(h)
    want = as_state("fp32", O.phase_space(g, ref, (0, 0, 0), g.n, 1))
    got, k = extract(s, h, (0, 0, 0), g.n, 1, 1000)
    assert k == 20_000  # the count of all selected, beyond the capacity
    assert np.array_equal(bits(got[:1000]), bits(want[:1000]))
    got, k = extract(s, h, (0, 0, 0), g.n, 1, 0)  # no room at all
    assert k == 20_000
    e = s.add_species({"q": 1.0, "m": 1836.0, "cell": np.zeros((3, 0), np.int32), "off": np.zeros((3, 0)),
                       "u": np.zeros((3, 0)), "w": np.zeros(0)})
    got, k = extract(s, e, (0, 0, 0), g.n, 1, 10)
    assert k == 0 and np.isnan(got).all()
    s.close()


def test_extract_particles_skips_removed_ones_at_open_faces():
    """With open x faces a weight-0 particle is a removed one: not output."""
    g = grid(3, (32, 16, 8))
    s = Simulation(3, g.n, g.dx, g.dt, 2, "fp64", tile=(8, 8, 4), max_particles=9000, open_x=True, absorb=6)
    sp = inputs.random_particles(g.n, 3, 9000, 0.1, (0.5, 1.5), seed=950)
    sp["w"][::7] = 0.0
    h = s.add_species(sp)
    ref = s.get_species(h)
    want = O.phase_space(g, ref, (0, 0, 0), g.n, 2, skip_weightless=True)
    got, k = extract(s, h, (0, 0, 0), g.n, 2, 9000)
    assert k == want.shape[0] and k < 4500
    assert np.array_equal(bits(got[:k]), bits(want))
    s.close()


def test_extract_calls_refuse_bad_arguments_with_a_workspace():
    g, s, h = particle_state(3, "fp32", 100, seed=960)
    out = torch.empty((10, 7), dtype=torch.float32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    for lo, hi, every in (((0, 0, 0), (25, 16, 12), 1), ((3, 0, 0), (2, 16, 12), 1), ((0, 0, 0), (24, 16, 12), 0)):
        with pytest.raises(L.PicError):
            s.extract_particles(h, s.box(lo, hi), every, out, cnt)
    s.close()


def test_output_manager_writes_what_the_state_holds(tmp_path):
    """Ten FP32 steps of a 3D box with two species and four requests (a field
    plane in a window, a strided sub-box of E, a density line, an electron
    phase-space dump with subsampling): every file written equals the state
    read synchronously right after the step it belongs to (the density to
    FP64 rounding, its deposit order being free), and the index lists them."""
    g = grid(3, N[3])
    s = Simulation(3, g.n, g.dx, g.dt, 2, "fp32", tile=TILE[3], max_particles=12_000, sort_every=4)
    e = inputs.round_f32(inputs.random_particles(g.n, 3, 12_000, 0.2, (0.5, 1.5), seed=970))
    i = inputs.round_f32(inputs.random_particles(g.n, 3, 6_000, 0.005, (1.0, 2.0), seed=971, q=1.0, m=1836.0))
    he, _ = s.add_species(e), s.add_species(i)
    reqs = [{"name": "plane", "kind": "fields", "components": ["Ey", "Bz", "Jx"],
             "box": {"lo": [0, 0, 6], "hi": [24, 16, 7]}, "every": 2, "from": 2, "to": 8},
            {"name": "sub", "kind": "fields", "components": ["E"],
             "box": {"lo": [2, 3, 1], "hi": [20, 15, 11], "stride": [3, 2, 5]}, "every": 5},
            {"name": "rho", "kind": "density", "species": [0], "box": {"lo": [0, 8, 0], "hi": [24, 9, 12]}, "every": 4},
            {"name": "elec", "kind": "particles", "species": 0, "cells": {"lo": [4, 0, 0], "hi": [20, 16, 6]},
             "subsample": 3, "every": 3}]
    m = OutputManager(s, reqs, str(tmp_path))
    expect = {}
    for _ in range(10):
        s.step(1)
        m.after_step()
        k = s.step_count
        for r in m.reqs:
            if not r.fires(k):
                continue
            if r.kind == "fields":
                grids = [s.fields[c[0]]["xyz".index(c[1])].cpu().numpy() for c in r.components]
                expect[(r.name, k)] = O.extract_box(g, grids, r.lo, r.hi, r.stride)
            elif r.kind == "density":
                rho = s.charge_density([s.species[0]])
                expect[(r.name, k)] = O.extract_box(g, [rho], r.lo, r.hi, r.stride)
            else:
                ref = s.get_species(he)
                expect[(r.name, k)] = as_state("fp32", O.phase_space(g, ref, r.lo, r.hi, r.subsample))
    m.close()
    assert sorted({n for n, _ in expect}) == ["elec", "plane", "rho", "sub"]
    assert sorted(k for n, k in expect if n == "plane") == [2, 4, 6, 8]
    for (name, k), want in expect.items():
        got = np.load(os.path.join(tmp_path, name, f"{k:08d}.npy"))
        assert got.shape == want.shape, (name, k)
        if name == "rho":
            np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())
        else:
            assert np.array_equal(bits(got), bits(want)), (name, k)
    for name in ("plane", "sub", "rho", "elec"):
        lines = [json.loads(x) for x in open(os.path.join(tmp_path, name, "index.jsonl"))]
        assert sorted(x["step"] for x in lines) == sorted(k for n, k in expect if n == name)
        for x in lines:
            assert math.isclose(x["time"], x["step"] * s.dt)
            if name == "elec":
                assert x["count"] == x["shape"][0] and not x["truncated"]
    desc = json.load(open(os.path.join(tmp_path, "outputs.json")))
    plane = [d for d in desc["outputs"] if d["name"] == "plane"][0]
    assert plane["components"] == ["Ey", "Bz", "Jx"] and plane["positions"]["Bz"] == [0.5, 0.5, 0]
    assert m.files == len(expect)
    s.close()
