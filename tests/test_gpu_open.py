"""Open x faces (first-order Mur), the laser current sheet and particle
removal: the HIP library against the FP64 oracle.  FP64 to 1e-12, FP32 to
the per-quantity tolerances of gpu_helpers.TOL; particles compared by their
(unique) weights among those not removed."""
import math

import numpy as np
import pytest
import torch

import oracle as O
from gpu_helpers import TOL, compare_fields, compare_species, grid, unique_weights
from paper_1503_02464_amd import inputs
from paper_1503_02464_amd.sim import Simulation

pytestmark = pytest.mark.gpu

ABSORB = 6


def open_grid(dims, order):
    return grid(dims, (48, 16) if dims == 2 else (32, 8, 8), dx=0.05, cfl=0.7, order=order)


def open_sim(g, prec, sort_every=4, max_particles=1):
    tile = (8, 4, 1) if g.dims == 2 else (8, 4, 4)
    return Simulation(g.dims, g.n, g.dx, g.dt, g.order, prec, tile=tile, slack=1, sort_every=sort_every,
                      max_particles=max_particles, open_x=True, absorb=ABSORB)


def laser_for(g):
    dx = g.dx[0]
    omega = 2 * math.pi / (16 * dx)  # 16 cells per wavelength
    return O.Laser(plane=3, e0=0.5, omega=omega, w0=4 * g.dx[1], tau=8 * g.dt, t0=5 * g.dt,
                   yc=0.5 * g.n[1] * g.dx[1], zc=0.5 * g.n[2] * g.dx[2] if g.dims == 3 else 0.0, pol=1)


def set_laser(s, las):
    s.set_laser(las.plane, las.e0, las.omega, las.w0, las.tau, las.t0, las.yc, las.zc, las.pol)


def species_pair(g, prec, seed):
    """Hot electrons over the live x range (some leave within a few steps) and
    ions at their positions; distinct weights, FP32-exact for the FP32 path."""
    hi = g.n[0] - ABSORB
    e = inputs.random_particles(g.n, g.dims, 3 * g.ncells // g.n[0] * (hi - ABSORB) // 4, 0.3, (1, 1), seed)
    e["cell"][0] = ABSORB + e["cell"][0] % (hi - ABSORB)
    e = unique_weights(e, seed + 1, scale=1e-3)
    i = inputs.co_located(e, 1.0, 1836.0, 0.01, seed + 2)
    i = unique_weights(i, seed + 3, scale=1e-3)
    if prec == "fp32":
        e, i = inputs.round_f32(e), inputs.round_f32(i)
    return e, i


def live(sp):
    keep = sp["w"] != 0
    return {"q": sp["q"], "m": sp["m"], "cell": sp["cell"][:, keep], "off": sp["off"][:, keep],
            "u": sp["u"][:, keep], "w": sp["w"][keep]}


@pytest.mark.parametrize("prec,dims", [(p, d) for p in ("fp64", "fp32") for d in (2, 3)])
def test_open_yee_step(prec, dims):
    g = open_grid(dims, 2)
    f = inputs.random_fields(g.ncells, 1.0, seed=400 + dims)
    f["J"] = inputs.rng(401).normal(size=(3, g.ncells))
    if prec == "fp32":
        f = inputs.round_fields_f32(f)
    s = open_sim(g, prec)
    s.set_fields(f["E"], f["B"], f["J"])
    s.yee_step()
    ref = {k: v.copy() for k, v in f.items()}
    O.yee_step_open(g, ref)
    compare_fields(prec, s.get_fields(), ref, keys=("E", "B"), what="open yee")
    s.close()


@pytest.mark.parametrize("prec,dims,pol", [("fp64", 2, 1), ("fp64", 3, 1), ("fp64", 3, 2), ("fp32", 3, 2)])
def test_laser_sheet(prec, dims, pol):
    g = open_grid(dims, 2)
    las = laser_for(g)
    las.pol = pol
    s = open_sim(g, prec)
    set_laser(s, las)
    ref = np.zeros((3, g.ncells))
    for t in (0.3 * g.dt, 4.5 * g.dt, 7.5 * g.dt):
        s.laser_current(t)
        O.laser_add(g, ref, las, t)
    got = s.get_fields()["J"]
    tol = 1e-12 if prec == "fp64" else 1e-6
    assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref)), np.max(np.abs(got - ref))
    assert np.max(np.abs(ref[pol])) > 0
    s.close()


@pytest.mark.parametrize("dims,order", [(2, 1), (2, 2), (3, 1), (3, 2)])
def test_open_steps_two_species_fp64(dims, order):
    """12 fused steps (re-sorted every 4) of electrons and ions with the laser
    on: the particles that remain, their states, and E, B, J all match the
    oracle, which removes the same particles in the same steps."""
    g = open_grid(dims, order)
    e, i = species_pair(g, "fp64", 410 + 10 * dims + order)
    f = inputs.random_fields(g.ncells, 0.2, seed=420)
    las = laser_for(g)
    s = open_sim(g, "fp64", max_particles=e["w"].shape[0])
    s.set_fields(f["E"], f["B"])
    set_laser(s, las)
    he, hi = s.add_species(e), s.add_species(i)
    ref_f = {k: v.copy() for k, v in f.items()}
    ref = [O.copy_species(e), O.copy_species(i)]
    removed = 0
    for n in range(12):
        s.step(1)
        ref, bad, rem = O.step_open(g, ref_f, ref, ABSORB, g.n[0] - ABSORB, las, n)
        assert bad == 0
        removed += rem
    s.check()
    assert removed > 0, "the case should remove particles"
    for h, r, what in ((he, ref[0], "electrons"), (hi, ref[1], "ions")):
        compare_species(g, "fp64", live(s.get_species(h)), r, what)
    compare_fields("fp64", s.get_fields(), ref_f, what="open step")
    s.close()


@pytest.mark.parametrize("dims,order", [(2, 2), (3, 2)])
def test_open_step_fp32(dims, order):
    """One fused FP32 step from an FP32-representable state with particles
    right at the removal edge."""
    g = open_grid(dims, order)
    e, i = species_pair(g, "fp32", 430 + dims)
    # push a tenth of the electrons to the first live cell, heading out
    k = e["w"].shape[0] // 10
    e["cell"][0, :k] = ABSORB
    e["off"][0, :k] = np.float32(0.05)
    e["u"][0, :k] = np.float32(-0.5)
    f = inputs.round_fields_f32(inputs.random_fields(g.ncells, 0.2, seed=431))
    las = laser_for(g)
    s = open_sim(g, "fp32", max_particles=e["w"].shape[0])
    s.set_fields(f["E"], f["B"])
    set_laser(s, las)
    he, hi = s.add_species(e), s.add_species(i)
    s.step(1)
    s.check()
    ref_f = {k_: v.copy() for k_, v in f.items()}
    ref, bad, rem = O.step_open(g, ref_f, [O.copy_species(e), O.copy_species(i)], ABSORB, g.n[0] - ABSORB, las, 0)
    assert bad == 0 and rem >= k
    for h, r, what in ((he, ref[0], "electrons"), (hi, ref[1], "ions")):
        compare_species(g, "fp32", live(s.get_species(h)), r, what)
    compare_fields("fp32", s.get_fields(), ref_f, what="open step fp32")
    s.close()


def test_open_unfused_step_fp64():
    """The same step composed from pic_gather_push, pic_deposit,
    pic_laser_current and pic_yee_step."""
    g = open_grid(2, 2)
    e, _ = species_pair(g, "fp64", 440)
    f = inputs.random_fields(g.ncells, 0.2, seed=441)
    las = laser_for(g)
    s = open_sim(g, "fp64", max_particles=e["w"].shape[0])
    s.set_fields(f["E"], f["B"])
    set_laser(s, las)
    h = s.add_species(e)
    ref_f = {k: v.copy() for k, v in f.items()}
    ref = [O.copy_species(e)]
    for n in range(6):
        s.zero_current()
        s.gather_push(h)
        s.deposit(h)
        s.laser_current((n + 0.5) * g.dt)
        s.yee_step()
        ref, bad, _ = O.step_open(g, ref_f, ref, ABSORB, g.n[0] - ABSORB, las, n)
        assert bad == 0
    s.check()
    compare_species(g, "fp64", live(s.get_species(h)), ref[0], "unfused open")
    compare_fields("fp64", s.get_fields(), ref_f, what="unfused open")
    s.close()


def test_sort_moves_removed_particles_behind_the_tiles():
    g = open_grid(3, 2)
    e, _ = species_pair(g, "fp64", 450)
    k = e["w"].shape[0] // 5
    e["cell"][0, :k] = ABSORB
    e["off"][0, :k] = 0.01
    e["u"][0, :k] = -0.9
    s = open_sim(g, "fp64", sort_every=1 << 30, max_particles=e["w"].shape[0])
    h = s.add_species(e)
    s.step(2)  # the first step sorts, both remove
    nlive = int(s.live(h).sum().item())
    assert nlive <= e["w"].shape[0] - k
    s.sort(h)
    start = s.tile_start(h)
    w = s.get_species(h)["w"]
    assert start[-1] == nlive
    assert h.np == nlive and h.struct.np == nlive  # the removed particles are dropped
    assert w.shape[0] == nlive and np.all(w != 0)
    s.step(1)  # the smaller species steps on
    s.check()
    s.close()


def test_every_particle_leaves():
    """A species that entirely leaves through the faces: nothing stays live,
    the current after that step is the laser sheet alone, the sort moves every
    particle behind the tiles, and later steps run on an empty species."""
    g = open_grid(2, 2)
    n0 = g.n[0]
    npart = 64
    sp = {"q": -1.0, "m": 1.0, "cell": np.zeros((3, npart), np.int32), "off": np.full((3, npart), 0.02),
          "u": np.zeros((3, npart)), "w": np.full(npart, 1e-3)}
    half = npart // 2
    sp["cell"][0, :half] = ABSORB  # first live cell, heading out through the low face
    sp["cell"][0, half:] = n0 - ABSORB - 1  # last live cell, heading out through the high face
    sp["off"][0, half:] = 0.98
    r = inputs.rng(460)
    sp["cell"][1] = r.integers(0, g.n[1], npart)
    sp["off"][1] = r.random(npart)
    sp["u"][0, :half] = -0.9
    sp["u"][0, half:] = 0.9
    sp["u"][1] = r.normal(0, 0.2, npart)  # so that the current, and B, vary in y
    s = open_sim(g, "fp64", sort_every=1 << 30, max_particles=npart)
    h = s.add_species(sp)
    s.step(1)
    s.check()
    assert int(s.live(h).sum().item()) == 0
    ref_f = O.new_fields(g)
    ref, bad, removed = O.step_open(g, ref_f, [O.copy_species(sp)], ABSORB, n0 - ABSORB, None, 0)
    assert bad == 0 and removed == npart and ref[0]["w"].shape[0] == 0
    compare_fields("fp64", s.get_fields(), ref_f, what="all leave")
    s.sort(h)
    assert s.tile_start(h)[-1] == 0 and h.np == 0
    s.step(3)
    s.check()
    d = s.diagnostics()
    assert d["Q"] == 0.0 and d["K"] == 0.0
    s.close()
