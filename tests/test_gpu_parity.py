"""HIP library vs the FP64 oracle, element by element, on seeded inputs.

FP64 path: 1e-12 (norm-relative for u, E, B, J; absolute cells for
positions).  FP32 path (cell index + FP32 offset, FP32 momenta, fields and
LDS current): the per-quantity tolerances in gpu_helpers.TOL."""
import numpy as np
import pytest

import oracle as O
from gpu_helpers import (TOL, by_weight, compare_fields, compare_species, grid, make_sim, pos_err, rel,
                         state)
from paper_1503_02464_amd import inputs

pytestmark = pytest.mark.gpu

VARIANTS = [(p, d, m) for p in ("fp64", "fp32") for d in (2, 3) for m in (1, 2)]
VID = [f"{p}-{d}d-m{m}" for p, d, m in VARIANTS]


def small_grid(dims, order, n2=(24, 20), n3=(16, 12, 8)):
    return grid(dims, n2 if dims == 2 else n3, dx=0.05, cfl=0.7, order=order)


def tiles(dims):
    return (8, 4, 1) if dims == 2 else (8, 4, 4)


@pytest.mark.parametrize("prec,dims", [(p, d) for p in ("fp64", "fp32") for d in (2, 3)])
def test_yee_step(prec, dims):
    g = small_grid(dims, 2)
    f = inputs.random_fields(g.ncells, 1.0, seed=21)
    f["J"] = inputs.rng(22).normal(size=(3, g.ncells))
    if prec == "fp32":
        f = inputs.round_fields_f32(f)
    s = make_sim(g, prec, tiles(dims), max_particles=1)
    s.set_fields(f["E"], f["B"], f["J"])
    s.yee_step()
    ref = {k: v.copy() for k, v in f.items()}
    O.yee_step(g, ref)
    compare_fields(prec, s.get_fields(), ref, keys=("E", "B"), what="yee")
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n,open_x", [((64, 16, 6), False), ((128, 8, 5), True), ((64, 8, 4), False)],
                         ids=["periodic", "open-two-x-tiles", "one-chunk"])
def test_yee_step_one_pass(prec, n, open_x):
    """The one-pass Yee step into the second field set (3D, x a multiple of 64,
    y of 8) against the oracle's three-part update, three steps in a row, so
    the field sets swap back and forth; with open x faces the Mur update runs
    inside the pass."""
    from paper_1503_02464_amd.sim import Simulation
    g = grid(3, n, dx=0.05, cfl=0.7, order=2)
    f = inputs.random_fields(g.ncells, 1.0, seed=23)
    f["J"] = inputs.rng(24).normal(size=(3, g.ncells))
    if prec == "fp32":
        f = inputs.round_fields_f32(f)
    kw = dict(open_x=True, absorb=6) if open_x else {}
    s = Simulation(3, g.n, g.dx, g.dt, 2, prec, tile=(8, 4, 1), max_particles=1, **kw)
    assert s.lib.pic_tile_lds_bytes(s.ctx) > 0
    s.set_fields(f["E"], f["B"], f["J"])
    ref = {k: v.copy() for k, v in f.items()}
    first = [t.data_ptr() for t in s.fields["E"]]
    for step in range(3):
        s.yee_step()
        (O.yee_step_open if open_x else O.yee_step)(g, ref)
        swapped = [t.data_ptr() for t in s.fields["E"]] != first
        assert swapped == (step % 2 == 0), "the one-pass step writes the second set and swaps"
        compare_fields(prec, s.get_fields(), ref, keys=("E", "B"), what=f"one-pass yee, step {step}")
    s.close()


@pytest.mark.parametrize("prec,dims,order", VARIANTS, ids=VID)
def test_unfused_gather_push_deposit(prec, dims, order):
    g = small_grid(dims, order)
    sp, f = state(g, prec, 3, 0.3, 0.2, seed=30 + dims + order, random_positions=False)
    s = make_sim(g, prec, tiles(dims), max_particles=sp["w"].shape[0])
    s.set_fields(f["E"], f["B"])
    h = s.add_species(sp)
    s.zero_current()
    s.gather_push(h)
    s.deposit(h)
    s.check()
    ref_sp = O.copy_species(sp)
    ref_f = {k: v.copy() for k, v in f.items()}
    ref_f["J"][:] = 0
    assert O.push_deposit(g, ref_f, ref_sp) == 0
    compare_species(g, prec, s.get_species(h), ref_sp, "unfused")
    compare_fields(prec, s.get_fields(), ref_f, keys=("J",), what="unfused")
    s.close()


TILE_CASES = {
    # (tile, slack, particle layout): ragged occupancy, empty tiles, seam crossings
    "uniform": (None, 1, "uniform"),
    "slack0": (None, 0, "uniform"),
    "clustered": (None, 2, "clustered"),
    "one_tile": ("full", 1, "uniform"),
}


def clustered(g, prec, seed):
    """Particles only in the lower half of x (empty tiles), random cells, so
    tile counts are ragged."""
    npart = g.ncells * 2
    sp, f = state(g, prec, npart, 0.3, 0.2, seed, random_positions=True)
    sp["cell"][0] = sp["cell"][0] % (g.n[0] // 2)
    return sp, f


@pytest.mark.parametrize("case", list(TILE_CASES))
@pytest.mark.parametrize("prec,dims,order", VARIANTS, ids=VID)
def test_step_fused(prec, dims, order, case):
    tile, slack, layout = TILE_CASES[case]
    # one tile spanning the whole box: a smaller 3D box keeps it within 160 KB of LDS
    g = small_grid(dims, order, n3=(8, 6, 4)) if tile == "full" else small_grid(dims, order)
    tile = tuple(g.n) if tile == "full" else tiles(dims)
    if layout == "uniform":
        sp, f = state(g, prec, 3, 0.3, 0.2, seed=40 + dims + order)
    else:
        sp, f = clustered(g, prec, seed=50 + dims + order)
    s = make_sim(g, prec, tile, slack=slack, max_particles=sp["w"].shape[0])
    s.set_fields(f["E"], f["B"])
    h = s.add_species(sp)
    s.step(1)
    s.check()
    ref_sp = O.copy_species(sp)
    ref_f = {k: v.copy() for k, v in f.items()}
    assert O.step(g, ref_f, [ref_sp]) == 0
    compare_species(g, prec, s.get_species(h), ref_sp, f"fused {case}")
    compare_fields(prec, s.get_fields(), ref_f, what=f"fused {case}")
    s.close()


@pytest.mark.parametrize("prec,dims,order", VARIANTS, ids=VID)
def test_sort(prec, dims, order):
    g = small_grid(dims, order)
    sp, _ = clustered(g, prec, seed=60)
    tile = tiles(dims)
    s = make_sim(g, prec, tile, max_particles=sp["w"].shape[0])
    h = s.add_species(sp)
    s.sort(h)
    out = s.get_species(h)
    start = s.tile_start(h)
    keys = O.tile_keys(g, tile, out["cell"])
    assert np.all(np.diff(keys) >= 0), "keys not sorted"
    ref, ref_start = O.tile_sort(g, tile, sp)
    assert np.array_equal(start, ref_start), "tile offsets differ"
    # per tile the same particles (the order inside a tile is unspecified)
    a, b = by_weight(out), by_weight(ref)
    assert np.array_equal(a["w"], b["w"])
    for k in ("cell", "off", "u"):
        assert np.array_equal(a[k], b[k]), k
    s.close()


@pytest.mark.parametrize("prec,dims,order", VARIANTS, ids=VID)
def test_sort_by_previous_runs(prec, dims, order):
    """A re-sort of a species this context sorted before ranks particles run
    by run (the tile ranges of the previous sort): after pushing it must still
    be the tile permutation the oracle's sort gives for the moved particles."""
    g = small_grid(dims, order)
    sp, f = clustered(g, prec, seed=61)
    tile = tiles(dims)
    s = make_sim(g, prec, tile, sort_every=1 << 30, max_particles=sp["w"].shape[0])
    s.set_fields(f["E"], f["B"])
    h = s.add_species(sp)
    s.step(3)  # the first step sorts (unsorted input), the next two only push
    before = s.get_species(h)
    s.sort(h)
    out = s.get_species(h)
    start = s.tile_start(h)
    keys = O.tile_keys(g, tile, out["cell"])
    assert np.all(np.diff(keys) >= 0), "keys not sorted"
    ref, ref_start = O.tile_sort(g, tile, before)
    assert np.array_equal(start, ref_start), "tile offsets differ"
    a, b = by_weight(out), by_weight(ref)
    assert np.array_equal(a["w"], b["w"])
    for k in ("cell", "off", "u"):
        assert np.array_equal(a[k], b[k]), k
    s.check()
    s.close()


def test_sort_rejects_runs_that_do_not_partition():
    """If the tile ranges a sorted species carries were overwritten so that they
    cover particles twice, the re-sort writes nothing out of bounds and the
    next check reports PIC_ESTATE."""
    import torch
    from paper_1503_02464_amd._lib import PicError
    g = small_grid(3, 2)
    sp, _ = clustered(g, "fp32", seed=62)
    tile = tiles(3)
    s = make_sim(g, "fp32", tile, sort_every=1 << 30, max_particles=sp["w"].shape[0])
    h = s.add_species(sp)
    s.sort(h)
    npart = h.np
    bad = torch.zeros_like(h.tile_start)
    bad[1::2] = npart  # runs [0, np), [np, 0) -> empty, [0, np), ...: every particle counted several times
    bad[-1] = npart
    h.tile_start.copy_(bad)
    s.sort(h)
    with pytest.raises(PicError) as e:
        s.check()
    assert e.value.status == -7  # PIC_ESTATE
    s.close()


def test_c1_100_steps_fp64():
    """The small 2D workload (64x64, 4 ppc, linear, 0.7 CFL) for 100 steps, FP64."""
    from paper_1503_02464_amd.configs import uniform_2d_small
    w = uniform_2d_small()
    g = grid(2, w.n[:2], dx=w.dx[0], cfl=w.cfl, order=w.order)
    sp = inputs.uniform_plasma(w.n, 2, w.ppc, w.u_sigma, w.weight, w.seed)
    from gpu_helpers import unique_weights
    sp = unique_weights(sp, 7, scale=w.weight)
    s = make_sim(g, "fp64", w.tile, sort_every=4, max_particles=sp["w"].shape[0])
    h = s.add_species(sp)
    ref_sp = O.copy_species(sp)
    ref_f = O.new_fields(g)
    errs = []
    for step in range(w.steps):
        s.step(1)
        O.step(g, ref_f, [ref_sp])
        if step % 25 == 24 or step == w.steps - 1:
            got = s.get_species(h)
            gf = s.get_fields()
            a, b = by_weight(got), by_weight(ref_sp)
            errs.append((step, pos_err(g, a, b), rel(a["u"], b["u"]), rel(gf["E"], ref_f["E"])))
    s.check()
    last = errs[-1]
    assert last[1] < 1e-12 and last[2] < 1e-12 and last[3] < 1e-12, errs
    s.close()


@pytest.mark.parametrize("prec,dims,order", VARIANTS, ids=VID)
def test_diagnostics(prec, dims, order):
    g = small_grid(dims, order)
    sp, f = state(g, prec, 3, 0.3, 0.05, seed=70)
    s = make_sim(g, prec, tiles(dims), max_particles=sp["w"].shape[0])
    s.set_fields(f["E"], f["B"])
    h = s.add_species(sp)
    d0 = s.diagnostics()
    ref = O.diagnostics(g, f, [sp])
    tol = 1e-12 if prec == "fp64" else 1e-6
    assert abs(d0["UE"] - ref["UE"]) <= tol * ref["UE"]
    assert abs(d0["UB"] - ref["UB"]) <= tol * ref["UB"]
    # gamma - 1 of slow particles: the oracle's sqrt(1+u^2) - 1 loses ~1e-16/u^2 relative
    assert abs(d0["K"] - ref["K"]) <= max(tol, 1e-10) * ref["K"]
    assert abs(d0["Q"] - ref["Q"]) <= 1e-12 * abs(ref["Q"])
    assert abs(d0["rho_max"] - np.max(np.abs(ref["rho"]))) <= tol * np.max(np.abs(ref["rho"]))
    assert abs(d0["gauss_max"] - np.max(np.abs(ref["gauss"]))) <= max(tol, 1e-12) * np.max(np.abs(ref["gauss"]))
    assert np.isnan(d0["gauss_change"]) and np.isnan(d0["continuity"])
    # the charge density and Gauss's residual node by node (FP64 sums of an
    # FP32-exact state: round-off only, for both precisions)
    rho0, g0 = s.charge_density(gauss=True)
    assert rel(rho0, ref["rho"]) <= 1e-12, rel(rho0, ref["rho"])
    assert rel(g0, ref["gauss"]) <= 1e-12, rel(g0, ref["gauss"])
    s.step(1)
    ref_sp, ref_f = O.copy_species(sp), {k: v.copy() for k, v in f.items()}
    assert O.step(g, ref_f, [ref_sp]) == 0
    rho1, g1 = s.charge_density(gauss=True)
    tol1 = 1e-12 if prec == "fp64" else 2e-6  # one FP32 step: positions to 4e-7 cells
    assert rel(rho1, O.rho(g, [ref_sp])) <= tol1, rel(rho1, O.rho(g, [ref_sp]))
    ref_g1 = O.div(g, ref_f["E"]) - O.rho(g, [ref_sp])
    assert rel(g1, ref_g1) <= tol1, rel(g1, ref_g1)
    d1 = s.diagnostics()
    # continuity and Gauss's law hold to round-off on the GPU path too
    scale = d1["rho_max"]
    eps = 1e-13 if prec == "fp64" else 2e-6
    assert d1["continuity"] <= eps * scale / g.dt, (d1["continuity"], scale / g.dt)
    assert d1["gauss_change"] <= eps * scale * 10, (d1["gauss_change"], scale)
    assert abs(d1["Q"] - d0["Q"]) <= 1e-13 * abs(d0["Q"])
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_empty_and_tiny_species(prec):
    """np = 0 alongside a species of one particle; a particle exactly on a node and one on the seam."""
    g = small_grid(3, 2)
    sp, f = state(g, prec, 3, 0.3, 0.2, seed=80, random_positions=True)
    sp["cell"][:, 0] = [g.n[0] - 1, 0, g.n[2] - 1]
    sp["off"][:, 0] = [0.0, 0.5, 0.999]
    sp["off"][:, 1] = [0.0, 0.0, 0.0]
    empty = {"q": 1.0, "m": 1836.0, "cell": np.zeros((3, 0), np.int32), "off": np.zeros((3, 0)),
             "u": np.zeros((3, 0)), "w": np.zeros(0)}
    s = make_sim(g, prec, tiles(3), max_particles=3)
    s.set_fields(f["E"], f["B"])
    he = s.add_species(empty)
    h = s.add_species(sp)
    s.step(1)
    s.check()
    ref_sp = O.copy_species(sp)
    ref_f = {k: v.copy() for k, v in f.items()}
    O.step(g, ref_f, [ref_sp])
    compare_species(g, prec, s.get_species(h), ref_sp, "tiny")
    compare_fields(prec, s.get_fields(), ref_f, what="tiny")
    assert s.get_species(he)["w"].shape[0] == 0
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_fast_and_slow_particles(prec):
    """Displacements near the one-cell limit (gamma ~ 50) and tiny ones (cold
    heavy ions, ~1e-6 cells) in the same step."""
    g = small_grid(3, 2)
    sp, f = state(g, prec, 2, 0.0, 0.01, seed=90)
    npart = sp["w"].shape[0]
    r = inputs.rng(91)
    fast = r.random(npart) < 0.3
    u = r.normal(size=(3, npart))
    u = u / np.linalg.norm(u, axis=0) * np.where(fast, 50.0, 1e-4)
    sp["u"] = np.ascontiguousarray(u.astype(np.float32).astype(np.float64) if prec == "fp32" else u)
    s = make_sim(g, prec, tiles(3), max_particles=npart)
    s.set_fields(f["E"], f["B"])
    h = s.add_species(sp)
    s.step(1)
    s.check()
    ref_sp = O.copy_species(sp)
    ref_f = {k: v.copy() for k, v in f.items()}
    O.step(g, ref_f, [ref_sp])
    compare_species(g, prec, s.get_species(h), ref_sp, "fast/slow")
    compare_fields(prec, s.get_fields(), ref_f, what="fast/slow")
    s.close()


def test_non_finite_particle_is_flagged_and_frozen():
    """A NaN momentum (forced from the host) is reported as PIC_ECROSS by the
    next check; that particle stays put and deposits nothing, the others are exact."""
    from paper_1503_02464_amd import _lib as L
    g = small_grid(2, 1)
    sp, f = state(g, "fp64", 2, 0.3, 0.1, seed=95)
    bad = int(np.argmax(sp["w"]))
    sp["u"][0, bad] = np.nan
    s = make_sim(g, "fp64", tiles(2), max_particles=sp["w"].shape[0])
    s.set_fields(f["E"], f["B"])
    h = s.add_species(sp)
    s.step(1)
    with pytest.raises(L.PicError) as ei:
        s.check()
    assert ei.value.status == L.PIC_ECROSS
    s.check()  # the flag is cleared after it is reported
    got = by_weight(s.get_species(h))
    keep = np.ones(sp["w"].shape[0], bool)
    keep[bad] = False
    ref_sp = {k: (v[..., keep] if isinstance(v, np.ndarray) else v) for k, v in sp.items()}
    ref_sp = O.copy_species(ref_sp)
    ref_f = {k: v.copy() for k, v in f.items()}
    O.step(g, ref_f, [ref_sp])
    last = got["w"].shape[0] - 1  # the NaN particle has the largest weight
    assert got["cell"][0, last] == sp["cell"][0, bad] and got["off"][0, last] == sp["off"][0, bad]
    rest = {k: (v[..., :last] if isinstance(v, np.ndarray) else v) for k, v in got.items()}
    compare_species(g, "fp64", rest, ref_sp, "nan neighbours")
    compare_fields("fp64", s.get_fields(), ref_f, keys=("J",), what="nan neighbours")
    s.close()


@pytest.mark.parametrize("dims,order", [(2, 1), (2, 2), (3, 1), (3, 2)])
def test_step_fused_fp32_lds_accumulation(dims, order):
    """The FP32 state with the current tile accumulated in FP32 (the default is FP64)."""
    from paper_1503_02464_amd.sim import Simulation
    g = small_grid(dims, order)
    sp, f = state(g, "fp32", 3, 0.3, 0.2, seed=100 + dims + order)
    s = Simulation(g.dims, g.n, g.dx, g.dt, g.order, "fp32", tile=tiles(dims), slack=1, sort_every=4,
                   max_particles=sp["w"].shape[0], current_accum="fp32")
    s.set_fields(f["E"], f["B"])
    h = s.add_species(sp)
    s.step(1)
    s.check()
    ref_sp = O.copy_species(sp)
    ref_f = {k: v.copy() for k, v in f.items()}
    O.step(g, ref_f, [ref_sp])
    compare_species(g, "fp32", s.get_species(h), ref_sp, "fp32 accumulation")
    compare_fields("fp32", s.get_fields(), ref_f, what="fp32 accumulation")
    s.close()


@pytest.mark.parametrize("order", [1, 2])
def test_sort_levels_spread_nodes(order):
    """Inside a tile the sort lays particles out level by level, so a 64-lane
    window rarely holds two particles with the same nearest node (cell for the
    linear shape), whatever order they came in (here: cell by cell)."""
    g = grid(3, (16, 16, 16), dx=0.05, cfl=0.7, order=order)
    sp = inputs.uniform_plasma(g.n, 3, 8, 0.05, 1.0, seed=110)  # 8 per cell, cell by cell
    tile = (8, 8, 8)
    s = make_sim(g, "fp32", tile, max_particles=sp["w"].shape[0])
    h = s.add_species(sp)
    s.sort(h)
    out = s.get_species(h)
    start = s.tile_start(h)
    node = out["cell"].astype(np.int64).copy()
    if order == 2:
        node = (node + (out["off"] >= 0.5)) % np.array(g.n)[:, None]
    key = node[0] + g.n[0] * (node[1] + g.n[1] * node[2])
    dup = total = 0
    for t in range(len(start) - 1):
        for b in range(start[t], start[t + 1], 64):
            k = key[b:min(b + 64, start[t + 1])]
            dup += k.size - np.unique(k).size
            total += k.size
    assert dup <= 0.05 * total, (dup, total)
    # the unsorted input has 7 duplicates in every 8
    k0 = (sp["cell"][0] + g.n[0] * (sp["cell"][1] + g.n[1] * sp["cell"][2]))[:4096]
    assert sum(k0[i:i + 64].size - np.unique(k0[i:i + 64]).size for i in range(0, 4096, 64)) > 0.8 * 4096
    s.close()
