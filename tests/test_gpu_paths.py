"""Paths of the fused kernel that the uniform workloads rarely take, against
the FP64 oracle: particles that drift out of their tile's slack between
sorts (the HBM straggler path), more window-changing particles in one tile
than its LDS list holds (deposited in place), more non-empty tiles than
resident workgroups (the per-XCD tile queues), and 3D tiles with too few
particles to stage (stepped by the straggler kernel).  FP64 to 1e-12; FP32
one step from an FP32-representable state (gpu_helpers.TOL)."""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_helpers import compare_fields, compare_species, grid, make_sim, state, unique_weights
from paper_1503_02464_amd import inputs

pytestmark = pytest.mark.gpu


def drifting(g, prec, ppc, u_mean, seed):
    sp = inputs.uniform_plasma(g.n, g.dims, ppc, 0.05, 1.0, seed, u_mean=u_mean)
    sp = inputs.shuffle(sp, seed + 1)
    sp = unique_weights(sp, seed + 2, scale=float(np.prod(g.dx[:g.dims])) / ppc)
    f = inputs.random_fields(g.ncells, 0.1, seed + 3)
    if prec == "fp32":
        sp, f = inputs.round_f32(sp), inputs.round_fields_f32(f)
    return sp, f


def gpu_state(s, h):
    sp = s.get_species(h)
    f = s.get_fields()
    return sp, f


def test_straggler_count_per_launch():
    """The fused launches alternate two banks of counters, each cleared by the
    launch before it: the launch after a sort reports no straggler although
    the launch before it had many, and every launch's particles and fields
    stay the oracle's (FP64, 3D, slack 0)."""
    g = grid(3, (16, 16, 8), dx=0.05, cfl=0.7, order=2)
    sp, f = drifting(g, "fp64", 2, (2.0, -1.0, 0.5), seed=640)
    s = make_sim(g, "fp64", (8, 4, 4), slack=0, sort_every=1 << 30, max_particles=sp["w"].shape[0])
    s.set_fields(f["E"], f["B"])
    h = s.add_species(sp)
    ref_sp, ref_f = O.copy_species(sp), {k: v.copy() for k, v in f.items()}
    counts = []
    for n in range(4):
        if n == 2:
            s.sort(h)
        s.step(1)
        counts.append(s.straggler_count())
        assert O.step(g, ref_f, [ref_sp]) == 0
    s.check()
    assert counts[0] == 0 and counts[2] == 0, counts
    assert counts[1] > sp["w"].shape[0] // 20 and counts[3] > sp["w"].shape[0] // 20, counts
    compare_species(g, "fp64", s.get_species(h), ref_sp, "straggler banks")
    compare_fields("fp64", s.get_fields(), ref_f, what="straggler banks")
    s.close()


@pytest.mark.parametrize("prec,dims", [(p, d) for p in ("fp64", "fp32") for d in (2, 3)])
def test_stragglers(prec, dims):
    """Slack 0 and no re-sort: after the first step every particle that left its
    tile is a straggler.  FP64: three steps against three oracle steps.  FP32:
    the third step against one oracle step from the GPU's second state."""
    g = grid(dims, (32, 16) if dims == 2 else (16, 16, 8), dx=0.05, cfl=0.7, order=2)
    sp, f = drifting(g, prec, 2, (2.0, -1.0, 0.5), seed=600 + dims)
    tile = (8, 4, 1) if dims == 2 else (8, 4, 4)
    s = make_sim(g, prec, tile, slack=0, sort_every=1 << 30, max_particles=sp["w"].shape[0])
    s.set_fields(f["E"], f["B"])
    h = s.add_species(sp)
    ref_sp, ref_f = O.copy_species(sp), {k: v.copy() for k, v in f.items()}
    for n in range(3):
        if prec == "fp32" and n == 2:
            ref_sp, ref_f = gpu_state(s, h)
            ref_sp["q"], ref_sp["m"] = sp["q"], sp["m"]
            ref_f["J"] = np.zeros_like(ref_f["J"])
        s.step(1)
        if prec == "fp64" or n == 2:
            assert O.step(g, ref_f, [ref_sp]) == 0
    s.check()
    assert s.straggler_count() > sp["w"].shape[0] // 20, s.straggler_count()
    compare_species(g, prec, s.get_species(h), ref_sp, "stragglers")
    compare_fields(prec, s.get_fields(), ref_f, what="stragglers")
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_wide_list_overflow(prec):
    """Several thousand particles in one tile all cross a half-cell in x in the
    same step (so each changes its deposit window): more than the LDS list of
    the production tile shape holds, so the rest deposit in place."""
    g = grid(3, (16, 16, 16), dx=0.05, cfl=0.7, order=2)
    r = inputs.rng(620)
    npart = 6000
    sp = {"q": -1.0, "m": 1.0, "cell": np.zeros((3, npart), np.int32), "off": np.zeros((3, npart)),
          "u": np.zeros((3, npart)), "w": np.ones(npart)}
    sp["cell"][0] = r.integers(0, 8, npart)
    sp["cell"][1] = r.integers(0, 8, npart)
    sp["cell"][2] = r.integers(0, 4 if prec == "fp64" else 8, npart)  # one tile of 8x8x4 (FP64) or 8^3 (FP32)
    sp["off"][0] = 0.5 - r.uniform(0.001, 0.05, npart)  # just below the half-cell, heading +x
    sp["off"][1] = r.random(npart)
    sp["off"][2] = r.random(npart)
    sp["u"][0] = r.uniform(0.6, 1.5, npart)
    sp["u"][1:] = r.normal(0, 0.1, (2, npart))
    sp = unique_weights(sp, 621, scale=1e-3)
    f = inputs.random_fields(g.ncells, 0.05, 622)
    if prec == "fp32":
        sp, f = inputs.round_f32(sp), inputs.round_fields_f32(f)
    tile = (8, 8, 8) if prec == "fp32" else (8, 8, 4)
    s = make_sim(g, prec, tile, slack=1, sort_every=4, max_particles=npart)
    s.set_fields(f["E"], f["B"])
    h = s.add_species(sp)
    s.step(1)
    s.check()
    ref_sp, ref_f = O.copy_species(sp), {k: v.copy() for k, v in f.items()}
    assert O.step(g, ref_f, [ref_sp]) == 0
    crossed = np.sum((ref_sp["off"][0] >= 0.5) | (ref_sp["cell"][0] != sp["cell"][0]))
    assert crossed > 4 * 512, crossed
    compare_species(g, prec, s.get_species(h), ref_sp, "wide overflow")
    compare_fields(prec, s.get_fields(), ref_f, what="wide overflow")
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_wide_list_overflow_2d(prec):
    """The same in 2D on the 8x8 tiles of dense foils, whose small boxes leave
    room for a list twice as long (1024 entries in FP32, 512 in FP64): 6000
    particles of one tile cross a half-cell in x, most of them in y too, with
    out-of-plane momentum (the J_z of the in-place deposit)."""
    g = grid(2, (16, 16), dx=0.05, cfl=0.7, order=2)
    r = inputs.rng(630)
    npart = 6000
    sp = {"q": -1.0, "m": 1.0, "cell": np.zeros((3, npart), np.int32), "off": np.zeros((3, npart)),
          "u": np.zeros((3, npart)), "w": np.ones(npart)}
    sp["cell"][0] = r.integers(0, 8, npart)
    sp["cell"][1] = r.integers(0, 8, npart)
    sp["off"][0] = 0.5 - r.uniform(0.001, 0.05, npart)  # just below the half-cell, heading +x
    sp["off"][1] = r.random(npart)
    sp["u"][0] = r.uniform(0.6, 1.5, npart)
    sp["u"][1] = r.normal(0, 0.6, npart)
    sp["u"][2] = r.normal(0, 0.5, npart)
    sp = unique_weights(sp, 631, scale=1e-3)
    f = inputs.random_fields(g.ncells, 0.05, 632)
    if prec == "fp32":
        sp, f = inputs.round_f32(sp), inputs.round_fields_f32(f)
    s = make_sim(g, prec, (8, 8), slack=1, sort_every=4, max_particles=npart)
    s.set_fields(f["E"], f["B"])
    h = s.add_species(sp)
    s.step(1)
    s.check()
    ref_sp, ref_f = O.copy_species(sp), {k: v.copy() for k, v in f.items()}
    assert O.step(g, ref_f, [ref_sp]) == 0
    crossed = np.sum((ref_sp["off"][0] >= 0.5) | (ref_sp["cell"][0] != sp["cell"][0]))
    assert crossed > 4 * 1024, crossed
    compare_species(g, prec, s.get_species(h), ref_sp, "wide overflow 2D")
    compare_fields(prec, s.get_fields(), ref_f, what="wide overflow 2D")
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_more_tiles_than_workgroups(prec):
    """More non-empty tiles than the device runs workgroups of the production
    tile shape at once, so workgroups take further tiles from the per-XCD
    queues (and from other XCDs' queues at the end); two steps, each sorting."""
    g = grid(3, (64, 64, 40), dx=0.05, cfl=0.7, order=2)
    sp, f = drifting(g, prec, 2 if prec == "fp64" else 4, (0.0, 0.0, 0.0), seed=640)
    tile = (8, 8, 8) if prec == "fp32" else (8, 8, 4)
    s = make_sim(g, prec, tile, slack=1, sort_every=1, max_particles=sp["w"].shape[0])
    assert s.ntiles > 256
    s.set_fields(f["E"], f["B"])
    h = s.add_species(sp)
    ref_sp, ref_f = O.copy_species(sp), {k: v.copy() for k, v in f.items()}
    nsteps = 2 if prec == "fp64" else 1
    for _ in range(nsteps):
        s.step(1)
        assert O.step(g, ref_f, [ref_sp]) == 0
    s.check()
    compare_species(g, prec, s.get_species(h), ref_sp, "queues")
    compare_fields(prec, s.get_fields(), ref_f, what="queues")
    s.close()


def test_sort_every_zero_sorts_only_unsorted_species():
    """sort_every = 0: the first step sorts the unsorted species, later steps
    keep its order (the array set never swaps again), and four steps still
    match four oracle steps."""
    g = grid(3, (16, 16, 8), dx=0.05, cfl=0.7, order=2)
    sp, f = drifting(g, "fp64", 2, (0.3, 0.0, -0.2), seed=650)
    s = make_sim(g, "fp64", (8, 8, 4), slack=1, sort_every=0, max_particles=sp["w"].shape[0])
    s.set_fields(f["E"], f["B"])
    h = s.add_species(sp)
    assert not h.struct.sorted
    s.step(1)
    assert h.struct.sorted
    cell_ptr, start = h.struct.cell, s.tile_start(h).copy()
    s.step(3)
    s.check()
    assert h.struct.cell == cell_ptr and np.array_equal(s.tile_start(h), start)
    ref_sp, ref_f = O.copy_species(sp), {k: v.copy() for k, v in f.items()}
    for _ in range(4):
        assert O.step(g, ref_f, [ref_sp]) == 0
    compare_species(g, "fp64", s.get_species(h), ref_sp, "sort_every 0")
    compare_fields("fp64", s.get_fields(), ref_f, what="sort_every 0")
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_resort_long_and_short_runs(prec):
    """The count pass ranks a run of at most 5 x 1024 particles in registers
    and a longer one through HBM.  A box with 24 particles per cell in its low-x
    half (6,144 per 8x8x4 tile) and 4 elsewhere (1,024 per tile) takes both;
    after four pushes the re-sort by the previous runs must be the oracle's tile
    permutation, and the next push must match the oracle."""
    g = grid(3, (16, 16, 8), dx=0.05, cfl=0.7, order=2)
    tile = (8, 8, 4)
    thin = inputs.uniform_plasma(g.n, 3, 4, 0.05, 1.0, 130, u_mean=(0.3, -0.2, 0.1))
    thick = inputs.uniform_plasma(g.n, 3, 20, 0.05, 1.0, 131, u_mean=(0.3, -0.2, 0.1))
    keep = thick["cell"][0] < 8
    sp = dict(thin)
    for k in ("cell", "off", "u"):
        sp[k] = np.ascontiguousarray(np.concatenate([thin[k], thick[k][:, keep]], axis=1))
    sp["w"] = np.ascontiguousarray(np.concatenate([thin["w"], thick["w"][keep]]))
    sp = inputs.shuffle(sp, 132)
    sp = unique_weights(sp, 133, scale=float(np.prod(g.dx[:3])) / 12)
    f = inputs.random_fields(g.ncells, 0.1, 134)
    if prec == "fp32":
        sp, f = inputs.round_f32(sp), inputs.round_fields_f32(f)
    s = make_sim(g, prec, tile, slack=1, sort_every=1 << 30, max_particles=sp["w"].shape[0])
    s.set_fields(f["E"], f["B"])
    h = s.add_species(sp)
    s.step(4)  # the first step sorts (unsorted input, in chunks), the next three only push
    runs = np.diff(s.tile_start(h))
    assert runs.max() > 5 * 1024 and 0 < runs.min() <= 5 * 1024, (runs.min(), runs.max())
    before = s.get_species(h)
    s.sort(h)
    out = s.get_species(h)
    start = s.tile_start(h)
    ref, ref_start = O.tile_sort(g, tile, before)
    assert np.array_equal(start, ref_start), "tile offsets differ"
    keys = O.tile_keys(g, tile, out["cell"])
    assert np.all(np.diff(keys) >= 0), "keys not sorted"
    order_a, order_b = np.argsort(out["w"], kind="stable"), np.argsort(ref["w"], kind="stable")
    assert np.array_equal(out["w"][order_a], ref["w"][order_b])
    for k in ("cell", "off", "u"):
        assert np.array_equal(out[k][:, order_a], ref[k][:, order_b]), k
    ref_sp, ref_f = s.get_species(h), s.get_fields()
    s.step(1)
    s.check()
    assert O.step(g, ref_f, [ref_sp]) == 0
    compare_species(g, prec, s.get_species(h), ref_sp, "after a re-sort of long and short runs")
    compare_fields(prec, s.get_fields(), ref_f, what="after a re-sort of long and short runs")
    s.close()


@pytest.mark.parametrize("prec,dims,order", [(p, d, m) for p in ("fp64", "fp32") for d in (2, 3) for m in (1, 2)])
def test_crossing_particles_on_one_two_three_axes(prec, dims, order):
    """Particles whose nearest node (cell, for the linear shape) changes along
    one, two or all three axes in one step take the workgroup's list of crossing
    particles, whose deposit relabels each particle's axes so that a crossed one
    leads.  The grid (16^3, or 32^2) is at least as wide as the tile boxes, so the
    staging and merge take the single-period wrap as well.  One step against the
    oracle."""
    g = grid(dims, (16, 16, 16) if dims == 3 else (32, 32), dx=0.05, cfl=0.7, order=order)
    sp, f = state(g, prec, 2, 0.0, 0.01, seed=140)
    npart = sp["w"].shape[0]
    r = inputs.rng(141)
    u = r.normal(size=(3, npart))
    u = u / np.linalg.norm(u, axis=0) * r.uniform(0.5, 6.0, npart)  # 0.2 to 0.4 cells per step along an axis
    sp["u"] = np.ascontiguousarray(u.astype(np.float32).astype(np.float64) if prec == "fp32" else u)
    tile = (16, 16, 1) if dims == 2 else ((8, 8, 4) if prec == "fp64" else (8, 8, 8))
    s = make_sim(g, prec, tile, max_particles=npart)
    s.set_fields(f["E"], f["B"])
    h = s.add_species(sp)
    s.sort(h)
    s.step(1)
    s.check()
    ref_sp = O.copy_species(sp)
    ref_f = {k: v.copy() for k, v in f.items()}
    assert O.step(g, ref_f, [ref_sp]) == 0
    # how many axes each particle crossed, from the oracle's move
    n = np.array(g.n)[:dims, None]
    if order == 2:
        before = (sp["cell"][:dims] + (sp["off"][:dims] >= 0.5)) % n
        after = (ref_sp["cell"][:dims] + (ref_sp["off"][:dims] >= 0.5)) % n
    else:
        before, after = sp["cell"][:dims] % n, ref_sp["cell"][:dims] % n
    axes = (before != after).sum(axis=0)
    counts = [int(np.sum(axes == k)) for k in range(dims + 1)]
    assert min(counts[1:]) >= 20, counts
    compare_species(g, prec, s.get_species(h), ref_sp, f"crossers {counts}")
    compare_fields(prec, s.get_fields(), ref_f, what=f"crossers {counts}")
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_sparse_tiles(prec):
    """Half the 3D box dense (256 particles per tile), the other half with a
    few particles per tile, some in no tile at all: the in-place launches
    leave the sparse tiles to the straggler kernel, the launches that fold a
    sort's copy take every tile.  FP64: four steps (two sorts) against four
    oracle steps; FP32: an in-place step after a sort against one oracle step
    from the GPU's state."""
    g = grid(3, (16, 16, 8), dx=0.05, cfl=0.7, order=2)
    r = inputs.rng(640)
    dense = inputs.uniform_plasma((8, 16, 8), 3, 2, 0.05, 1.0, 641)  # x < 8: 2048 particles over 8 tiles
    nsp = 37  # x >= 8: a few particles in each of some of the 8 tiles there
    cell = np.concatenate([dense["cell"], np.stack([r.integers(8, 16, nsp), r.integers(0, 16, nsp),
                                                    r.integers(0, 8, nsp)]).astype(np.int32)], axis=1)
    npart = cell.shape[1]
    sp = {"q": -1.0, "m": 1.0, "cell": cell, "off": r.random((3, npart)), "u": r.normal(0, 0.05, (3, npart)),
          "w": np.ones(npart)}
    sp = unique_weights(sp, 642, scale=0.05 ** 3 / 2)
    f = inputs.random_fields(g.ncells, 0.1, 643)
    if prec == "fp32":
        sp, f = inputs.round_f32(sp), inputs.round_fields_f32(f)
    s = make_sim(g, prec, (8, 4, 4), slack=1, sort_every=2, max_particles=npart)
    s.set_fields(f["E"], f["B"])
    h = s.add_species(sp)
    ref_sp, ref_f = O.copy_species(sp), {k: v.copy() for k, v in f.items()}
    for n in range(4):  # steps 0 and 2 sort (and fold the copy), 1 and 3 run in place
        if prec == "fp32" and n == 3:
            ref_sp, ref_f = gpu_state(s, h)
            ref_sp["q"], ref_sp["m"] = sp["q"], sp["m"]
            ref_f["J"] = np.zeros_like(ref_f["J"])
        s.step(1)
        if prec == "fp64" or n == 3:
            assert O.step(g, ref_f, [ref_sp]) == 0
    s.check()
    compare_species(g, prec, s.get_species(h), ref_sp, "sparse tiles")
    compare_fields(prec, s.get_fields(), ref_f, what="sparse tiles")
    s.close()


@pytest.mark.parametrize("dims", [2, 3])
def test_weights_raised_after_the_tile_bounds_were_taken(dims):
    """FP32 state: the first fused launch after a sort finds each tile's
    largest weight (the scale of its fixed-point current) and the later ones
    reuse it.  Weights raised fourfold between steps, without a sort, must
    not overflow that scale: those particles take the HBM path, and one step
    from the changed state matches the oracle."""
    g = grid(dims, (32, 16) if dims == 2 else (16, 16, 8), dx=0.05, cfl=0.7, order=2)
    sp, f = drifting(g, "fp32", 4, (0.3, -0.2, 0.1), seed=650 + dims)
    tile = (8, 4, 1) if dims == 2 else (8, 4, 4)
    s = make_sim(g, "fp32", tile, slack=1, sort_every=1 << 30, max_particles=sp["w"].shape[0])
    s.set_fields(f["E"], f["B"])
    h = s.add_species(sp)
    s.step(2)  # the first step sorts and takes the bounds, the second reuses them
    w = h.current()["w"]
    heavy = torch.arange(0, h.np, 7, device=w.device)
    w[heavy] *= 4.0
    ref_sp, ref_f = gpu_state(s, h)
    ref_sp["q"], ref_sp["m"] = sp["q"], sp["m"]
    ref_f["J"] = np.zeros_like(ref_f["J"])
    s.step(1)
    s.check()
    assert s.straggler_count() >= heavy.numel() * 9 // 10, s.straggler_count()
    assert O.step(g, ref_f, [ref_sp]) == 0
    compare_species(g, "fp32", s.get_species(h), ref_sp, "raised weights")
    compare_fields("fp32", s.get_fields(), ref_f, what="raised weights")
    s.close()
