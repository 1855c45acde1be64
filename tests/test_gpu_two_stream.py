"""The two-stream workload (the paper's Sec. 4 scaling case) on the HIP path:
a small two-beam box against the FP64 oracle step by step, and the GPU's
linear growth against the cold-beam rate that pins the oracle."""
import math

import numpy as np
import pytest

import oracle as O
import pins
from gpu_helpers import compare_fields, compare_species, grid, unique_weights
from paper_1503_02464_amd import inputs
from paper_1503_02464_amd.sim import Simulation

pytestmark = pytest.mark.gpu


def beams(g, prec, ppc, seed):
    dV = float(np.prod([g.dx[d] for d in range(g.dims)]))
    a, b = inputs.two_beams(g.n, g.dims, ppc, 0.1, 0.001, 0.5 * dV / ppc, seed)
    a = unique_weights(a, seed + 10, scale=0.5 * dV / ppc)
    b = unique_weights(b, seed + 11, scale=0.5 * dV / ppc)
    if prec == "fp32":
        a, b = inputs.round_f32(a), inputs.round_f32(b)
    return a, b


def test_two_beams_fp64_twenty_steps():
    """Two beams of 6 particles per cell each, 16x16x8 cells, quadratic shape,
    20 fused steps re-sorted every 4: particles, E, B and J to 1e-12."""
    g = grid(3, (16, 16, 8), dx=0.05, cfl=0.7, order=2)
    a, b = beams(g, "fp64", 6, 600)
    s = Simulation(3, g.n, g.dx, g.dt, 2, "fp64", tile=(8, 4, 4), slack=1, sort_every=4,
                   max_particles=a["w"].shape[0])
    ha, hb = s.add_species(a), s.add_species(b)
    ref = [O.copy_species(a), O.copy_species(b)]
    ref_f = O.new_fields(g)
    for _ in range(20):
        s.step(1)
        assert O.step(g, ref_f, ref) == 0
    s.check()
    compare_species(g, "fp64", s.get_species(ha), ref[0], "beam +")
    compare_species(g, "fp64", s.get_species(hb), ref[1], "beam -")
    compare_fields("fp64", s.get_fields(), ref_f, what="two beams")
    s.close()


def test_two_beams_fp32_one_step():
    """The FP32 state (fixed-point on-chip current) for one step from an
    FP32-exact state with random fields, against the FP64 oracle."""
    g = grid(3, (16, 16, 8), dx=0.05, cfl=0.7, order=2)
    a, b = beams(g, "fp32", 6, 610)
    f = inputs.round_fields_f32(inputs.random_fields(g.ncells, 0.05, seed=611))
    s = Simulation(3, g.n, g.dx, g.dt, 2, "fp32", tile=(8, 4, 4), slack=1, sort_every=4,
                   max_particles=a["w"].shape[0])
    s.set_fields(f["E"], f["B"])
    ha, hb = s.add_species(a), s.add_species(b)
    ref = [O.copy_species(a), O.copy_species(b)]
    ref_f = {k: v.copy() for k, v in f.items()}
    s.step(1)
    assert O.step(g, ref_f, ref) == 0
    compare_species(g, "fp32", s.get_species(ha), ref[0], "beam +")
    compare_species(g, "fp32", s.get_species(hb), ref[1], "beam -")
    compare_fields("fp32", s.get_fields(), ref_f, what="two beams fp32")
    s.close()


@pytest.mark.parametrize("prec,eps,lo,hi,tol", [("fp64", 1e-7, 7.0, 11.5, 0.02), ("fp32", 1e-5, 6.0, 9.0, 0.03)])
def test_two_stream_growth_on_the_gpu(prec, eps, lo, hi, tol):
    """The quiet-start box of the oracle's growth pin, stepped by the fused GPU
    path: the seeded mode grows at the cold-beam rate (FP32 starts from a
    larger seed, so that FP32 rounding of the momenta stays far below it, and
    fits an earlier window, before saturation)."""
    g, sps, k = pins.two_stream_box(eps=eps)
    if prec == "fp32":
        sps = [inputs.round_f32(sp) for sp in sps]
    gam = pins.two_stream_rate(0.1, k)
    steps = int(math.ceil((hi + 0.1) / gam / g.dt))
    s = Simulation(2, g.n, g.dx, g.dt, g.order, prec, tile=(8, 4), slack=1, sort_every=8,
                   max_particles=sps[0]["w"].shape[0])
    for sp in sps:
        s.add_species(sp)
    amp = []
    for _ in range(steps):
        s.step(1)
        Ex = s.fields["E"][0].double().cpu().numpy()
        amp.append(pins.mode_amplitude(g, Ex, k))
    s.check()
    s.close()
    rate = pins.growth_rate(amp, g.dt, gam, lo, hi)
    assert abs(rate / gam - 1) < tol, (rate, gam)
