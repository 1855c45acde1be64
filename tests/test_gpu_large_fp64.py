"""An FP64 species past 4 GiB per particle array: 512x512x256 cells at 9 ppc
(603,979,776 particles; each FP64 offset, momentum and weight array spans 4.5
GiB), quadratic shape, the FP64 launch configuration (8x8x4 tiles, slack 1).
The fused kernel forms 32-bit byte offsets only while every array spans at
most 4 GiB, so here it takes its 64-bit path, and the sort indexes past 2^29.

Sampled particles (random ones and the last 4096 of the array) after a step
that does not re-sort, against the oracle's gather, Boris and move from the
GPU's fields of the step before (FP64, 1e-12), as the full-size FP32 test does
for the benchmark box."""
import math

import numpy as np
import pytest
import torch

import oracle as O
from gpu_helpers import TOL
from paper_1503_02464_amd import inputs
from paper_1503_02464_amd.configs import BENCH_LAUNCH
from paper_1503_02464_amd.sim import Simulation, unpack_cells

pytestmark = pytest.mark.gpu

N = (512, 512, 256)
PPC = 9


def sample(sim, h, idx):
    cur = h.current()
    it = torch.as_tensor(idx, device=sim.device)
    return {"q": -1.0, "m": 1.0, "cell": unpack_cells(cur["cell"][it].cpu().numpy(), sim.bits),
            "off": np.stack([t[it].double().cpu().numpy() for t in cur["off"]]),
            "u": np.stack([t[it].double().cpu().numpy() for t in cur["u"]]),
            "w": cur["w"][it].double().cpu().numpy()}


def test_fp64_species_past_4gib_arrays():
    npart = N[0] * N[1] * N[2] * PPC
    assert npart * 8 > 1 << 32
    free, _ = torch.cuda.mem_get_info()
    need = 2 * npart * 60 + npart * 44 + 16 * N[0] * N[1] * N[2] * 8
    if free < 1.2 * need:
        pytest.skip(f"needs about {need / 2**30:.0f} GiB of device memory")
    dx = (0.05, 0.05, 0.05)
    dt = 0.7 / math.sqrt(sum(1.0 / d ** 2 for d in dx))
    lc = BENCH_LAUNCH["fp64"]
    sim = Simulation(3, N, dx, dt, 2, "fp64", tile=lc["tile"], slack=lc["slack"], sort_every=lc["sort_every"],
                     max_particles=npart)
    h = sim.new_species(-1.0, 1.0, npart)
    weight = 0.05 ** 3 / PPC
    inputs.uniform_plasma_device(h.sets[0], N, 3, sim.bits, PPC, (0.0, 0.0, 0.0), 0.05, weight, seed=1200)
    sim.step(1)  # sorts (the copy folded into the push), deposits, Yee: E, B non-zero
    g = O.Grid(3, N, dx, dt, 2)
    rng = inputs.rng(1201)
    idx = np.concatenate([np.sort(rng.choice(npart - 4096, 4096, replace=False)), np.arange(npart - 4096, npart)])
    before = sample(sim, h, idx)
    f1 = sim.get_fields()
    sim.step(1)  # no re-sort: every particle keeps its index
    sim.check()
    after = sample(sim, h, idx)
    sim.close()
    ref = O.copy_species(before)
    EB = O.gather(g, f1["E"], f1["B"], ref["cell"], ref["off"])
    ref["u"] = O.boris(ref["q"], ref["m"], g.dt, EB, ref["u"])
    ref["cell"], ref["off"], _, bad = O.move(g, ref["u"], ref["cell"], ref["off"])
    assert bad == 0
    assert np.array_equal(after["w"], ref["w"])
    t = TOL["fp64"]
    du = np.max(np.abs(after["u"] - ref["u"])) / np.max(np.abs(ref["u"]))
    n = np.array(g.n)[:, None]
    dpos = (after["cell"] + after["off"] - ref["cell"] - ref["off"] + n / 2) % n - n / 2
    assert du <= t["u"], du
    assert np.max(np.abs(dpos)) <= t["pos"], np.max(np.abs(dpos))
    assert np.abs(f1["E"]).max() > 0  # the sampled step gathered non-zero fields
