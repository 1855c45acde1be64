"""Parity at the benchmark's full size and launch configuration: the 3D3V
thermal plasma, 256^3 cells, 8 ppc (134,217,728 particles), quadratic shape,
FP32 state, 8x8x8 tiles, slack 1, sort every 12 steps, FP64 LDS current.

The oracle cannot step the whole box in a test, so it checks what it can
compute piecewise: sampled particles of a step that does not re-sort (the
particle order is kept, so indices match), the current inside sample boxes
from every particle that can reach them, and E, B everywhere from the GPU's
current; plus the continuity and Gauss residuals from the FP64 diagnostics."""
import numpy as np
import pytest
import torch

import oracle as O
from gpu_helpers import TOL
from paper_1503_02464_amd import inputs
from paper_1503_02464_amd.configs import BENCH_LAUNCH, thermal_3d
from paper_1503_02464_amd.sim import Simulation, unpack_cells

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def run():
    w = thermal_3d()
    lc = BENCH_LAUNCH["fp32"]
    sp = inputs.uniform_plasma(w.n, 3, w.ppc, w.u_sigma, w.weight, w.seed)
    sim = Simulation(3, w.n, w.dx, w.dt, w.order, "fp32", tile=lc["tile"], slack=lc["slack"],
                     sort_every=lc["sort_every"], max_particles=sp["w"].shape[0])
    h = sim.add_species(sp)
    del sp
    d0 = sim.diagnostics()
    sim.step(1)  # sorts, pushes, deposits, Yee: E^1, B^1 non-zero
    d1 = sim.diagnostics()
    g = O.Grid(3, w.n, w.dx, w.dt, w.order)
    # state after step 1 (on device), then one more step without a re-sort
    cur = h.current()
    npart = h.np
    state1 = {"cell": cur["cell"][:npart].clone(), "off": [t[:npart].clone() for t in cur["off"]],
              "u": [t[:npart].clone() for t in cur["u"]], "w": cur["w"][:npart].clone()}
    f1 = sim.get_fields()
    sim.step(1)
    d2 = sim.diagnostics()
    sim.check()
    cur2 = h.current()
    f2 = sim.get_fields()
    yield dict(w=w, g=g, sim=sim, h=h, state1=state1, f1=f1, f2=f2, cur2=cur2, npart=npart, d=(d0, d1, d2))
    sim.close()


def host_species(sim, st, idx, q=-1.0, m=1.0):
    idx_t = torch.as_tensor(idx, device=st["cell"].device)
    cell = unpack_cells(st["cell"][idx_t].cpu().numpy(), sim.bits)
    return {"q": q, "m": m, "cell": cell,
            "off": np.stack([t[idx_t].double().cpu().numpy() for t in st["off"]]),
            "u": np.stack([t[idx_t].double().cpu().numpy() for t in st["u"]]),
            "w": st["w"][idx_t].double().cpu().numpy()}


def test_sampled_particles(run):
    sim, g = run["sim"], run["g"]
    idx = np.sort(inputs.rng(300).choice(run["npart"], 8192, replace=False))
    before = host_species(sim, run["state1"], idx)
    after = host_species(sim, run["cur2"], idx)
    ref = O.copy_species(before)
    EB = O.gather(g, run["f1"]["E"], run["f1"]["B"], ref["cell"], ref["off"])
    ref["u"] = O.boris(ref["q"], ref["m"], g.dt, EB, ref["u"])
    ref["cell"], ref["off"], _, bad = O.move(g, ref["u"], ref["cell"], ref["off"])
    assert bad == 0
    assert np.array_equal(after["w"], ref["w"])
    t = TOL["fp32"]
    du = np.max(np.abs(after["u"] - ref["u"])) / np.max(np.abs(ref["u"]))
    n = np.array(g.n)[:, None]
    dx = (after["cell"] + after["off"] - ref["cell"] - ref["off"] + n / 2) % n - n / 2
    assert du <= t["u"], du
    assert np.max(np.abs(dx)) <= t["pos"], np.max(np.abs(dx))


def box_origins(g, tile=8, count=64, seed=301):
    """Origins of 4^3 boxes that straddle tile seams on every axis (from two
    cells below a seam to one above), the periodic seam among them (lo = n - 2
    on every axis for the first box), the rest at seeded seams."""
    r = inputs.rng(seed)
    out = [np.array([g.n[d] - 2 for d in range(3)])]
    while len(out) < count:
        out.append(np.array([(tile * int(r.integers(0, g.n[d] // tile)) - 2) % g.n[d] for d in range(3)]))
    return out


def test_current_in_sample_boxes(run):
    """J^{3/2} inside 64 boxes of 4^3 nodes, each straddling tile seams on all
    three axes (one the periodic seam), from every particle whose cell lies
    within three cells of a box (the Esirkepov window reaches at most that
    far): the merged per-tile current boxes must add up across the seams."""
    sim, g = run["sim"], run["g"]
    st = run["state1"]
    cells = torch.stack([torch.as_tensor(c, device="cuda") for c in
                         unpack_cells(st["cell"].cpu().numpy(), sim.bits)]).long()
    Jgpu = run["f2"]["J"]
    for b, lo in enumerate(box_origins(g)):
        sel = torch.ones(cells.shape[1], dtype=torch.bool, device="cuda")
        for d in range(3):
            rel = (cells[d] - int(lo[d]) + 3) % g.n[d]
            sel &= rel < 4 + 6
        idx = torch.nonzero(sel).squeeze(1).cpu().numpy()
        sp = host_species(sim, st, idx)
        J = np.zeros((3, g.ncells))
        EB = O.gather(g, run["f1"]["E"], run["f1"]["B"], sp["cell"], sp["off"])
        u = O.boris(sp["q"], sp["m"], g.dt, EB, sp["u"])
        c1, o1, dc, bad = O.move(g, u, sp["cell"], sp["off"])
        assert bad == 0
        O.deposit(g, sp["q"], sp["cell"], sp["off"], dc, o1, u, sp["w"], J)
        ii = [(lo[d] + np.arange(4)) % g.n[d] for d in range(3)]
        K, Jj, I = np.meshgrid(ii[2], ii[1], ii[0], indexing="ij")
        flat = (I + g.n[0] * (Jj + g.n[1] * K)).ravel()
        ref = J[:, flat]
        got = Jgpu[:, flat]
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        assert err <= TOL["fp32"]["J"], (b, err)


def test_fields_everywhere(run):
    """E^2, B^2 from E^1, B^1 and the GPU's J^{3/2} through the oracle's Yee update."""
    g = run["g"]
    f = {k: v.copy() for k, v in run["f1"].items()}
    f["J"] = run["f2"]["J"].copy()
    O.yee_step(g, f)
    for k in ("E", "B"):
        err = np.max(np.abs(run["f2"][k] - f[k])) / np.max(np.abs(f[k]))
        assert err <= TOL["fp32"][k], (k, err)


def test_conservation_at_full_size(run):
    d0, d1, d2 = run["d"]
    assert abs(d1["Q"] - d0["Q"]) <= 1e-12 * abs(d0["Q"])
    scale = d2["rho_max"]
    # FP32 positions: continuity holds to the FP32 rounding of the offsets
    assert d2["continuity"] <= 2e-6 * scale / run["g"].dt, (d2["continuity"], scale / run["g"].dt)
    assert d2["gauss_change"] <= 2e-5 * scale, (d2["gauss_change"], scale)
