"""The tiled reverse step (pic_particle_adjoint given the particles' tile
ranges) against the per-particle HBM reverse step on identical inputs, with
many particles drifted beyond their tile's slack (they take the HBM path
inside the tiled call too).  The HBM path is itself held to the independent
torch FP64 reference gradient by the rollout tests.  FP64: 1e-12
norm-relative on lam_E, lam_B, lam_x, lam_u; FP32: 1e-5 (summation order of
the lam_E, lam_B atomics)."""
import ctypes

import numpy as np
import pytest
import torch

from gpu_helpers import grid, make_sim, unique_weights
from paper_1503_02464_amd import _lib as L
from paper_1503_02464_amd import inputs
from paper_1503_02464_amd.autograd import _fields_struct, _species_struct
from paper_1503_02464_amd.sim import _ptr, _stream

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float((a - b).abs().max() / b.abs().max().clamp_min(1e-300))


@pytest.mark.parametrize("prec,dims,order", [("fp64", 2, 1), ("fp64", 2, 2), ("fp64", 3, 1), ("fp32", 2, 1)])
def test_tiled_reverse_step_matches_hbm_path(prec, dims, order):
    g = grid(dims, (32, 24) if dims == 2 else (16, 16, 8), dx=0.05, cfl=0.7, order=order)
    tile = (16, 8, 1) if dims == 2 else (8, 8, 4)
    sp = inputs.uniform_plasma(g.n, dims, 3, 0.05, 1.0, 700 + dims + order, u_mean=(1.5, -1.0, 0.5))
    sp = unique_weights(sp, 701, scale=float(np.prod(g.dx[:dims])) / 3)
    f = inputs.random_fields(g.ncells, 0.1, 702)
    if prec == "fp32":
        sp, f = inputs.round_f32(sp), inputs.round_fields_f32(f)
    s = make_sim(g, prec, tile, slack=1, sort_every=0, max_particles=sp["w"].shape[0])
    s.set_fields(f["E"], f["B"])
    h = s.add_species(sp)
    s.sort(h)
    s.step(6)  # no re-sort: particles drift up to ~2 cells from their sorted tiles
    s.check()
    cur = h.current()
    n = h.np
    st = ctypes.c_void_p(_stream())
    dev, dt = s.device, s.dtype
    r = torch.Generator(device="cpu").manual_seed(703)
    lam_in = {k: [torch.randn(s.ncells, generator=r, dtype=torch.float64).to(dev, dt) for _ in range(3)]
              for k in ("E", "B", "J")}
    lx_in = [torch.randn(n, generator=r, dtype=torch.float64).to(dev, dt) for _ in range(3)]
    lu_in = [torch.randn(n, generator=r, dtype=torch.float64).to(dev, dt) for _ in range(3)]
    out = []
    for tiled in (True, False):
        lam = {k: [t.clone() for t in v] for k, v in lam_in.items()}
        lx = [t.clone() for t in lx_in]
        lu = [t.clone() for t in lu_in]
        spn = _species_struct(sp["q"], sp["m"], n, cur["cell"], cur["off"], cur["u"], cur["w"])
        if tiled:
            spn.tile_start = h.struct.tile_start
        fn = _fields_struct(s.fields["E"], s.fields["B"], s.fields["J"])
        lf = _fields_struct(lam["E"], lam["B"], lam["J"])
        lsp = L.SpeciesAdjoint()
        lsp.x = L._c3p(*[_ptr(t) for t in lx])
        lsp.u = L._c3p(*[_ptr(t) for t in lu])
        s._call(s.lib.pic_particle_adjoint(s.ctx, ctypes.byref(spn), ctypes.byref(fn), ctypes.byref(lf),
                                           ctypes.byref(lsp), st), "pic_particle_adjoint")
        if tiled:
            stragglers = s.straggler_count()  # the tiled call lists its stragglers in the same counter
        torch.cuda.synchronize()
        out.append((lam, lx, lu))
    s.check()
    assert stragglers > n // 20, (stragglers, n)
    tol = 1e-12 if prec == "fp64" else 1e-5
    (la, xa, ua), (lb, xb, ub) = out
    for k in ("E", "B"):
        for d in range(3):
            assert rel(la[k][d], lb[k][d]) <= tol, (k, d, rel(la[k][d], lb[k][d]))
    for d in range(3):
        if d < dims:
            assert rel(xa[d], xb[d]) <= tol, ("x", d)
        assert rel(ua[d], ub[d]) <= tol, ("u", d)
    s.close()
