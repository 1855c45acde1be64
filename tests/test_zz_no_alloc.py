"""The allocation-free diagnostics (pic_diagnostics_noalloc) against
pic_diagnostics, both called through the C ABI: two calls in a row, the
second on a smaller box with fewer particles, each compared with the
workspace path's first call on a fresh context."""
import ctypes
import math

import numpy as np
import pytest

from gpu_helpers import grid, make_sim, state
from paper_1503_02464_amd import _lib as L

pytestmark = pytest.mark.gpu


def _noalloc(sim, species):
    arr = (L.Species * max(len(species), 1))()
    for i, s in enumerate(species):
        arr[i] = s.struct
    out = (ctypes.c_double * L.PIC_NDIAG)()
    import torch
    st = sim.lib.pic_diagnostics_noalloc(sim.ctx, arr, len(species), ctypes.byref(sim.fstruct), out,
                                         ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    L.check(sim.lib, sim.ctx, st, "pic_diagnostics_noalloc")
    return list(out)


def _reference(g, prec, tile, sp, f):
    sim = make_sim(g, prec, tile, max_particles=sp["w"].shape[0])
    sim.set_fields(f["E"], f["B"])
    sim.add_species(sp)
    d = sim.diagnostics()
    sim.close()
    return [d[k] for k in ("UE", "UB", "K", "Q", "rho_max", "gauss_max", "gauss_change", "continuity")]


@pytest.mark.parametrize("prec,dims", [("fp64", 3), ("fp32", 2)])
def test_noalloc_matches_workspace_path(prec, dims):
    cases = [((24, 20, 16) if dims == 3 else (96, 80), 3), ((16, 12, 8) if dims == 3 else (40, 24), 1)]
    for n, ppc in cases:  # the second call is smaller: stale scratch must not leak into it
        g = grid(dims, n[:dims], dx=0.05, cfl=0.7, order=2)
        tile = (8, 4, 4) if dims == 3 else (8, 4, 1)
        sp, f = state(g, prec, ppc, 0.3, 0.05, seed=90 + len(n) + ppc)
        want = _reference(g, prec, tile, sp, f)
        sim = make_sim(g, prec, tile, max_particles=sp["w"].shape[0])
        sim.set_fields(f["E"], f["B"])
        h = sim.add_species(sp)
        got = _noalloc(sim, [h])
        sim.close()
        # fixed-order reductions: the energies and the charge are bit-identical
        assert got[:4] == want[:4], (got[:4], want[:4])
        # maxima of the charge grid, built with FP64 atomics: round-off
        for i in (4, 5):
            assert abs(got[i] - want[i]) <= 1e-12 * abs(want[i]), (i, got[i], want[i])
        assert math.isnan(got[6]) and math.isnan(got[7]) and math.isnan(want[6]) and math.isnan(want[7])


def test_noalloc_rejects_large_grid():
    # 256 x 256 x 128 nodes = 2^23 > PIC_NOALLOC_MAX_CELLS: refused on the host
    g = grid(3, (256, 256, 128), dx=0.05, cfl=0.7, order=1)
    sim = make_sim(g, "fp32", (8, 8, 8), max_particles=1)
    with pytest.raises(L.PicError, match="PIC_NOALLOC_MAX_CELLS"):
        _noalloc(sim, [])
    sim.close()
