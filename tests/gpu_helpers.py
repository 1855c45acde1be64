"""Shared helpers of the GPU parity tests: build the same seeded state for the
HIP library and for the oracle, run both, and compare.

Particles are matched by weight: every test state gives each particle a
distinct weight (exactly representable in FP32), so sorting both sides by
weight lines them up whatever order the GPU sort left them in."""
from __future__ import annotations

import math

import numpy as np

import oracle as O
from paper_1503_02464_amd import inputs

# Tolerances.  FP64: 1e-12 norm-relative (positions:
# absolute, in cells).  FP32 (one step from an FP32-representable state
# against the FP64 oracle): a few units of FP32 rounding (2^-24 ~ 6e-8) times
# the operation depth of each quantity.
TOL = {
    "fp64": {"pos": 1e-12, "u": 1e-12, "E": 1e-12, "B": 1e-12, "J": 1e-12},
    "fp32": {"pos": 4e-7, "u": 2e-6, "E": 2e-6, "B": 2e-6, "J": 1e-5},
}


def grid(dims, n, dx=0.05, cfl=0.7, order=2):
    n3 = tuple(n) + (1,) * (3 - len(n))
    dxs = tuple(dx for _ in range(dims)) + (1.0,) * (3 - dims) if not isinstance(dx, tuple) else dx
    dt = cfl / math.sqrt(sum(1.0 / dxs[d] ** 2 for d in range(dims)))
    return O.Grid(dims, n3, dxs, dt, order)


def unique_weights(sp: dict, seed: int, scale: float = 1.0) -> dict:
    """Distinct weights in scale * [0.5, 1.5), FP32-exact, in random order
    (scale is rounded to a power of two so the values stay FP32-exact)."""
    npart = sp["w"].shape[0]
    assert npart < (1 << 22)
    perm = inputs.rng(seed).permutation(npart)
    s2 = 2.0 ** round(math.log2(scale))
    w = s2 * (0.5 + (perm.astype(np.float64) / (1 << 22)))
    out = dict(sp)
    out["w"] = np.ascontiguousarray(w)
    return out


def by_weight(sp: dict) -> dict:
    order = np.argsort(sp["w"], kind="stable")
    out = dict(sp)
    for k in ("cell", "off", "u"):
        out[k] = sp[k][:, order]
    out["w"] = sp["w"][order]
    return out


def rel(a, b) -> float:
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = max(float(np.max(np.abs(b))), 1e-300)
    return float(np.max(np.abs(a - b))) / den if a.size else 0.0


def pos_err(g: O.Grid, a: dict, b: dict) -> float:
    """Largest absolute position difference in cells, across the periodic seam."""
    err = 0.0
    for d in range(g.dims):
        xa = a["cell"][d] + a["off"][d]
        xb = b["cell"][d] + b["off"][d]
        diff = (xa - xb + g.n[d] / 2) % g.n[d] - g.n[d] / 2
        err = max(err, float(np.max(np.abs(diff))) if diff.size else 0.0)
    return err


def make_sim(g: O.Grid, prec: str, tile, slack=1, sort_every=4, max_particles=0):
    from paper_1503_02464_amd.sim import Simulation
    return Simulation(g.dims, g.n, g.dx, g.dt, g.order, prec, tile=tile, slack=slack, sort_every=sort_every,
                      max_particles=max_particles)


def state(g: O.Grid, prec: str, npart_or_ppc, sigma, field_scale, seed, random_positions=False, q=-1.0, m=1.0):
    """Seeded species (unique weights) and fields, snapped to FP32 values for the FP32 path."""
    if random_positions:
        sp = inputs.random_particles(g.n, g.dims, npart_or_ppc, sigma, (1, 1), seed, q=q, m=m)
    else:
        sp = inputs.uniform_plasma(g.n, g.dims, npart_or_ppc, sigma, 1.0, seed, q=q, m=m)
        sp = inputs.shuffle(sp, seed + 1)
    dV = float(np.prod([g.dx[d] for d in range(g.dims)]))
    ppc = sp["w"].shape[0] / g.ncells
    sp = unique_weights(sp, seed + 2, scale=dV / max(ppc, 1e-9))
    f = inputs.random_fields(g.ncells, field_scale, seed + 3)
    if prec == "fp32":
        sp = inputs.round_f32(sp)
        f = inputs.round_fields_f32(f)
    return sp, f


def compare_species(g, prec, gpu_sp, ora_sp, what=""):
    t = TOL[prec]
    a, b = by_weight(gpu_sp), by_weight(ora_sp)
    assert np.array_equal(a["w"], b["w"]), f"{what}: particle sets differ"
    pe = pos_err(g, a, b)
    ue = rel(a["u"], b["u"])
    assert pe <= t["pos"], f"{what}: position error {pe:.3e} cells > {t['pos']}"
    assert ue <= t["u"], f"{what}: momentum error {ue:.3e} > {t['u']}"
    return pe, ue


def compare_fields(prec, gpu_f, ora_f, keys=("E", "B", "J"), what=""):
    t = TOL[prec]
    errs = {}
    for k in keys:
        e = rel(gpu_f[k], ora_f[k])
        errs[k] = e
        assert e <= t[k], f"{what}: {k} error {e:.3e} > {t[k]}"
    return errs
