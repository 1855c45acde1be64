"""Throughput of the PIC hot path on one MI355X.

Workload: the 3D3V periodic uniform thermal plasma, 256^3 cells, 8 electrons
per cell (134,217,728 particles), Maxwellian momenta with spread 0.05 m_e c,
quadratic shape, dx = 0.05 c/omega_p, dt = 0.7 of the Yee limit; synthetic,
seeded inputs resident in HBM before timing starts.

One step = the whole forward step: the tile sort (every 4th step, amortised),
clearing J, the fused gather + Boris + Esirkepov deposit per tile, and the Yee
update.  value = particle pushes per second over the timed steps.

Also printed, in the same JSON line:
* roofline: algorithmic bytes of the fused particle kernel per launch over its
  average launch time (HIP events on the launch stream, inside this run),
  against the 8 TB/s HBM peak;
* cpu_baseline: the FP64 CPU oracle, one thread, one step of a 64^3 box of
  the same workload;
* fp64: the same step in FP64 (value and roofline).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
SORT_EVERY = 4
# cells per tile and guard slack of the fused kernel, per precision (the FP64
# tile is halved in z so fields + current fit the 160 KB of LDS)
TILE = {"fp32": ((8, 8, 8), 1), "fp64": ((8, 8, 4), 1)}


def particle_bytes(prec: str, dims: int) -> int:
    """Algorithmic HBM bytes per particle-step of the fused kernel: read cell,
    offsets, momenta, weight; write cell, offsets, momenta."""
    e = 4 if prec == "fp32" else 8
    return (4 + dims * e + 3 * e + e) + (4 + dims * e + 3 * e)


def cell_bytes(prec: str) -> int:
    """Algorithmic HBM bytes per cell of the fused kernel: read E and B once,
    read-modify-write J once."""
    e = 4 if prec == "fp32" else 8
    return 6 * e + 3 * 2 * e


def yee_cell_bytes(prec: str) -> int:
    """Algorithmic bytes per cell of one Yee step: read E, B, J; write E, B."""
    e = 4 if prec == "fp32" else 8
    return 15 * e


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def build_sim(w, prec: str, scale_note: str = ""):
    import numpy as np
    import torch

    from paper_1503_02464_amd import inputs
    from paper_1503_02464_amd.sim import Simulation

    t0 = time.time()
    sp = inputs.uniform_plasma(w.n, w.dims, w.ppc, w.u_sigma, w.weight, w.seed)
    log(f"generated {sp['w'].shape[0]} particles in {time.time() - t0:.1f}s {scale_note}")
    tile, slack = TILE[prec]
    sim = Simulation(w.dims, w.n, w.dx, w.dt, w.order, prec, tile=tile, slack=slack, sort_every=SORT_EVERY,
                     max_particles=sp["w"].shape[0])
    h = sim.add_species(sp)
    del sp
    torch.cuda.synchronize()
    log(f"{prec}: uploaded, workspace {sim._ws.numel() / 2**30:.2f} GiB, LDS/tile {sim.lib.pic_tile_lds_bytes(sim.ctx)} B")
    return sim, h


def run_precision(w, prec: str, steps: int, warmup: int) -> dict:
    import torch

    sim, h = build_sim(w, prec)
    npart = h.np
    sim.step(warmup)
    torch.cuda.synchronize()
    sim.check()
    log(f"{prec}: warmup {warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sim.check()
    elapsed = t1 - t0
    log(f"{prec}: timed {steps} steps in {elapsed * 1e3:.1f} ms")
    # per-kernel durations with HIP events on the launch stream
    sim.set_timing(True)
    sim.step(steps)
    tim = sim.get_timing()
    sim.set_timing(False)
    diag = sim.diagnostics()
    sim.close()
    push_ms, push_n = tim["push_deposit"]
    yee_ms, yee_n = tim["yee"]
    sort_ms, sort_n = tim["sort"]
    zero_ms, zero_n = tim["zero_current"]
    per_launch_bytes = npart * particle_bytes(prec, w.dims) + w.ncells * cell_bytes(prec)
    push_avg_s = push_ms / max(push_n, 1) / 1e3
    achieved = per_launch_bytes / push_avg_s / 1e9
    yee_avg_s = yee_ms / max(yee_n, 1) / 1e3
    return {
        "value": npart * steps / elapsed,
        "ms_per_step": elapsed / steps * 1e3,
        "particles": npart,
        "phases_ms_per_launch": {
            "sort": sort_ms / max(sort_n, 1), "zero_current": zero_ms / max(zero_n, 1),
            "push_deposit": push_ms / max(push_n, 1), "yee_step": yee_ms / max(yee_n, 1),
        },
        "roofline": {
            "kernel": "push_deposit_tiled",
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None,
            "bytes_per_launch": per_launch_bytes,
        },
        "yee_cell_updates_per_s": w.ncells / yee_avg_s,
        "yee_achieved_GBs": w.ncells * yee_cell_bytes(prec) / yee_avg_s / 1e9,
        "diagnostics": {k: (None if v != v else v) for k, v in diag.items()},
    }


def cpu_baseline(w) -> dict:
    """The FP64 oracle, one thread, one step of a 64^3 box of the same workload."""
    import oracle as O
    from paper_1503_02464_amd import inputs
    from paper_1503_02464_amd.configs import c3_thermal_3d

    ws = c3_thermal_3d(scale=4)
    g = O.Grid(3, ws.n, ws.dx, ws.dt, ws.order)
    sp = inputs.uniform_plasma(ws.n, 3, ws.ppc, ws.u_sigma, ws.weight, ws.seed)
    f = O.new_fields(g)
    t0 = time.perf_counter()
    O.step(g, f, [sp])
    el = time.perf_counter() - t0
    npart = sp["w"].shape[0]
    return {"value": npart / el, "unit": "particle pushes/s", "cores": 1, "kind": "oracle",
            "sample": f"one FP64 step of {ws.n[0]}^3 cells x {ws.ppc} ppc ({npart} particles), same dx, dt, "
                      f"shape and momentum spread; {el:.1f} s"}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--scale", type=int, default=1, help="divide the 256^3 box by this per dimension (testing)")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU spatial decomposition "
              "is not part of this build", file=sys.stderr)
        return 2
    import torch

    from paper_1503_02464_amd.configs import c3_thermal_3d

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    w = c3_thermal_3d(scale=args.scale)
    res32 = run_precision(w, "fp32", args.steps, args.warmup)
    res64 = None if args.no_fp64 else run_precision(w, "fp64", args.steps, args.warmup)
    base = None if args.no_cpu_baseline else cpu_baseline(w)
    line = {
        "metric": "particle pushes/s (gather+Boris+deposit), FP32 vs FP64 at stated error; HBM %",
        "value": res32["value"],
        "unit": "particle pushes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "cells": list(w.n), "particles": res32["particles"], "ppc": w.ppc,
                   "shape_order": w.order, "dx": w.dx[0], "dt": w.dt, "u_sigma": w.u_sigma,
                   "tile": list(TILE["fp32"][0]), "slack": TILE["fp32"][1], "sort_every": SORT_EVERY,
                   "positions": "int32 cell + f32 offset"},
        "roofline": res32["roofline"],
        "cpu_baseline": base,
        "phases_ms_per_launch": res32["phases_ms_per_launch"],
        "yee_cell_updates_per_s": res32["yee_cell_updates_per_s"],
        "yee_achieved_GBs": res32["yee_achieved_GBs"],
        "fp64": None if res64 is None else {k: res64[k] for k in ("value", "ms_per_step", "roofline",
                                                                  "phases_ms_per_launch",
                                                                  "yee_cell_updates_per_s")},
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
