"""Throughput of the PIC hot path on one MI355X.

Workload: the 3D3V periodic uniform thermal plasma, 256^3 cells, 8 electrons
per cell (134,217,728 particles), Maxwellian momenta with spread 0.05 m_e c,
quadratic shape, dx = 0.05 c/omega_p, dt = 0.7 of the Yee limit; synthetic,
seeded inputs resident in HBM before timing starts.

One step = the whole forward step: the tile sort (every 12th step, amortised),
clearing J, the fused gather + Boris + Esirkepov deposit per tile, and the Yee
update.  value = particle pushes per second over the timed steps.

Also printed, in the same JSON line:
* roofline: algorithmic bytes of the fused particle kernel per launch over its
  average launch time (HIP events on the launch stream, inside this run),
  against the 8 TB/s HBM peak; traffic = HBM bytes per launch from the
  FETCH_SIZE / WRITE_SIZE counters recorded under profiles/ (null once the
  kernel sources differ from the ones they were taken on); binding = the
  same record's SQ counters: the fractions of the kernel's cycles the LDS is
  busy and replaying conflicts, and VALU issue (the kernel is bound by LDS
  and VALU work, not by HBM); copy_GBs = what a plain 4 GiB device copy
  reaches on this GPU, the practical HBM roof beside the 8 TB/s peak;
* cpu_baseline: the FP64 CPU oracle on the host: one thread on a 64^3 box
  and every core (the oracle's all-core timing build) on a 128^3 box of the
  same workload, with the host's core count and CPU model;
* fp64: the same step in FP64 (value and roofline);
* adjoint: forward and backward time of the differentiable 2D rollout;
* laser_foil: time per step of the two laser-on-foil boxes (FP32), once the
  laser has reached the foil, and with the output manager writing a field
  plane, a density plane and an electron phase-space dump every 4 steps;
* two_stream: the paper's scaling workload at its full size (1.81 G particles).
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
LDS_CURRENT = "auto"  # accumulator of the fused kernel's on-chip current (FP32 state), set by --lds-current


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


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "traffic_push_deposit_thermal3d_256c_8ppc.json")


def measured_profile(w, prec: str):
    """The fused kernel's recorded counters (profiles/), if they were taken on
    this workload, precision and the current kernel sources; else None."""
    import hashlib
    if prec != "fp32" or w.n != (256, 256, 256):
        return None
    try:
        with open(TRAFFIC_PROFILE) as f:
            prof = json.load(f)
        h = hashlib.sha256()
        for rel in prof["sources"]:
            with open(os.path.join(ROOT, rel), "rb") as f:
                h.update(f.read())
    except (OSError, KeyError, ValueError):
        return None
    if h.hexdigest() != prof["sha256"]:
        log("fused kernel sources changed since the counters were taken: traffic = null")
        return None
    return prof


def measured_traffic(w, prec: str):
    """HBM bytes per launch of the fused kernel from the FETCH_SIZE and
    WRITE_SIZE counters (scaled by a plain copy of known size), or None."""
    prof = measured_profile(w, prec)
    return None if prof is None else int(prof["traffic_bytes_per_launch"])


def measured_binding(w, prec: str):
    """What binds the fused kernel, from its SQ counters (fractions of the
    kernel's busy cycles: LDS unit active per CU, LDS bank-conflict replays,
    VALU issue per SIMD), or None.  unit names the busiest of LDS and VALU
    (both when they are within 0.05 of each other): the kernel is limited by
    on-chip work (the current box's atomics, the gather's LDS reads and the
    per-particle arithmetic), not by HBM."""
    prof = measured_profile(w, prec)
    if prof is None or "lds_active_frac" not in prof:
        return None
    lds, valu = prof["lds_active_frac"], prof["valu_issue_frac"]
    unit = "LDS+VALU" if abs(lds - valu) < 0.05 else ("LDS" if lds > valu else "VALU")
    return {"unit": unit, "lds_active_frac": lds, "lds_bank_conflict_frac": prof["lds_bank_conflict_frac"],
            "valu_issue_frac": valu}


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
    from paper_1503_02464_amd.configs import BENCH_LAUNCH
    lc = BENCH_LAUNCH[prec]
    sim = Simulation(w.dims, w.n, w.dx, w.dt, w.order, prec, tile=lc["tile"], slack=lc["slack"],
                     sort_every=lc["sort_every"], max_particles=sp["w"].shape[0],
                     current_accum=LDS_CURRENT if prec == "fp32" else "auto")
    h = sim.add_species(sp)
    del sp
    # Set-up: the first sort bins the generator's cell-by-cell order into
    # tiles and levels; the second puts each level in node order, the order
    # every later sort keeps.  Timing starts from that steady state.
    sim.sort(h)
    sim.sort(h)
    torch.cuda.synchronize()
    log(f"{prec}: uploaded, workspace {sim._ws.numel() / 2**30:.2f} GiB, LDS/tile {sim.lib.pic_tile_lds_bytes(sim.ctx)} B")
    return sim, h


LASER_SORT_EVERY = 8  # the laser-driven electrons move faster than the thermal plasma


def sim_sort_every(prec: str) -> int:
    from paper_1503_02464_amd.configs import BENCH_LAUNCH
    return BENCH_LAUNCH[prec]["sort_every"]


def to_sort_step(sim, warmup: int) -> int:
    """Extra warmup steps so that the first timed step is one that sorts: a
    timed run of K steps then holds ceil(K / sort_every) sorts, never fewer
    than the amortised share (exactly that share when K is a multiple)."""
    every = sim.sort_every
    return (-(sim.step_count + warmup)) % every


def sorts_in(sim, steps: int) -> int:
    """Sorts the last `steps` steps made (the step counter sorts at multiples of sort_every)."""
    every, end = sim.sort_every, sim.step_count
    return sum(1 for k in range(end - steps, end) if k % every == 0)


def run_precision(w, prec: str, steps: int, warmup: int) -> dict:
    import torch

    sim, h = build_sim(w, prec)
    npart = h.np
    sim.step(warmup + to_sort_step(sim, warmup))
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
    sorts = sorts_in(sim, steps)
    sim.set_timing(True)
    sim.step(steps)
    tim = sim.get_timing()
    sim.set_timing(False)
    timed_sorts = sorts_in(sim, steps)  # the sort steps among the event-timed ones
    diag = sim.diagnostics()
    sim.close()
    push_ms, push_n = tim["push_deposit"]
    yee_ms, yee_n = tim["yee"]
    sort_ms, sort_n = tim["sort"]
    zero_ms, zero_n = tim["zero_current"]
    per_launch_bytes = npart * particle_bytes(prec, w.dims) + w.ncells * cell_bytes(prec)
    # In 3D a sort step's push also takes over the sort's copy: it reads each
    # particle's source index and writes its weight into the second set.
    folded = timed_sorts if w.dims == 3 else 0
    folded_bytes = per_launch_bytes + npart * (4 + (4 if prec == "fp32" else 8))
    timed_bytes = (push_n - folded) * per_launch_bytes + folded * folded_bytes
    push_avg_s = push_ms / max(push_n, 1) / 1e3
    achieved = timed_bytes / (push_ms / 1e3) / 1e9
    yee_avg_s = yee_ms / max(yee_n, 1) / 1e3
    return {
        "value": npart * steps / elapsed,
        "ms_per_step": elapsed / steps * 1e3,
        "particles": npart,
        "sort_every": sim_sort_every(prec),
        "sorts_in_timed_steps": sorts,
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
            "traffic": measured_traffic(w, prec),
            "bytes_per_launch": per_launch_bytes,
            "bytes_per_folded_launch": folded_bytes,
            "launches": {"in_place": push_n - folded, "folded": folded},
            "binding": measured_binding(w, prec),
        },
        "yee_cell_updates_per_s": w.ncells / yee_avg_s,
        "yee_achieved_GBs": w.ncells * yee_cell_bytes(prec) / yee_avg_s / 1e9,
        "diagnostics": {k: (None if v != v else v) for k, v in diag.items()},
    }


def adjoint_timing(prec: str = "fp32") -> dict:
    """The differentiable 2D3V rollout at its full size (512^2 cells, 16 ppc,
    linear shape, 200 steps, checkpoint every 20): forward and backward time
    of the second of two passes."""
    import numpy as np
    import torch

    from paper_1503_02464_amd import inputs
    from paper_1503_02464_amd.autograd import Rollout, rollout_loss
    from paper_1503_02464_amd.configs import diff_2d

    w = diff_2d()
    sp = inputs.uniform_plasma(w.n, 2, w.ppc, w.u_sigma, w.weight, w.seed)
    src = inputs.rng(w.seed + 1).normal(0, w.extra["src_sigma"], w.ncells)
    roll = Rollout(2, w.n, w.dx, w.dt, w.order, prec, sp, w.steps, w.extra["checkpoint_every"])
    # the second of two forward + backward passes is timed (the first warms the
    # allocator's pools and the library's first-call paths)
    for _ in range(2):
        s = torch.tensor(src, dtype=torch.float64, device="cuda", requires_grad=True)
        u0 = torch.tensor(sp["u"], dtype=torch.float64, device="cuda", requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L = rollout_loss(roll, s, u0)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        L.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
    npart = sp["w"].shape[0]
    roll.sim.close()
    log(f"adjoint rollout: forward {t1 - t0:.2f}s backward {t2 - t1:.2f}s")
    return {"workload": w.name, "particles": npart, "steps": w.steps, "checkpoint_every": w.extra["checkpoint_every"],
            "precision": prec, "forward_ms_per_step": (t1 - t0) / w.steps * 1e3,
            "backward_ms_per_step": (t2 - t1) / w.steps * 1e3,
            "backward_over_forward": (t2 - t1) / (t1 - t0), "loss": float(L.item()),
            "grad_norm_src": float(s.grad.norm().item()), "grad_norm_u0": float(u0.grad.norm().item())}


def pulse_at_foil_steps(w) -> int:
    """Steps until the laser's peak reaches the foil's front surface: the
    envelope peaks at t0 on the sheet, which is (foil_x0 - plane) dx from the
    foil, travelled at c = 1."""
    import math
    return int(math.ceil((w.t0 + (w.foil_x[0] - w.laser_plane) * w.dx[0]) / w.dt))


def laser_outputs(w, every: int) -> list:
    """A laser-foil run's output requests (paper Sec. 3.1): E_x, E_y and B_z on
    the plane through the laser axis (z = n_z / 2 in 3D, the whole grid in 2D),
    the electron charge density on the same plane, and the electrons' phase
    space in the foil's x range (every 32nd particle), each every `every` steps."""
    n = w.n
    plane = ({"lo": [0, 0, n[2] // 2], "hi": [n[0], n[1], n[2] // 2 + 1]} if w.dims == 3
             else {"lo": [0, 0], "hi": [n[0], n[1]]})
    foil = {"lo": [max(w.foil_x[0] - 8, 0)] + [0] * (w.dims - 1),
            "hi": [min(w.foil_x[1] + 40, n[0])] + list(n[1:w.dims])}
    return [{"name": "fields", "kind": "fields", "components": ["Ex", "Ey", "Bz"], "box": plane, "every": every},
            {"name": "rho_e", "kind": "density", "species": [0], "box": plane, "every": every},
            {"name": "electrons", "kind": "particles", "species": 0, "cells": foil, "subsample": 32, "every": every}]


def output_overhead(sim, w, steps: int, every: int) -> dict:
    """Time per step over `steps` steps, one pic_step call per step, without
    and then with the output manager writing laser_outputs(w, every) to a
    scratch directory (device extraction on the step's stream, copies on a
    side stream, writes on host threads)."""
    import shutil
    import tempfile

    import torch

    from paper_1503_02464_amd.outputs import OutputManager

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        sim.step(1)
    torch.cuda.synchronize()
    plain = time.perf_counter() - t0
    out = tempfile.mkdtemp(prefix="pic_outputs_")
    try:
        m = OutputManager(sim, laser_outputs(w, every), out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            sim.step(1)
            m.after_step()
        torch.cuda.synchronize()
        stepped = time.perf_counter() - t0
        m.flush()
        drained = time.perf_counter() - t0
        ext_ms, ext_n = m.extraction_ms()
        m.close()
        nbytes = sum(os.path.getsize(os.path.join(d, f)) for d, _, fs in os.walk(out) for f in fs)
        files = m.files
    finally:
        shutil.rmtree(out, ignore_errors=True)
    return {"every": every, "steps": steps, "files": files, "bytes_written": nbytes,
            "ms_per_step_without": plain / steps * 1e3, "ms_per_step_with": stepped / steps * 1e3,
            "overhead": stepped / plain - 1.0, "ms_until_written": drained * 1e3,
            "extraction_ms_per_output": ext_ms / max(ext_n, 1), "outputs": ext_n,
            "written_GBs": nbytes / drained / 1e9,
            "requests": [r["name"] for r in laser_outputs(w, every)]}


def laser_foil_timing(w, steps: int, warmup: int) -> dict:
    """A laser-on-foil box (open x faces, laser sheet, electrons + ions) in its
    launch configuration, FP32, timed over `steps` steps that start once the
    laser's peak has reached the foil (the run first steps there): time per
    whole step and pushes per second of the particles still live, with the
    live and straggler counts at the end."""
    import torch

    from paper_1503_02464_amd.sim import Simulation

    t0 = time.time()
    e, i = w.species()
    npart = e["w"].shape[0] + i["w"].shape[0]
    sim = Simulation(w.dims, w.n, w.dx, w.dt, w.order, "fp32", tile=w.tile, slack=1, sort_every=LASER_SORT_EVERY,
                     max_particles=e["w"].shape[0], open_x=True, absorb=w.absorb, sort_levels=w.sort_levels,
                     current_accum=LDS_CURRENT)
    sim.set_laser(**w.laser())
    hs = [sim.add_species(e), sim.add_species(i)]
    for h in hs:
        sim.sort(h)  # tiles and levels, then node order (as in build_sim)
        sim.sort(h)
    del e, i
    log(f"{w.name}: set up {npart} particles in {time.time() - t0:.1f}s")
    reach = pulse_at_foil_steps(w)
    t1 = time.time()
    sim.step(max(reach, warmup) + to_sort_step(sim, max(reach, warmup)))
    torch.cuda.synchronize()
    sim.check()
    log(f"{w.name}: stepped to {sim.step_count} (pulse peak at the foil after {reach}) in {time.time() - t1:.1f}s")
    live0 = sum(int(sim.live(h).sum().item()) for h in hs)
    t2 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t2
    sim.check()
    strays = sim.straggler_count()
    live1 = sum(int(sim.live(h).sum().item()) for h in hs)
    sorts = sorts_in(sim, steps)
    sim.set_timing(True)
    sim.step(steps)
    tim = sim.get_timing()
    sim.set_timing(False)
    diag = sim.diagnostics()
    outs = output_overhead(sim, w, steps, every=4)
    log(f"{w.name}: outputs every 4 steps: {outs['ms_per_step_without']:.3f} -> {outs['ms_per_step_with']:.3f} ms "
        f"per step ({outs['files']} files, {outs['bytes_written'] / 2**20:.1f} MiB)")
    sim.close()
    return {"workload": w.name, "particles": npart, "cells": w.ncells, "steps": steps,
            "timed_from_step": reach, "pulse_peak_at_foil_step": reach,
            "sort_every": LASER_SORT_EVERY, "sorts_in_timed_steps": sorts,
            "live_particles": {"start": live0, "end": live1, "removed_before": npart - live0},
            "stragglers_last_launch": strays,
            "ms_per_step": el / steps * 1e3, "pushes_per_s": 0.5 * (live0 + live1) * steps / el,
            "phases_ms_per_launch": {k: v[0] / max(v[1], 1) for k, v in tim.items()},
            "energy": {k: diag[k] for k in ("UE", "UB", "K")}, "outputs": outs}


def two_stream_timing(steps: int, warmup: int, scale: int = 1) -> dict:
    """The paper's scaling workload (Sec. 4) at its full size on one GPU: two
    counter-streaming electron beams, 512x512x128 cells, 27 particles per cell
    per beam (1.81 G particles, about 58 GB per particle set in FP32), drawn
    on the device; FP32, quadratic shape.  Time per step, pushes per second
    and the fused kernel's HBM fraction."""
    import torch

    from paper_1503_02464_amd import inputs
    from paper_1503_02464_amd.configs import two_stream_3d
    from paper_1503_02464_amd.sim import Simulation

    w = two_stream_3d(scale)
    ppb = w.ppc // 2
    npb = w.ncells * ppb
    # two particle sets per beam (32 B per particle each), the workspace (32 B per particle of one beam)
    need = 2 * 2 * npb * 32 + npb * 32 + 16 * w.ncells * 4
    free, total = torch.cuda.mem_get_info()
    if need > 0.95 * free:
        log(f"{w.name}: needs {need / 2**30:.0f} GiB, {free / 2**30:.0f} GiB free: skipped")
        return {"workload": w.name, "skipped": "not enough device memory"}
    t0 = time.time()
    sim = Simulation(3, w.n, w.dx, w.dt, w.order, "fp32", tile=w.tile, slack=1, sort_every=12, max_particles=npb,
                     sort_levels=w.extra["sort_levels"], current_accum=LDS_CURRENT)
    hs = []
    for b, sign in enumerate((1.0, -1.0)):
        h = sim.new_species(-1.0, 1.0, npb)
        inputs.uniform_plasma_device(h.sets[0], w.n, 3, sim.bits, ppb, (sign * w.extra["u0"], 0.0, 0.0), w.u_sigma,
                                     w.weight, w.seed + b)
        hs.append(h)
    torch.cuda.synchronize()
    for h in hs:
        sim.sort(h)
        sim.sort(h)
    torch.cuda.synchronize()
    log(f"{w.name}: {2 * npb} particles drawn and sorted in {time.time() - t0:.1f}s, "
        f"{torch.cuda.memory_allocated() / 2**30:.0f} GiB allocated")
    sim.step(warmup + to_sort_step(sim, warmup))
    torch.cuda.synchronize()
    sim.check()
    t1 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    sim.check()
    sorts = sorts_in(sim, steps)
    sim.set_timing(True)
    sim.step(steps)
    tim = sim.get_timing()
    sim.set_timing(False)
    timed_sorts = sorts_in(sim, steps)
    strays = sim.straggler_count()
    diag = sim.diagnostics()
    sim.close()
    push_ms, push_n = tim["push_deposit"]
    per_launch = npb * particle_bytes("fp32", 3) + w.ncells * cell_bytes("fp32")
    folded = 2 * timed_sorts
    timed_bytes = (push_n - folded) * per_launch + folded * (per_launch + npb * 8)
    achieved = timed_bytes / (push_ms / 1e3) / 1e9
    log(f"{w.name}: {el / steps * 1e3:.1f} ms per step")
    return {"workload": w.name, "particles": 2 * npb, "cells": w.ncells, "steps": steps,
            "sort_every": 12, "sorts_in_timed_steps": sorts, "ms_per_step": el / steps * 1e3,
            "pushes_per_s": 2 * npb * steps / el,
            "phases_ms_per_launch": {k: v[0] / max(v[1], 1) for k, v in tim.items()},
            "push_deposit_roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                                      "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                                      "bytes_per_launch": per_launch},
            "stragglers_last_launch": strays, "energy": {k: diag[k] for k in ("UE", "UB", "K")},
            "data": "drawn on the device (torch's seeded generator)"}


def copy_probe(nbytes: int = 1 << 30) -> None:
    """One plain device-to-device copy of nbytes (twice), to calibrate the
    FETCH_SIZE / WRITE_SIZE counters against a kernel of known traffic."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"copy probe: {nbytes} bytes read and written per copy")


def copy_bandwidth(nbytes: int = 4 << 30, reps: int = 10) -> float:
    """HBM bandwidth a plain device-to-device copy reaches on this GPU (bytes
    read + written per second, GB/s): the practical roof beside the 8 TB/s
    of the specification."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        b.copy_(a)
    t1.record()
    torch.cuda.synchronize()
    gbs = 2 * nbytes * reps / (t0.elapsed_time(t1) / 1e3) / 1e9
    del a, b
    log(f"copy bandwidth: {gbs:.0f} GB/s")
    return gbs


def host_facts() -> dict:
    """The host's cores (this process's CPU affinity), the thread count the
    all-core leg uses (OMP_NUM_THREADS when set, at most the affinity) and
    the CPU model."""
    aff = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS", "")
    threads = min(aff, int(env)) if env.isdigit() and int(env) > 0 else aff
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cores_in_affinity": aff, "omp_num_threads": env or None, "threads_used": threads, "cpu_model": model}


def cpu_baseline(w) -> dict:
    """The FP64 CPU oracle on the host cores, two legs, each whole steps of a
    scaled box of the same workload (same dx, dt, shape, momentum spread):
    one thread on a 64^3 box (about 10 s), then every core of the all-core
    timing build (particles in per-thread chunks, Yee serial) on a 128^3 box
    (about 10 s).  value = the all-core leg."""
    import oracle as O
    from paper_1503_02464_amd import inputs
    from paper_1503_02464_amd.configs import thermal_3d

    host = host_facts()

    def leg(scale: int, threads: int, budget_s: float) -> dict:
        ws = thermal_3d(scale=scale)
        g = O.Grid(3, ws.n, ws.dx, ws.dt, ws.order)
        sp = inputs.uniform_plasma(ws.n, 3, ws.ppc, ws.u_sigma, ws.weight, ws.seed)
        f = O.new_fields(g)
        steps, el = 0, 0.0
        t0 = time.perf_counter()
        while steps < 4 and el < budget_s:
            if threads == 1:
                O.step(g, f, [sp])
            else:
                O.step_threads(g, f, [sp], threads)
            steps += 1
            el = time.perf_counter() - t0
        npart = sp["w"].shape[0]
        return {"value": npart * steps / el, "threads": threads,
                "sample": f"{steps} FP64 steps of {ws.n[0]}^3 cells x {ws.ppc} ppc ({npart} particles); {el:.1f} s"}

    one = leg(4, 1, 10.0)
    log(f"cpu baseline, 1 thread: {one['value']:.3e} pushes/s ({one['sample']})")
    allc = leg(2, host["threads_used"], 8.0)
    log(f"cpu baseline, {allc['threads']} threads: {allc['value']:.3e} pushes/s ({allc['sample']})")
    return {"value": allc["value"], "unit": "particle pushes/s", "cores": allc["threads"], "kind": "oracle",
            "sample": allc["sample"] + "; the all-core timing build of the oracle (same arithmetic, particle chunks "
                                       "per thread, Yee serial)",
            "single_thread": {"value": one["value"], "cores": 1, "sample": one["sample"]},
            "host": host}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=24)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--scale", type=int, default=1, help="divide the 256^3 box by this per dimension (testing)")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--copy-probe", action="store_true", help="also run a 1 GiB device copy (counter calibration)")
    ap.add_argument("--no-laser", action="store_true", help="skip the two laser-on-foil boxes")
    ap.add_argument("--no-two-stream", action="store_true", help="skip the two-stream box (1.81 G particles)")
    ap.add_argument("--lds-current", default="auto", choices=["auto", "fix64", "fp64", "fp32"],
                    help="accumulator of the fused kernel's on-chip current for the FP32 state")
    args = ap.parse_args()
    global LDS_CURRENT
    LDS_CURRENT = args.lds_current
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU spatial decomposition "
              "is not implemented", file=sys.stderr)
        return 2
    import torch

    from paper_1503_02464_amd.configs import BENCH_LAUNCH, thermal_3d

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    w = thermal_3d(scale=args.scale)
    copy_gbs = copy_bandwidth()
    res32 = run_precision(w, "fp32", args.steps, args.warmup)
    res64 = None if args.no_fp64 else run_precision(w, "fp64", args.steps, args.warmup)
    adj = None if (args.no_adjoint or args.scale != 1) else adjoint_timing("fp32")
    laser = None
    if not args.no_laser and args.scale == 1:
        from paper_1503_02464_amd.configs import laser_foil_2d, laser_foil_3d
        laser = [laser_foil_timing(wl, args.steps, args.warmup) for wl in (laser_foil_2d(), laser_foil_3d())]
    two = None
    if not args.no_two_stream and args.scale == 1:
        two = two_stream_timing(args.steps, args.warmup)
    if args.copy_probe:
        copy_probe()
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
                   **{k: (list(v) if isinstance(v, tuple) else v) for k, v in BENCH_LAUNCH["fp32"].items()},
                   "positions": "int32 cell + f32 offset",
                   "lds_current": "fixed point, 64-bit" if args.lds_current in ("auto", "fix64") else args.lds_current},
        "roofline": dict(res32["roofline"], copy_GBs=round(copy_gbs, 1),
                         frac_of_copy=round(res32["roofline"]["achieved"] / copy_gbs, 4)),
        "cpu_baseline": base,
        "phases_ms_per_launch": res32["phases_ms_per_launch"],
        "sorts_in_timed_steps": res32["sorts_in_timed_steps"],
        "yee_cell_updates_per_s": res32["yee_cell_updates_per_s"],
        "yee_achieved_GBs": res32["yee_achieved_GBs"],
        "fp64": None if res64 is None else {k: res64[k] for k in ("value", "ms_per_step", "roofline",
                                                                  "phases_ms_per_launch", "sort_every",
                                                                  "sorts_in_timed_steps", "yee_cell_updates_per_s")},
        "adjoint": adj,
        "laser_foil": laser,
        "two_stream": two,
        # error bounds against the FP64 CPU oracle that the GPU parity tests
        # enforce on this path (one step from an FP32-representable state for
        # FP32; every quantity for FP64), including at this workload's full size
        "error_vs_oracle": {
            "fp32": {"position_cells_abs": 4e-7, "u_rel": 2e-6, "E_rel": 2e-6, "B_rel": 2e-6, "J_rel": 1e-5},
            "fp64_rel": 1e-12,
            "enforced_by": ["tests/test_gpu_parity.py", "tests/test_gpu_fullsize.py"],
        },
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
