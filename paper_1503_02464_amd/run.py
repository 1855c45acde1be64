"""Run a simulation described by a JSON input file (the paper's Sec. 3.2:
typical setups without code editing).

    python -m paper_1503_02464_amd.run FILE [--steps N] [--diag-every K]
                                           [--outputs SPEC.json] [--out DIR]

Builds the run with ``inputfile``, advances it with pic_step in chunks of
``--diag-every`` steps and prints one JSON line of FP64 diagnostics (U_E,
U_B, K, Q, live particles) after each chunk.  With ``--outputs`` (a JSON list
of output requests, see ``outputs``) it also writes the requested field
planes, lines, boxes and particle samples under ``--out``.
"""
from __future__ import annotations

import argparse
import json
import sys
import time


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("file")
    ap.add_argument("--steps", type=int, default=None, help="override the file's step count")
    ap.add_argument("--diag-every", type=int, default=50)
    ap.add_argument("--outputs", default=None, help="JSON list of output requests")
    ap.add_argument("--out", default="run_out")
    a = ap.parse_args(argv)

    import torch

    from . import inputfile
    if not torch.cuda.is_available():
        print("run: a GPU is required (the HIP library is the only implementation)", file=sys.stderr)
        return 2
    spec = inputfile.load(a.file)
    steps = spec.steps if a.steps is None else a.steps
    t0 = time.time()
    sim, handles = spec.simulation()
    for h in handles:
        sim.sort(h)
    manager = None
    if a.outputs:
        from .outputs import OutputManager
        with open(a.outputs) as f:
            manager = OutputManager(sim, json.load(f), a.out)
    print(json.dumps({"run": spec.name, "particles": sum(h.np for h in handles), "cells": sim.ncells,
                      "setup_s": round(time.time() - t0, 2)}), flush=True)
    done = 0
    every = max(1, a.diag_every)
    while done < steps:
        k = min(every, steps - done)
        if manager is not None:
            for _ in range(k):
                sim.step(1)
                manager.after_step(sim.step_count)
        else:
            sim.step(k)
        done += k
        d = sim.diagnostics()
        live = sum(int(sim.live(h).sum().item()) for h in handles) if spec.open_x else sum(h.np for h in handles)
        print(json.dumps({"step": sim.step_count, "UE": d["UE"], "UB": d["UB"], "K": d["K"], "Q": d["Q"],
                          "live": live}), flush=True)
    if manager is not None:
        manager.close()
    sim.check()
    sim.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
