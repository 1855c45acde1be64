"""The runner end to end on the GPU (paper Sec. 3.2: a run described by an
input file; Sec. 3.1: outputs in time windows): the 64x64 2D run file for 12
steps with diagnostics every 4 and three output requests, and every printed
line and written file checked against the run's own state."""
import json
import os

import numpy as np
import pytest

from paper_1503_02464_amd import run

pytestmark = pytest.mark.gpu

RUNS = os.path.join(os.path.dirname(run.__file__), "runs")


def test_runner_prints_diagnostics_and_writes_outputs(tmp_path, capsys):
    reqs = [{"name": "ey", "kind": "fields", "components": ["Ey", "Ex"], "box": {"lo": [0, 32], "hi": [64, 33]},
             "every": 4},
            {"name": "rho", "kind": "density", "box": {"lo": [0, 0], "hi": [64, 64], "stride": [2, 2]},
             "every": 6, "from": 6, "to": 12},
            {"name": "phase", "kind": "particles", "species": 0, "cells": {"lo": [0, 0], "hi": [32, 64]},
             "subsample": 3, "every": 12}]
    spec = tmp_path / "outputs.json"
    spec.write_text(json.dumps(reqs))
    out = tmp_path / "out"
    rc = run.main([os.path.join(RUNS, "uniform_2d_64.json"), "--steps", "12", "--diag-every", "4",
                   "--outputs", str(spec), "--out", str(out)])
    assert rc == 0
    lines = [json.loads(x) for x in capsys.readouterr().out.splitlines() if x.startswith("{")]
    head, diags = lines[0], lines[1:]
    assert head["particles"] == 64 * 64 * 4 and head["cells"] == 64 * 64
    assert [d["step"] for d in diags] == [4, 8, 12]
    for d in diags:
        assert np.isfinite([d["UE"], d["UB"], d["K"]]).all() and d["live"] == 64 * 64 * 4
        assert abs(d["Q"] + 64 * 64 * 4 * 0.05 ** 2 / 4) < 1e-9  # charge: -1 x weight (density dA / ppc) each
    # files at exactly the requested steps, with the requested shapes
    for name, steps, shape in (("ey", [4, 8, 12], (2, 1, 1, 64)), ("rho", [6, 12], (1, 1, 32, 32))):
        idx = [json.loads(x) for x in open(out / name / "index.jsonl")]
        assert sorted(x["step"] for x in idx) == steps
        for x in idx:
            a = np.load(out / name / x["file"])
            assert a.shape == shape and np.isfinite(a).all()
    (ph,) = [json.loads(x) for x in open(out / "phase" / "index.jsonl")]
    a = np.load(out / "phase" / ph["file"])
    assert ph["step"] == 12 and not ph["truncated"] and a.shape == (ph["count"], 6)
    assert 0.45 * 64 * 64 * 4 / 3 < ph["count"] < 0.55 * 64 * 64 * 4 / 3  # half the cells, every third particle
    assert (a[:, 0] >= 0).all() and (a[:, 0] < 32 * 0.05).all()  # x inside the cell box
    # the density of a neutral-free electron plasma: -1 per unit volume on average
    rho = [np.load(out / "rho" / x["file"]) for x in (json.loads(y) for y in open(out / "rho" / "index.jsonl"))]
    for r in rho:
        assert abs(r.mean() + 1.0) < 0.05
    desc = json.load(open(out / "outputs.json"))
    assert [d["name"] for d in desc["outputs"]] == ["ey", "rho", "phase"]
