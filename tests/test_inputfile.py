"""JSON input files (the paper's Sec. 3.2): every shipped file describes exactly
the workload the code path builds, its particles are the same seeded draws,
and malformed files are refused with a message."""
import copy
import json
import os

import numpy as np
import pytest

from paper_1503_02464_amd import configs, inputfile, inputs

RUNS = os.path.join(os.path.dirname(inputfile.__file__), "runs")

CASES = {
    "uniform_2d_64.json": configs.uniform_2d_small,
    "laser_foil_2d.json": configs.laser_foil_2d,
    "thermal_3d_256.json": configs.thermal_3d,
    "laser_foil_3d.json": configs.laser_foil_3d,
    "diff_2d_512.json": configs.diff_2d,
    "two_stream_3d.json": configs.two_stream_3d,
}


def doc(name):
    with open(os.path.join(RUNS, name)) as f:
        return json.load(f)


def test_every_run_file_is_covered():
    runs = [f for f in os.listdir(RUNS) if not f.endswith("_outputs.json")]
    assert sorted(runs) == sorted(CASES)


def test_output_requests_file_fits_its_run():
    """The example output requests (Sec. 3.1) of the 3D laser-foil run parse
    against that run's grid and species."""
    from paper_1503_02464_amd.outputs import parse_requests
    spec = inputfile.load(os.path.join(RUNS, "laser_foil_3d.json"))
    w = spec.workload()
    with open(os.path.join(RUNS, "laser_foil_3d_outputs.json")) as f:
        reqs = parse_requests(json.load(f), w.dims, w.n, 2)
    kinds = sorted({r.kind for r in reqs})
    assert kinds == ["density", "fields", "particles"]
    line = [r for r in reqs if r.name == "ey_axis_line"][0]
    assert line.points() == (512, 1, 1) and line.fires(400) and not line.fires(401) and not line.fires(502)


@pytest.mark.parametrize("name", sorted(CASES))
def test_file_is_the_configured_workload(name):
    spec = inputfile.load(os.path.join(RUNS, name))
    want = CASES[name]()
    got = spec.workload()
    assert got == want, (got, want)
    assert spec.dt == want.dt


def same_species(a, b):
    for k in ("cell", "off", "u", "w"):
        np.testing.assert_array_equal(a[k], b[k])
    assert a["q"] == b["q"] and a["m"] == b["m"]


def test_small_box_particles_are_the_seeded_draws():
    spec = inputfile.load(os.path.join(RUNS, "uniform_2d_64.json"))
    w = configs.uniform_2d_small()
    (got,) = spec.species()
    same_species(got, inputs.uniform_plasma(w.n, w.dims, w.ppc, w.u_sigma, w.weight, w.seed))


def test_laser_foil_particles_are_the_seeded_draws():
    spec = inputfile.load(os.path.join(RUNS, "laser_foil_2d.json"))
    e, i = spec.species()
    we, wi = configs.laser_foil_2d().species()
    same_species(e, we)
    same_species(i, wi)


def test_two_beams_are_the_seeded_draws():
    """The two-stream file scaled down (the full box holds 1.8 G particles):
    the beams are inputs.two_beams of the configured workload."""
    d = doc("two_stream_3d.json")
    d["grid"]["cells"] = [16, 16, 4]
    d["launch"]["tile"] = [8, 8, 4]
    spec = inputfile.parse(d)
    a, b = spec.species()
    w = configs.two_stream_3d(scale=32)
    wa, wb = inputs.two_beams(w.n, 3, w.ppc // 2, w.extra["u0"], w.u_sigma, w.weight, w.seed)
    same_species(a, wa)
    same_species(b, wb)


BAD = [
    (lambda d: d["grid"].update(dims=4), "dims"),
    (lambda d: d["grid"].update(cfl=1.0), "Yee limit"),
    (lambda d: d["launch"].update(tile=[7, 8, 8]), "does not divide"),
    (lambda d: d.update(precision="fp16"), "precision"),
    (lambda d: d.update(shape_order=3), "shape_order"),
    (lambda d: d.update(laser={"plane": 4, "a0": 1.0, "waist": 1.0, "duration_fwhm": 1.0}), "open x"),
    (lambda d: d["species"][0].update(profile={"kind": "sphere"}), "profile kind"),
    (lambda d: d["species"][0].pop("ppc"), "ppc"),
    (lambda d: d["species"][0].update(mass=0.0), "mass"),
    (lambda d: d.update(species=[]), "at least one species"),
]


@pytest.mark.parametrize("edit,msg", BAD, ids=[m for _, m in BAD])
def test_malformed_files_are_refused(edit, msg):
    d = copy.deepcopy(doc("thermal_3d_256.json"))
    edit(d)
    with pytest.raises(inputfile.InputError, match=msg):
        spec = inputfile.parse(d)
        spec.species() if d.get("species") else None


def test_slab_outside_the_box_is_refused():
    d = copy.deepcopy(doc("laser_foil_2d.json"))
    d["species"][0]["profile"]["x_cells"] = [2000, 2100]
    with pytest.raises(inputfile.InputError, match="x_cells"):
        inputfile.parse(d)
