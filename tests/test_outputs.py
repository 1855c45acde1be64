"""Host logic of the output manager (paper Sec. 3.1: outputs within a temporal
window at a chosen frequency, reduced-dimension and subdomain boxes): request
parsing, defaults, the firing schedule and the refusal of malformed
requests.  No GPU."""
import pytest

from paper_1503_02464_amd.outputs import OutputError, parse_requests

N3 = (64, 32, 16)


def one(r, dims=3, n=N3, nspecies=2):
    (req,) = parse_requests([r], dims, n, nspecies)
    return req


def test_window_and_frequency():
    r = one({"name": "a", "kind": "fields", "every": 5, "from": 10, "to": 30})
    assert [s for s in range(0, 50) if r.fires(s)] == [10, 15, 20, 25, 30]
    r = one({"name": "a", "kind": "fields", "every": 3})
    assert [s for s in range(0, 10) if r.fires(s)] == [0, 3, 6, 9]
    r = one({"name": "a", "kind": "fields", "from": 7, "to": 7})
    assert [s for s in range(20) if r.fires(s)] == [7]


def test_defaults_whole_grid_and_groups():
    r = one({"name": "all", "kind": "fields"})
    assert r.components == ["Ex", "Ey", "Ez", "Bx", "By", "Bz"]
    assert (r.lo, r.hi, r.stride) == ((0, 0, 0), N3, (1, 1, 1))
    assert r.points() == N3
    r = one({"name": "j", "kind": "fields", "components": ["J", "Ey"]})
    assert r.components == ["Jx", "Jy", "Jz", "Ey"]


def test_plane_line_and_strided_box_points():
    plane = one({"name": "p", "kind": "fields", "box": {"lo": [0, 0, 8], "hi": [64, 32, 9]}})
    assert plane.points() == (64, 32, 1)
    line = one({"name": "l", "kind": "fields", "box": {"lo": [0, 16, 8], "hi": [64, 17, 9], "stride": [2, 1, 1]}})
    assert line.points() == (32, 1, 1)
    sub = one({"name": "s", "kind": "fields", "box": {"lo": [3, 1, 0], "hi": [20, 32, 16], "stride": [4, 3, 5]}})
    assert sub.points() == (5, 11, 4)  # ceil(17/4), ceil(31/3), ceil(16/5)


def test_2d_boxes_take_two_axes():
    r = one({"name": "l", "kind": "fields", "box": {"lo": [0, 5], "hi": [64, 6]}}, dims=2, n=(64, 32, 1))
    assert (r.lo, r.hi, r.stride) == ((0, 5, 0), (64, 6, 1), (1, 1, 1))
    with pytest.raises(OutputError, match="2 entries"):
        one({"name": "l", "kind": "fields", "box": {"lo": [0, 5, 0], "hi": [64, 6, 1]}}, dims=2, n=(64, 32, 1))


def test_particles_and_density_requests():
    r = one({"name": "e", "kind": "particles", "species": 1, "cells": {"lo": [0, 0, 0], "hi": [8, 8, 8]},
             "subsample": 4, "every": 10})
    assert r.species == [1] and r.subsample == 4 and r.capacity is None and r.stride == (1, 1, 1)
    r = one({"name": "rho", "kind": "density"})
    assert r.species == [0, 1] and r.components == ["rho"]


BAD = [
    ({"kind": "fields"}, "name"),
    ({"name": "x/y", "kind": "fields"}, "name"),
    ({"name": "a", "kind": "movie"}, "kind"),
    ({"name": "a", "kind": "fields", "every": 0}, "every"),
    ({"name": "a", "kind": "fields", "from": 10, "to": 5}, "from"),
    ({"name": "a", "kind": "fields", "components": ["Ew"]}, "component"),
    ({"name": "a", "kind": "fields", "components": ["E", "B", "J", "E", "B", "J"]}, "16"),
    ({"name": "a", "kind": "fields", "box": {"lo": [0, 0, 0], "hi": [65, 32, 16]}}, "lo <= hi"),
    ({"name": "a", "kind": "fields", "box": {"lo": [5, 0, 0], "hi": [4, 32, 16]}}, "lo <= hi"),
    ({"name": "a", "kind": "fields", "box": {"stride": [0, 1, 1]}}, "stride"),
    ({"name": "a", "kind": "fields", "box": {"lo": [0.5, 0, 0]}}, "integers"),
    ({"name": "a", "kind": "particles"}, "species"),
    ({"name": "a", "kind": "particles", "species": 2}, "species"),
    ({"name": "a", "kind": "particles", "species": 0, "subsample": 0}, "subsample"),
    ({"name": "a", "kind": "particles", "species": 0, "capacity": 0}, "capacity"),
    ({"name": "a", "kind": "density", "species": [3]}, "species"),
]


@pytest.mark.parametrize("req,msg", BAD, ids=[m + str(i) for i, (_, m) in enumerate(BAD)])
def test_malformed_requests_are_refused(req, msg):
    with pytest.raises(OutputError, match=msg):
        parse_requests([req], 3, N3, 2)


def test_duplicate_names_are_refused():
    with pytest.raises(OutputError, match="duplicate"):
        parse_requests([{"name": "a", "kind": "fields"}, {"name": "a", "kind": "density"}], 3, N3, 1)
