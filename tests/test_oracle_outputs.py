"""Pins of the oracle's output definitions (paper Sec. 3.1: reduced-dimension
and subdomain outputs; Sec. 3.3: a particle's seven phase-space values),
against hand-counted cases and closed forms, so that a swapped axis, a wrong
stride or an off-by-one bound fails."""
import numpy as np
import pytest

import oracle as O


def test_box_hand_counted():
    """n = (4, 3, 2); grid value = flat index i + 4 (j + 3 k).  Box x 1..3 step 2,
    y 0..2 step 2, z 1: points (1,0,1) (3,0,1) (1,2,1) (3,2,1) -> 13 15 21 23."""
    g = O.Grid(3, (4, 3, 2), (1.0, 1.0, 1.0), 0.1, 1)
    F = np.arange(24, dtype=np.float64)
    got = O.extract_box(g, [F], (1, 0, 1), (4, 3, 2), (2, 2, 1))
    assert got.shape == (1, 1, 2, 2)
    np.testing.assert_array_equal(got[0, 0], [[13, 15], [21, 23]])


def test_box_two_grids_keep_their_order():
    g = O.Grid(3, (4, 3, 2), (1.0, 1.0, 1.0), 0.1, 1)
    F = np.arange(24, dtype=np.float64)
    got = O.extract_box(g, [F, -F], (0, 1, 0), (1, 2, 2), (1, 1, 1))  # a z line at x=0, y=1
    np.testing.assert_array_equal(got.reshape(2, 2), [[4, 16], [-4, -16]])


@pytest.mark.parametrize("n,lo,hi,st", [((8, 6, 5), (1, 2, 0), (8, 6, 5), (3, 1, 2)),
                                        ((16, 8, 1), (0, 3, 0), (16, 4, 1), (1, 1, 1)),
                                        ((7, 5, 3), (6, 0, 2), (7, 5, 3), (1, 4, 5)),
                                        ((5, 5, 5), (2, 2, 2), (2, 5, 5), (1, 1, 1))])
def test_box_closed_form(n, lo, hi, st):
    """With value = flat index, entry [c, b, a] = x_a + n0 y_b + n0 n1 z_c with
    x_a = lo0 + a st0 and so on: an outer sum, and the point counts are
    ceil((hi - lo) / st)."""
    g = O.Grid(3 if n[2] > 1 else 2, n, (1.0, 1.0, 1.0), 0.1, 1)
    F = np.arange(n[0] * n[1] * n[2], dtype=np.int64)
    got = O.extract_box(g, [F], lo, hi, st)[0]
    m = [max(0, -(-(hi[d] - lo[d]) // st[d])) for d in range(3)]
    assert got.shape == (m[2], m[1], m[0])
    x = lo[0] + st[0] * np.arange(m[0])
    y = lo[1] + st[1] * np.arange(m[1])
    z = lo[2] + st[2] * np.arange(m[2])
    want = z[:, None, None] * n[0] * n[1] + y[None, :, None] * n[0] + x[None, None, :]
    np.testing.assert_array_equal(got, want)


def particles():
    # five particles in a 3D box of 8 x 4 x 4 cells, dx = (0.5, 0.25, 2.0)
    return {"q": -1.0, "m": 1.0,
            "cell": np.array([[3, 7, 3, 0, 5], [1, 2, 3, 0, 1], [0, 3, 2, 1, 0]], np.int32),
            "off": np.array([[0.25, 0.5, 0.75, 0.0, 0.5], [0.5, 0.0, 0.25, 0.5, 0.5], [0.0, 0.5, 0.5, 0.25, 0.75]]),
            "u": np.array([[1.0, 2.0, 3.0, 4.0, 5.0], [-1.0, -2.0, -3.0, -4.0, -5.0], [0.5, 0.25, 0.125, 0.0, 1.5]]),
            "w": np.array([1.0, 2.0, 0.0, 4.0, 5.0])}


def test_phase_space_hand_counted():
    """Cells x in [2, 8), y in [1, 4), z in [0, 4): particles 0, 1, 2, 4 (3 has x = 0).
    Particle 0: x = 3.25 * 0.5 = 1.625, y = 1.5 * 0.25 = 0.375, z = 0 * 2 = 0."""
    g = O.Grid(3, (8, 4, 4), (0.5, 0.25, 2.0), 0.1, 2)
    rec = O.phase_space(g, particles(), (2, 1, 0), (8, 4, 4))
    np.testing.assert_array_equal(rec, [[1.625, 0.375, 0.0, 1.0, -1.0, 0.5, 1.0],
                                        [3.75, 0.5, 7.0, 2.0, -2.0, 0.25, 2.0],
                                        [1.875, 0.8125, 5.0, 3.0, -3.0, 0.125, 0.0],
                                        [2.75, 0.375, 1.5, 5.0, -5.0, 1.5, 5.0]])


def test_phase_space_subsampling_and_removed():
    """every = 2 keeps storage indices 0, 2, 4; skipping weight 0 drops particle 2."""
    g = O.Grid(3, (8, 4, 4), (0.5, 0.25, 2.0), 0.1, 2)
    rec = O.phase_space(g, particles(), (0, 0, 0), (8, 4, 4), every=2, skip_weightless=True)
    np.testing.assert_array_equal(rec[:, 3], [1.0, 5.0])  # u_0 of particles 0 and 4
    assert O.phase_space(g, particles(), (4, 0, 0), (4, 4, 4)).shape == (0, 7)  # an empty box


def test_phase_space_2d_has_two_positions():
    g = O.Grid(2, (8, 4, 1), (0.5, 0.25, 1.0), 0.1, 1)
    sp = particles()
    sp["cell"][2] = 0
    rec = O.phase_space(g, sp, (0, 0, 0), (8, 4, 1))
    assert rec.shape == (5, 6)
    np.testing.assert_array_equal(rec[3], [0.0, 0.125, 4.0, -4.0, 0.0, 4.0])
