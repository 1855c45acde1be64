"""The pins must catch plausible mistakes: each case below compiles a copy of
the oracle with one planted mistake (on the CPU, in a temporary directory) and
asserts that at least one pin fails against it."""
import os
import subprocess

import numpy as np
import pytest

import oracle
import pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

# (name, original text, mutated text): each replaces the first occurrence
MUTANTS = [
    ("quadratic_centre", "if (a <= 0.5) return 0.75 - a * a;", "if (a <= 0.5) return 0.75 - a;"),
    ("linear_shape", "return a < 1.0 ? 1.0 - a : 0.0;", "return a < 1.0 ? 1.0 - a * a : 0.0;"),
    ("gather_stagger_Bx", "{0.0, 0.5, 0.5}, {0.5, 0.0, 0.5}", "{0.5, 0.5, 0.5}, {0.5, 0.0, 0.5}"),
    ("gather_stagger_sign", "((double)(-di) - STAG[c][0]) + off[0]", "((double)(-di) + STAG[c][0]) + off[0]"),
    ("boris_s_factor", "double s[3] = {2.0 * t[0] / (1.0 + t2), 2.0 * t[1] / (1.0 + t2), 2.0 * t[2] / (1.0 + t2)};",
     "double s[3] = {t[0] / (1.0 + t2), t[1] / (1.0 + t2), t[2] / (1.0 + t2)};"),
    ("boris_cross_sign", "um[0] + (up[1] * s[2] - up[2] * s[1])", "um[0] + (up[2] * s[1] - up[1] * s[2])"),
    ("boris_second_kick", "ux[p] = uplus[0] + h * E[0];", "ux[p] = uplus[0];"),
    ("boris_gamma", "double t[3] = {h * B[0] / gm, h * B[1] / gm, h * B[2] / gm};",
     "double t[3] = {h * B[0], h * B[1], h * B[2]};"),
    ("move_nonrelativistic", "double disp = g->dt * (u[d] / gam) / g->dx[d];", "double disp = g->dt * u[d] / g->dx[d];"),
    ("move_wrong_dx", "double disp = g->dt * (u[d] / gam) / g->dx[d];", "double disp = g->dt * (u[d] / gam) / g->dx[0];"),
    ("esirkepov_half", "+ 0.5 * DS[1][j] * S0[2][k]", "+ DS[1][j] * S0[2][k]"),
    ("esirkepov_third", "DS[1][j] * DS[2][k] / 3.0", "DS[1][j] * DS[2][k] / 2.0"),
    ("esirkepov_sign", "double cx = -qw * g->dx[0] / g->dt, cy", "double cx = qw * g->dx[0] / g->dt, cy"),
    ("esirkepov_new_cell", "double xi1 = (2.0 + (double)dcell[(int64_t)d * np + p]) + o1[d][p];",
     "double xi1 = 2.0 + o1[d][p];"),
    ("esirkepov_2d_jz_velocity", "qw * vz * Wz[j][i]", "qw * uz[p] * Wz[j][i]"),
    ("esirkepov_2d_jz_weight", "Wz[j][i] = S0[0][i] * S0[1][j] + 0.5 * DS[0][i] * S0[1][j]",
     "Wz[j][i] = S0[0][i] * S0[1][j] + DS[0][i] * S0[1][j]"),
    ("yee_b_sign", "Bx[o] -= c * (dEz_dy - dEy_dz);", "Bx[o] -= c * (dEz_dy + dEy_dz);"),
    ("yee_b_dz", "double dEy_dz = three ? (Ey[lin(g, i, j, k + 1)] - Ey[o]) / g->dx[2] : 0.0;",
     "double dEy_dz = three ? (Ey[lin(g, i, j, k + 1)] - Ey[o]) / g->dx[1] : 0.0;"),
    ("yee_e_current_sign", "Ex[o] += c * ((dBz_dy - dBy_dz) - Jx[o]);", "Ex[o] += c * ((dBz_dy - dBy_dz) + Jx[o]);"),
    ("yee_e_forward_difference", "double dBz_dy = (Bz[o] - Bz[lin(g, i, j - 1, k)]) / g->dx[1];",
     "double dBz_dy = (Bz[lin(g, i, j + 1, k)] - Bz[o]) / g->dx[1];"),
    ("mur_coefficient_sign", "const double a = (g->dt - g->dx[0]) / (g->dt + g->dx[0]);",
     "const double a = (g->dx[0] - g->dt) / (g->dt + g->dx[0]);"),
    ("mur_low_planes", "f[0 + n0 * jk] = o[1 * nyz + jk] + a * (f[1 + n0 * jk] - o[0 * nyz + jk]);",
     "f[0 + n0 * jk] = o[0 * nyz + jk] + a * (f[1 + n0 * jk] - o[1 * nyz + jk]);"),
    ("mur_high_planes", "o[2 * nyz + jk] + a * (f[(n0 - 2) + n0 * jk] - o[3 * nyz + jk]);",
     "o[3 * nyz + jk] + a * (f[(n0 - 2) + n0 * jk] - o[2 * nyz + jk]);"),
    ("laser_sheet_factor", "return -e0 * dt * sin(k * dx) / (dx * dx * s);",
     "return -e0 * dt * sin(0.5 * k * dx) / (dx * dx * s);"),
    ("laser_sign", "return -e0 * dt * sin(k * dx) / (dx * dx * s);", "return e0 * dt * sin(k * dx) / (dx * dx * s);"),
    ("laser_stagger", "double y = ((double)j + (pol == 1 ? 0.5 : 0.0)) * g->dx[1];", "double y = (double)j * g->dx[1];"),
    ("absorb_edge", "(ix[p] < lo || ix[p] >= hi)", "(ix[p] <= lo || ix[p] >= hi)"),
    ("rho_volume", "+= q * w[p] / dV * (wx * wy * wz);", "+= q * w[p] * (wx * wy * wz);"),
    ("div_stagger", "double d = (Fx[o] - Fx[lin(g, i - 1, j, k)]) / g->dx[0]",
     "double d = (Fx[lin(g, i + 1, j, k)] - Fx[o]) / g->dx[0]"),
    ("field_energy_half", "return 0.5 * s * cell_volume(g);", "return s * cell_volume(g);"),
    ("field_energy_volume", "return 0.5 * s * cell_volume(g);", "return 0.5 * s;"),
    ("kinetic_gamma", "s += w[p] * m * (gam - 1.0);", "s += w[p] * m * gam;"),
    ("kinetic_mass", "s += w[p] * m * (gam - 1.0);", "s += w[p] * (gam - 1.0);"),
]


def _run_pins():
    failed = []
    for i, p in enumerate(pins.ALL_PINS):
        try:
            p()
        except AssertionError:
            failed.append(i)
        except Exception:  # a crash or a NaN comparison counts as caught
            failed.append(i)
    return failed


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(tmp_path, name, old, new):
    src = open(SRC).read()
    assert old in src, f"mutation target for {name} not found"
    mutated = src.replace(old, new, 1)
    c = tmp_path / "oracle_mut.c"
    c.write_text(mutated)
    so = tmp_path / "liboracle_mut.so"
    subprocess.check_call(["gcc", *oracle.CFLAGS, "-o", str(so), str(c), "-lm"])
    with oracle.use_library(str(so)):
        failed = _run_pins()
    assert failed, f"no pin caught mutant {name}"


def _keys_y_fastest(grid, tile, cell):
    nty = grid.n[1] // tile[1]
    ntx = grid.n[0] // tile[0]
    tz = cell[2] // tile[2] if grid.dims == 3 else np.zeros_like(cell[0])
    return (cell[1] // tile[1] + nty * (cell[0] // tile[0] + ntx * tz)).astype(np.int64)


def _keys_no_z(grid, tile, cell):
    ntx = grid.n[0] // tile[0]
    return (cell[0] // tile[0] + ntx * (cell[1] // tile[1])).astype(np.int64)


def _sort_reversed_ties(grid, tile, sp):
    keys = oracle.tile_keys(grid, tile, sp["cell"])
    order = np.lexsort((-np.arange(keys.shape[0]), keys))  # equal keys in reverse order
    out = dict(sp)
    for k in ("cell", "off", "u"):
        out[k] = np.ascontiguousarray(sp[k][:, order])
    out["w"] = np.ascontiguousarray(sp["w"][order])
    ntiles = (grid.n[0] // tile[0]) * (grid.n[1] // tile[1]) * (grid.n[2] // tile[2])
    start = np.zeros(ntiles + 1, np.int64)
    start[1:] = np.cumsum(np.bincount(keys, minlength=ntiles))
    return out, start


def _sort_starts_shifted(grid, tile, sp):
    out, start = _ORIG_SORT(grid, tile, sp)
    start = start.copy()
    start[1:-1] += 1
    return out, start


_ORIG_SORT = oracle.tile_sort


@pytest.mark.parametrize("name,attr,fn", [("keys_y_fastest", "tile_keys", _keys_y_fastest),
                                          ("keys_drop_z", "tile_keys", _keys_no_z),
                                          ("sort_unstable", "tile_sort", _sort_reversed_ties),
                                          ("sort_starts", "tile_sort", _sort_starts_shifted)])
def test_tile_pin_catches_python_mutant(monkeypatch, name, attr, fn):
    monkeypatch.setattr(oracle, attr, fn)
    with pytest.raises(AssertionError):
        pins.pin_tile_sort_hand_counted()
