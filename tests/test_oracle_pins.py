"""The oracle against closed forms, identities, special cases and brute force."""
import pytest

import pins

IDS = [
    "shape_values", "shape_moments",
    "gather_uniform_3d_q", "gather_uniform_2d_l",
    "gather_linear_3d_q", "gather_linear_3d_l", "gather_linear_2d_q",
    "gather_brute_3d_q", "gather_brute_2d_l",
    "boris_gyration", "boris_exb", "boris_pure_e", "free_streaming",
    "yee_eigenmode_3d", "yee_eigenmode_2d", "yee_stability",
    "yee_energy_3d", "yee_energy_2d",
    "continuity_3d_q", "continuity_3d_l", "continuity_2d_q", "continuity_2d_l",
    "total_current_3d_q", "total_current_2d_l",
    "x_only_q", "x_only_l", "jz_2d_q", "jz_2d_l", "jz_2d_time_average",
    "cold_k0_2d_l", "cold_k0_3d_q", "plasma_frequency",
    "gauss_3d_q", "gauss_2d_l", "translation_3d_q", "translation_2d_l",
    "mur_reflection_2d", "mur_reflection_3d", "laser_plane_wave", "absorption_gauss",
    "field_energy_uniform_3d", "field_energy_uniform_2d", "field_energy_wave_3d", "field_energy_wave_2d",
    "kinetic_energy_rational", "tile_sort_hand_counted",
]
assert len(IDS) == len(pins.ALL_PINS)


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=IDS)
def test_pin(pin):
    pin()


def test_two_stream_growth_rate():
    """The whole FP64 loop against the cold two-stream growth rate (kept out of
    the mutant sweep, which runs every pin per planted mistake, for its length)."""
    pins.pin_two_stream_growth()
