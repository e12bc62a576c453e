"""The pins are sensitive: every planted mistake in the oracle (a dropped
term, a wrong sign, swapped weights, a wrong factor, a shifted stencil) trips
at least one of them.  The mistakes are planted in the CPU oracle only."""
import pytest

import oracle as O
import oracle_pins as P

# cheapest first: a mutation is reported by the first pin it trips
PINS = [
    ("feq_moments", lambda: P.pin_feq_moments(O.D2Q9)),
    ("feq_closed_form", P.pin_feq_closed_form_d2q9),
    ("collision_special", lambda: P.pin_collision_special(O.D2Q9)),
    ("temporal", P.pin_temporal_interp),
    ("cubic", P.pin_cubic_interp),
    ("filter2", lambda: P.pin_filter(2)),
    ("filter3", lambda: P.pin_filter(3)),
    ("rescaling", P.pin_rescaling),
    ("stencils", lambda: P.pin_ring_stencils(O.D2Q9)),
    ("relations_2d_rr", lambda: P.pin_interface_relations(O.D2Q9, O.RR)),
    ("relations_2d_hrr", lambda: P.pin_interface_relations(O.D2Q9, O.HRR)),
    ("plane_wave_rr", lambda: P.pin_plane_wave(O.D2Q9, O.RR, 0.8, (2, 3), 32, steps=6)),
    ("plane_wave_hrr", lambda: P.pin_plane_wave(O.D2Q9, O.HRR, 0.8, (2, 3), 32, steps=6, sigma=0.3)),
    ("two_level_shear", lambda: P.pin_two_level_vs_uniform("shear", O.RR)),
    ("two_level_acoustic", lambda: P.pin_two_level_vs_uniform("acoustic", O.RR)),
    ("two_level_hrr_sigma0", lambda: P.pin_two_level_vs_uniform("shear", O.HRR, sigma=0.0)),
]
# pins of the three-dimensional interface (D3Q19 ring, face centres, 27-point
# filter, strain-rate hand-off)
PINS_3D = [
    ("stencils_3d", lambda: P.pin_ring_stencils(O.D3Q19)),
    ("relations_3d_rr", lambda: P.pin_interface_relations(O.D3Q19, O.RR)),
    ("relations_3d_hrr", lambda: P.pin_interface_relations(O.D3Q19, O.HRR)),
    ("two_level_3d_shear", lambda: P.pin_two_level_vs_uniform("shear", O.RR, lat=O.D3Q19)),
    ("two_level_3d_acoustic", lambda: P.pin_two_level_vs_uniform("acoustic", O.HRR, sigma=0.0, lat=O.D3Q19)),
]
# mistakes that only exist in three dimensions, or that the 3D pins must see
# on their own
MUTATIONS_3D = ["filter_zoff", "face_axes", "sc_half", "rescale_swap", "temporal_rev", "tauf", "spatial_lin"]


def _first_failing(pins):
    for name, fn in pins:
        try:
            fn()
        except (AssertionError, ValueError, FloatingPointError):
            return name
    return None


def test_all_pins_pass_without_mutation():
    O.set_mutation(None)
    bad = [name for name, fn in PINS + PINS_3D if _first_failing([(name, fn)])]
    assert bad == []


# (the nest_* mistakes act only in nested grids; the nested pins catch them)
@pytest.mark.parametrize("mutation", sorted(m for m in O.MUTATIONS if not m.startswith("nest_")))
def test_mutation_is_detected(mutation):
    O.set_mutation(mutation)
    try:
        hit = _first_failing(PINS + PINS_3D)
    finally:
        O.set_mutation(None)
    assert hit, f"planted mistake {mutation!r} passed every pin"


@pytest.mark.parametrize("mutation", MUTATIONS_3D)
def test_mutation_is_detected_by_3d_pins(mutation):
    O.set_mutation(mutation)
    try:
        hit = _first_failing(PINS_3D)
    finally:
        O.set_mutation(None)
    assert hit, f"planted mistake {mutation!r} passed every three-dimensional pin"
