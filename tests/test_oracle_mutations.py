"""The pins are sensitive: every planted mistake in the oracle (a dropped
term, a wrong sign, swapped weights, a wrong factor) trips at least one of
them.  The mistakes are planted in the CPU oracle only."""
import pytest

import oracle as O
import oracle_pins as P

PINS = [
    ("feq_moments", lambda: P.pin_feq_moments(O.D2Q9)),
    ("feq_closed_form", P.pin_feq_closed_form_d2q9),
    ("collision_special", lambda: P.pin_collision_special(O.D2Q9)),
    ("plane_wave_rr", lambda: P.pin_plane_wave(O.D2Q9, O.RR, 0.8, (2, 3), 32, steps=6)),
    ("plane_wave_hrr", lambda: P.pin_plane_wave(O.D2Q9, O.HRR, 0.8, (2, 3), 32, steps=6, sigma=0.3)),
    ("temporal", P.pin_temporal_interp),
    ("cubic", P.pin_cubic_interp),
    ("stencils", lambda: P.pin_ring_stencils(O.D2Q9)),
    ("filter2", lambda: P.pin_filter(2)),
    ("filter3", lambda: P.pin_filter(3)),
    ("rescaling", P.pin_rescaling),
    ("two_level_shear", lambda: P.pin_two_level_vs_uniform("shear", O.RR)),
    ("two_level_acoustic", lambda: P.pin_two_level_vs_uniform("acoustic", O.RR)),
    ("two_level_hrr_sigma0", lambda: P.pin_two_level_vs_uniform("shear", O.HRR, sigma=0.0)),
]


def _failing():
    bad = []
    for name, fn in PINS:
        try:
            fn()
        except (AssertionError, ValueError, FloatingPointError):
            bad.append(name)
    return bad


def test_all_pins_pass_without_mutation():
    O.set_mutation(None)
    assert _failing() == []


@pytest.mark.parametrize("mutation", sorted(O.MUTATIONS))
def test_mutation_is_detected(mutation):
    O.set_mutation(mutation)
    try:
        bad = _failing()
    finally:
        O.set_mutation(None)
    assert bad, f"planted mistake {mutation!r} passed every pin"
