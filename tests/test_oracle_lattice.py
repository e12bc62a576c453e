"""Oracle pins: lattices, equilibrium, collisions (Sec. 3)."""
import pytest

import oracle as O
import oracle_pins as P


@pytest.mark.parametrize("lat", [O.D2Q9, O.D3Q19])
def test_lattice_tables_and_isotropy(lat):
    P.pin_lattice(lat)


@pytest.mark.parametrize("lat", [O.D2Q9, O.D3Q19])
def test_equilibrium_moments(lat):
    P.pin_feq_moments(lat)


def test_equilibrium_matches_printed_closed_form():
    P.pin_feq_closed_form_d2q9()


@pytest.mark.parametrize("lat", [O.D2Q9, O.D3Q19])
@pytest.mark.parametrize("model", [O.BGK, O.RR, O.HRR])
def test_collision_conserves_mass_and_momentum(lat, model):
    P.pin_collision_invariants(lat, model)


@pytest.mark.parametrize("lat", [O.D2Q9, O.D3Q19])
def test_collision_special_cases(lat):
    P.pin_collision_special(lat)
