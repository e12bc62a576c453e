"""Oracle pins: equilibrium fixed point and exact conservation on periodic
uniform grids."""
import pytest

import oracle as O
import oracle_pins as P


@pytest.mark.parametrize("lat", [O.D2Q9, O.D3Q19])
@pytest.mark.parametrize("model", [O.BGK, O.RR, O.HRR])
def test_equilibrium_is_fixed_point(lat, model):
    P.pin_fixed_point(lat, model, L=8 if lat == O.D2Q9 else 5, steps=200 if lat == O.D2Q9 else 60)


@pytest.mark.parametrize("lat", [O.D2Q9, O.D3Q19])
@pytest.mark.parametrize("model", [O.BGK, O.RR, O.HRR])
def test_mass_momentum_conserved(lat, model):
    P.pin_conservation(lat, model, L=16 if lat == O.D2Q9 else 6, steps=300 if lat == O.D2Q9 else 60)
