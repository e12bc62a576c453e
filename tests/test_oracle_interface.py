"""Oracle pins: refinement-interface primitives and two-level runs (Sec. 4)."""
import pytest

import oracle as O
import oracle_pins as P


def test_temporal_interpolation():
    P.pin_temporal_interp()


def test_cubic_interpolation():
    P.pin_cubic_interp()


@pytest.mark.parametrize("lat", [O.D2Q9, O.D3Q19])
def test_ring_stencils_reproduce_cubics(lat):
    P.pin_ring_stencils(lat)


@pytest.mark.parametrize("D", [2, 3])
def test_filter(D):
    P.pin_filter(D)


def test_rescaling():
    P.pin_rescaling()


@pytest.mark.parametrize("lat,n,lo,hi", [(O.D2Q9, 64, 16, 48), (O.D2Q9, 30, 5, 14), (O.D3Q19, 20, 4, 12),
                                         (O.D3Q19, 24, 6, 17)])
def test_node_class_counts(lat, n, lo, hi):
    P.pin_counts(lat, n, lo, hi)


@pytest.mark.parametrize("lat", [O.D2Q9, O.D3Q19])
@pytest.mark.parametrize("model", [O.BGK, O.RR, O.HRR])
def test_uniform_flow_stays_uniform(lat, model):
    P.pin_uniform_flow(lat, model, steps=60 if lat == O.D2Q9 else 12)


@pytest.mark.parametrize("lat", [O.D2Q9, O.D3Q19])
@pytest.mark.parametrize("kind", ["shear", "acoustic"])
@pytest.mark.parametrize("model,sigma", [(O.BGK, 0.995), (O.RR, 0.995), (O.HRR, 0.995), (O.HRR, 0.0)])
def test_two_level_within_refinement_difference(lat, kind, model, sigma):
    P.pin_two_level_vs_uniform(kind, model, sigma=sigma, lat=lat)


@pytest.mark.parametrize("lat", [O.D2Q9, O.D3Q19])
@pytest.mark.parametrize("kind", ["shear", "acoustic"])
@pytest.mark.parametrize("model", [O.BGK, O.RR, O.HRR])
def test_interface_relations_after_step(lat, kind, model):
    P.pin_interface_relations(lat, model, kind)
