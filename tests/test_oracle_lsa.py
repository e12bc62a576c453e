"""Oracle pins: linear stability analysis (Sec. 5, App. A) and plane waves."""
import pytest

import oracle as O
import oracle_pins as P


def test_mode_counts_match_paper():
    P.pin_lsa_mode_counts()


def test_spurious_ac_damping_ratio_418():
    P.pin_spurious_ac_ratio()


def test_small_k_limit_is_navier_stokes():
    P.pin_ns_limit()


@pytest.mark.parametrize("model", [O.BGK, O.RR, O.HRR])
@pytest.mark.parametrize("tau,nvec", [(0.51, (1, 0)), (0.8, (2, 3))])
def test_plane_wave_d2q9(model, tau, nvec):
    P.pin_plane_wave(O.D2Q9, model, tau, nvec, 32)


@pytest.mark.parametrize("model", [O.BGK, O.RR, O.HRR])
def test_plane_wave_d3q19(model):
    P.pin_plane_wave(O.D3Q19, model, 0.55, (1, 2, 1), 10, steps=8)
