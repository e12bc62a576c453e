"""Oracle pins of the dynamic-sigma H-RR variant, which Sec. 9.3 and Sec. 11
suggest without defining: sigma is lowered (more finite-difference stress)
only at nodes where the non-hydrodynamic sensors of Sec. 7 fire.

Reading (stated in the oracle): at each bulk H-RR collision the SpuriousAc and
SpuriousS tests compare the divergence and curl of the velocity gradient the
collision uses with those of the node's previous bulk collision; where either
product lies below -thr the node takes sigma_dyn, elsewhere the grid's sigma
(thr = 0 is the paper's tie-break; a small thr keeps the products of a
field's rounding noise, e.g. the divergence of a pure shear wave, from
switching).

The pins tie the switch to the sensors, which are pinned by eigenmodes of the
linearised scheme (test_oracle_sensors.py), and to the static scheme:
* sigma_dyn equal to sigma reproduces the static scheme bit for bit;
* the nodes that take sigma_dyn are exactly those the Sec. 7 sensors flag
  (SpuriousAc or SpuriousS) for the same iteration, on both levels, in 2D
  and 3D;
* a SpuriousAc eigenmode fires everywhere from the second step, so two
  dynamic steps equal one static step at sigma followed by one static step
  at sigma_dyn, bit for bit;
* a physical shear or acoustic wave switches only where a zero crossing
  passes a node, once the threshold clears rounding noise.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2004_11863_amd import inputs as I
from test_oracle_sensors import _mode_state, _near_pi, _physical


def _grid(wl, lat=O.D2Q9, sigma=0.995, tau=0.51):
    g = wl.geom
    D = g.D
    lo = g.lo[:D] if g.has_fine else None
    hi = g.hi[:D] if g.has_fine else None
    r = O.Grid(lat, O.HRR, g.n[:D], lo, hi, tau_c=tau, sigma=sigma)
    for lv in ((0, 1) if g.has_fine else (0,)):
        rho, u = I.fields(wl, lv)
        r.set_state(lv, rho, u)
    return r


def _vortex_and_pulse():
    wl = I.vortex_crossing_64(1)
    wl.pulses = [I.Pulse(center=(40.0, 30.0), A=1e-2)]
    return wl


def _pulse_3d():
    geom = I.Geometry(3, (22, 20, 24), (5, 4, 6), (15, 14, 17))
    return I.Workload(geom=geom, U=(0.1 / math.sqrt(3), 0.01, -0.005),
                      pulses=[I.Pulse(center=(15.2, 9.6, 11.1), A=1e-3, R=2.5)])


def test_sigma_dyn_equal_to_sigma_is_the_static_scheme():
    a = _grid(_vortex_and_pulse())
    a.set_dynamic_sigma(True, 0.995)
    b = _grid(_vortex_and_pulse())
    a.step(10)
    b.step(10)
    for lv in (0, 1):
        assert np.array_equal(a.get_populations(lv), b.get_populations(lv))
    assert a.dynamic_mask(0).any()  # the switch fired, with no effect


def test_dynamic_sigma_needs_hrr_and_a_valid_sigma():
    wl = I.vortex_crossing_64(0)
    g = wl.geom
    r = O.Grid(O.D2Q9, O.RR, g.n[:2], g.lo[:2], g.hi[:2], tau_c=0.51, sigma=0.995)
    with pytest.raises(ValueError):
        r.set_dynamic_sigma(True, 0.0)
    h = _grid(wl)
    with pytest.raises(ValueError):
        h.set_dynamic_sigma(True, 1.5)


@pytest.mark.parametrize("thr", [0.0, 1e-12])
@pytest.mark.parametrize("case", ["2d", "3d"])
def test_switched_nodes_are_the_sensor_flags(case, thr):
    """The nodes that took sigma_dyn are those whose Sec. 7 divergence or curl
    product (as the sensors report it for the same iteration) lies below
    -thr; thr = 0 is the sensors' own SpuriousAc / SpuriousS flags."""
    wl, lat, steps = (_vortex_and_pulse(), O.D2Q9, 7) if case == "2d" else (_pulse_3d(), O.D3Q19, 5)
    r = _grid(wl, lat)
    r.set_dynamic_sigma(True, 0.0, thr)
    evolved = {0: np.isin(r.class_map(0), [O.C_MIDDLE, O.C_TFC]),
               1: np.isin(r.class_map(1), [O.F_MIDDLE, O.F_TNF])}
    seen = 0
    for t in range(steps):
        r.step(1)
        if t == 0:
            # the coarse level has no earlier collision to compare with; the
            # fine level's second substep compares with its first
            assert not r.dynamic_mask(0).any()
        for lv in ((1,) if t == 0 else (0, 1)):
            m = r.dynamic_mask(lv).astype(bool)
            fl, dp, cp, _ = r.sensors(lv, 1e-8)
            ev = evolved[lv]
            assert np.array_equal(m[ev], (dp[ev] < -thr) | (cp[ev] < -thr)), (t, lv)
            if thr == 0.0:
                assert np.array_equal(m[ev], (fl[ev] & 3) != 0), (t, lv)
            assert not m[~ev].any()
            seen += int(m.sum())
    assert seen > 0


@pytest.mark.parametrize("n,axis,thr", [(15, 0, 0.0), (15, 1, 0.0), (15, 0, 1e-24)])
def test_spurious_ac_mode_takes_sigma_dyn_everywhere(n, axis, thr):
    """A mode with pulsation within 0.35 of pi: the product of consecutive
    divergences, cos(phi) cos(phi - omega) at phase phi, is negative at every
    node when omega is close enough to pi for the 32 phases of a row (n = 15;
    at n = 2 some nodes fall in the positive band of width pi - |omega|)."""
    L, sd = 32, 0.0
    a, _ = _mode_state(O.HRR, n, L, axis, _near_pi("lon"))
    a.set_dynamic_sigma(True, sd, thr)
    a.step(1)
    assert not a.dynamic_mask(0).any()  # nothing to compare with before the first collision
    a.step(1)
    assert a.dynamic_mask(0).all()
    b, _ = _mode_state(O.HRR, n, L, axis, _near_pi("lon"))
    b.step(1)
    c = O.Grid(O.D2Q9, O.HRR, (L, L), tau_c=0.51, sigma=sd)
    c.set_populations(0, b.get_populations(0))
    c.step(1)
    assert np.array_equal(a.get_populations(0), c.get_populations(0))


@pytest.mark.parametrize("content", ["tra", "lon"])
@pytest.mark.parametrize("n", [1, 2])
def test_physical_wave_switches_only_at_zero_crossings(n, content):
    """A physical shear (acoustic) wave along x has no divergence (curl) at
    all, so that product is rounding noise; above a threshold of 1e-24
    (products of the wave itself are ~1e-15) a node switches only where a zero
    crossing passes it: at most 2n / L of the nodes per step."""
    L = 32
    a, wr = _mode_state(O.HRR, n, L, 0, _physical(content))
    a.set_dynamic_sigma(True, 0.0, 1e-24)
    a.step(1)
    for _ in range(4):
        a.step(1)
        assert a.dynamic_mask(0).mean() <= 2 * n / L, (n, wr, a.dynamic_mask(0).mean())
