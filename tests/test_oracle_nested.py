"""Oracle pins of three nested levels (more than two levels, as the cylinder
case of Sec. 10 nests refinement domains).  Reading: the two-level step of
Sec. 4.3 applied to each pair -- every substep of level 1 is a whole step of
the pair (level 1, level 2) -- with tau = 2 tau - 1/2 from one level to the
next (eq rescTau); the child pair receives the level-1 ring's rho and u at
its time, across which its H-RR collision takes centred differences.  BGK,
RR and H-RR.

* A uniform flow stays uniform on all three levels.
* After a few steps both interfaces obey the closed-form transfer relations
  of Sec. 4.2 exactly (the two-level pin's relations, rebuilt from their
  definitions, applied to the pair (0, 1) and to the pair (1, 2)); with
  H-RR at sigma = 0 also the collision relation a2 = (1 - 1/tau)(-2 tau rho
  c_s^2 S) at every node a level collides with its own centred differences
  -- on level 1 up to its ring, so the ring velocities the child used are
  checked against those of the ring's final state.  The child run without
  them (planted) breaks that relation.
* Derived bound, one level up: the three-level grid is the two-level grid
  with part of its patch refined once more; with a consistent interface its
  solution departs from the two-level one by no more than a uniformly
  refined solution departs from the uniform one at the patch's resolution:
  E(three-level - two-level) <= E(uniform 4x - uniform 2x), acoustic norm at
  the coarse nodes, smooth shear and acoustic fields.  Two planted mistakes
  in the nesting (the second child step started from the state at t; no
  ring rebuilt at t+1/2) break it by two orders of magnitude.
"""
import math

import numpy as np
import pytest

import oracle as O
from oracle_pins import acoustic_norm, check_interface_relations, fields_at

CS = 1.0 / math.sqrt(3.0)
TAU = 0.8


def _mesh(coords, D):
    g = np.meshgrid(*coords, indexing="ij")
    return [a.transpose(tuple(range(D))[::-1]).reshape(-1) for a in g]


def _coords(D, n, lo, hi, lo2, hi2, lv):
    if lv == 0:
        return [np.arange(n, dtype=float)] * D
    if lv == 1:
        return [lo + 0.5 * np.arange(2 * (hi - lo) + 1)] * D
    return [lo + 0.5 * (lo2 + 0.5 * np.arange(2 * (hi2 - lo2) + 1))] * D


def _nested(lat, model, kind, n, lo, hi, lo2, hi2, sigma=0.995):
    D = 2 if lat == O.D2Q9 else 3
    g = O.Nested(lat, model, (n,) * D, (lo,) * D, (hi,) * D, (lo2,) * D, (hi2,) * D, tau_c=TAU, sigma=sigma)
    for lv in (0, 1, 2):
        g.set_state(lv, *fields_at(kind, _mesh(_coords(D, n, lo, hi, lo2, hi2, lv), D), n, D))
    return g


SIZES = {O.D2Q9: (32, 8, 24, 8, 24), O.D3Q19: (16, 4, 12, 4, 12)}


@pytest.mark.parametrize("model", [O.BGK, O.RR, O.HRR])
@pytest.mark.parametrize("lat", [O.D2Q9, O.D3Q19])
def test_uniform_flow_stays_uniform(lat, model):
    D = 2 if lat == O.D2Q9 else 3
    n, lo, hi, lo2, hi2 = SIZES[lat]
    g = O.Nested(lat, model, (n,) * D, (lo,) * D, (hi,) * D, (lo2,) * D, (hi2,) * D, tau_c=TAU)
    U = np.array([0.05, -0.02, 0.01][:D])
    for lv in (0, 1, 2):
        N = g.nodes(lv)
        g.set_state(lv, np.ones(N), np.repeat(U[:, None], N, 1))
    g.step(8)
    for lv in (0, 1, 2):
        r, u = g.get_macros(lv)
        assert np.abs(r - 1).max() <= 1e-13 and np.abs(u - U[:, None]).max() <= 1e-13, lv


@pytest.mark.parametrize("kind", ["shear", "acoustic"])
@pytest.mark.parametrize("model", [O.BGK, O.RR])
@pytest.mark.parametrize("lat", [O.D2Q9, O.D3Q19])
def test_interface_relations_at_both_interfaces(lat, model, kind):
    n, lo, hi, lo2, hi2 = SIZES[lat]
    g = _nested(lat, model, kind, n, lo, hi, lo2, hi2)
    g.step(3)
    check_interface_relations(g.get_populations(0), g.get_populations(1), g.class_map(1), None, lat, model, n, lo,
                              hi, TAU, 1e-13, label=("levels 0-1", kind))
    check_interface_relations(g.get_populations(1), g.get_populations(2), g.class_map(2), None, lat, model,
                              2 * (hi - lo) + 1, lo2, hi2, 2 * TAU - 0.5, 1e-13, label=("levels 1-2", kind))


def _hrr_relations(lat, kind, steps=3):
    """H-RR, sigma = 0: the relations of both interfaces and of the collision
    (see the module docstring).  Level-1 nodes the child covers or transfers
    to are left out of the pair (0, 1)'s collision relation (level 2 decides
    them), and the level-1 ring out of the pair (1, 2)'s (the pair (0, 1)
    rebuilds it)."""
    n, lo, hi, lo2, hi2 = SIZES[lat]
    g = _nested(lat, O.HRR, kind, n, lo, hi, lo2, hi2, sigma=0.0)
    g.step(steps)
    c1, cc = g.class_map(1), g.child.class_map(0)
    f01 = c1.copy()
    f01[(cc == O.C_COVERED) | (cc == O.C_TNC)] = 99
    check_interface_relations(g.get_populations(0), g.get_populations(1), f01, g.class_map(0), lat, O.HRR, n, lo,
                              hi, TAU, 1e-13, label=("levels 0-1", kind))
    c12 = cc.copy()
    c12[np.isin(c1, [O.F_TFF, O.F_IE, O.F_IEFACE])] = 99
    check_interface_relations(g.get_populations(1), g.get_populations(2), g.class_map(2), c12, lat, O.HRR,
                              2 * (hi - lo) + 1, lo2, hi2, 2 * TAU - 0.5, 1e-13, label=("levels 1-2", kind))


@pytest.mark.parametrize("kind", ["shear", "acoustic"])
@pytest.mark.parametrize("lat", [O.D2Q9, O.D3Q19])
def test_hrr_relations_at_both_interfaces(lat, kind):
    _hrr_relations(lat, kind)


@pytest.mark.parametrize("lat", [O.D2Q9, O.D3Q19])
def test_hrr_child_without_ring_velocities_is_caught(lat):
    O.set_mutation("nest_inj")
    try:
        with pytest.raises(AssertionError):
            _hrr_relations(lat, "shear")
    finally:
        O.set_mutation(None)


def _bound(model, kind, steps=40):
    lat, D = O.D2Q9, 2
    n, lo, hi, lo2, hi2 = SIZES[lat]
    g3 = _nested(lat, model, kind, n, lo, hi, lo2, hi2)
    g3.step(steps)
    g2 = O.Grid(lat, model, (n,) * D, (lo,) * D, (hi,) * D, tau_c=TAU)
    for lv in (0, 1):
        g2.set_state(lv, *fields_at(kind, _mesh(_coords(D, n, lo, hi, 0, 0, lv), D), n, D))
    g2.step(steps)
    m = g2.class_map(0) != O.C_COVERED
    r3, u3 = g3.get_macros(0)
    r2, u2 = g2.get_macros(0)
    e = acoustic_norm((r3 - r2)[m], (u3 - u2)[:, m])
    ref = []
    for f, tau in ((2, 2 * TAU - 0.5), (4, 2 * (2 * TAU - 0.5) - 0.5)):
        u = O.Grid(lat, model, (f * n,) * D, tau_c=tau)
        u.set_state(0, *fields_at(kind, _mesh([np.arange(f * n) / f] * D, D), n, D))
        u.step(f * steps)
        r, v = u.get_macros(0)
        sub = (slice(None, None, f),) * D
        ref.append((r.reshape((f * n,) * D)[sub].reshape(-1), v.reshape((D,) + (f * n,) * D)[(slice(None),) + sub].reshape(D, -1)))
    eref = acoustic_norm(ref[1][0] - ref[0][0], ref[1][1] - ref[0][1])
    return e, eref


@pytest.mark.parametrize("kind", ["shear", "acoustic"])
@pytest.mark.parametrize("model", [O.BGK, O.RR, O.HRR])
def test_three_levels_within_the_refinement_difference(model, kind):
    e, eref = _bound(model, kind)
    assert e <= eref, (e, eref)


@pytest.mark.parametrize("mut", ["nest_sync", "nest_ring"])
def test_nesting_mistakes_are_caught(mut):
    O.set_mutation(mut)
    try:
        caught = any(e > eref for e, eref in (_bound(O.RR, kind) for kind in ("shear", "acoustic")))
    finally:
        O.set_mutation(None)
    assert caught
