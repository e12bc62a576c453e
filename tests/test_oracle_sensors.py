"""Oracle pins of the non-hydrodynamic-mode sensors (Sec. 7, eqs
sensorSpuriousAc, sensorSpuriousS, fneqSplit, reguProceduref1S,
sensorSpuriousG).

Eigenmodes of the linearised scheme (oracle/lsa.py, Sec. 5) are set on a
uniform periodic grid and stepped once by the oracle:
* the SpuriousAc mode (acoustic content, pulsation near pi) flips the sign
  of the velocity divergence every step: its flag is set on every node;
* the SpuriousS mode (shear content, pulsation near pi) flips the curl: its
  flag is set on every node;
* physical shear and acoustic waves do not flip: a sign changes only where a
  zero crossing of the wave passes a node within the step, which bounds the
  flagged fraction by 2n / L for n periods over L nodes (each of the 2n
  crossings per row moves by less than one node per step);
* the ghost sensor tests the norm of the non-equilibrium part left after the
  second-order Hermite projection: zero for an equilibrium state or a purely
  second-order one, positive for fourth-order (ghost) content.
"""
import math

import numpy as np
import pytest

import oracle as O
from oracle import lsa

CS = math.sqrt(1.0 / 3.0)
NAMES = {O.BGK: "BGK", O.RR: "RR", O.HRR: "HRR"}


def _mode_state(model, n, L, axis, pick, tau=0.51, sigma=0.995, A=1e-6):
    """Uniform D2Q9 grid of L x L nodes holding one eigenmode of wave number
    2 pi n / L along `axis`, chosen by pick(wr, longitudinal, transverse):
    the momentum content along and across k (a mean flow across k mixes in
    a little of the other, hence ratios rather than zeros)."""
    s = lsa.Scheme("D2Q9", NAMES[model], tau, sigma)
    k = np.zeros(2)
    k[axis] = 2 * math.pi * n / L
    ub = np.array([0.1 * CS, 0.0])
    lam, V = s.eig(1.0, ub, k)
    M = lsa.macro_content(s, V)
    wr, _ = lsa.omega(lam)
    best, bscore = None, None
    for i in range(len(lam)):
        if abs(lam[i]) < 0.3:
            continue
        nrm = np.linalg.norm(V[:, i])
        lon = abs(M[1 + axis, i]) / nrm
        tra = abs(M[2 - axis, i]) / nrm
        sc = pick(wr[i], lon, tra)
        if sc is not None and (bscore is None or sc < bscore):
            best, bscore = i, sc
    assert best is not None
    F = np.exp(-1j * (s.xi @ k)) * V[:, best]  # post-collision eigenvector
    X = np.tile(np.arange(L), L)
    Y = np.repeat(np.arange(L), L)
    phase = np.exp(-1j * (k[0] * X + k[1] * Y + 0.37))
    g = O.Grid(O.D2Q9, model, (L, L), tau_c=tau, sigma=sigma)
    fbar = O.feq(O.D2Q9, 1.0, ub)
    g.set_populations(0, fbar[:, None] + A * np.real(F[:, None] * phase[None, :]))
    return g, wr[best]


def _near_pi(content):
    def pick(wr, lon, tra):
        if abs(abs(wr) - math.pi) > 0.35:
            return None
        if content == "lon" and not (lon > 1e-3 and tra < 1e-2 * lon):
            return None
        if content == "tra" and not (tra > 1e-3 and lon < 1e-2 * tra):
            return None
        return abs(abs(wr) - math.pi)
    return pick


def _physical(content):
    def pick(wr, lon, tra):
        if abs(wr) > 0.5:
            return None
        if content == "lon" and not (lon > 1e-3 and tra < 1e-2 * lon):
            return None
        if content == "tra" and not (tra > 1e-3 and lon < 1e-2 * tra):
            return None
        return abs(wr)
    return pick


@pytest.mark.parametrize("model", [O.BGK, O.RR, O.HRR])
@pytest.mark.parametrize("n,axis", [(15, 0), (2, 0), (15, 1)])
def test_spurious_ac_mode_flags_every_node(model, n, axis):
    g, wr = _mode_state(model, n, 32, axis, _near_pi("lon"))
    g.step(1)
    fl, dp, cp, gn = g.sensors(0, 1e-12)
    assert (fl & 1).all(), (NAMES[model], n, wr, (fl & 1).mean())
    assert not (fl & 4).any()  # the ghost flag yields to the SpuriousAc one


@pytest.mark.parametrize("model", [O.BGK, O.RR, O.HRR])
@pytest.mark.parametrize("axis", [0, 1])
def test_spurious_s_mode_flags_every_node(model, axis):
    g, wr = _mode_state(model, 2, 32, axis, _near_pi("tra"))
    g.step(1)
    fl, dp, cp, gn = g.sensors(0, 1e-12)
    assert ((fl >> 1) & 1).all(), (NAMES[model], wr, ((fl >> 1) & 1).mean())
    assert not (fl & 4).any()


@pytest.mark.parametrize("model", [O.BGK, O.RR, O.HRR])
@pytest.mark.parametrize("n", [1, 2, 3])
def test_physical_modes_flip_only_at_zero_crossings(model, n):
    L = 32
    g, wr = _mode_state(model, n, L, 0, _physical("tra"))
    g.step(1)
    fl, dp, cp, gn = g.sensors(0, 1e-12)
    assert ((fl >> 1) & 1).mean() <= 2 * n / L, ("shear", ((fl >> 1) & 1).mean())
    g, wr = _mode_state(model, n, L, 0, _physical("lon"))
    g.step(1)
    fl, dp, cp, gn = g.sensors(0, 1e-12)
    assert (fl & 1).mean() <= 2 * n / L, ("acoustic", (fl & 1).mean())


def _uniform(f):
    g = O.Grid(O.D2Q9, O.BGK, (8, 8), tau_c=0.7)
    g.set_populations(0, np.repeat(f[:, None], 64, axis=1))
    g.step(1)
    return g.sensors(0, 1e-12)


def test_ghost_sensor():
    D, Q, xi, w = O.lattice(O.D2Q9)
    rho, u = 1.02, np.array([0.04, -0.03])
    f0 = O.feq(O.D2Q9, rho, u)
    cx, cy = xi[:, 0].astype(float), xi[:, 1].astype(float)
    # equilibrium: no non-equilibrium part at all
    fl, dp, cp, gn = _uniform(f0)
    assert not fl.any() and gn.max() < 1e-15
    # second-order non-equilibrium only (eq reguProceduref1S form): no ghost part
    a = np.array([[2e-3, -1e-3], [-1e-3, 5e-4]])
    H = lambda i: np.array([[cx[i] * cx[i] - 1 / 3, cx[i] * cy[i]], [cx[i] * cy[i], cy[i] * cy[i] - 1 / 3]])
    f1s = np.array([w[i] * 4.5 * np.sum(H(i) * a) for i in range(Q)])
    fl, dp, cp, gn = _uniform(f0 + f1s)
    assert not fl.any() and gn.max() < 1e-15
    # fourth-order content H_xxyy = (cx^2 - 1/3)(cy^2 - 1/3): orthogonal to
    # 1, xi and H^(2) on D2Q9, so it is all ghost
    h4 = np.array([w[i] * (cx[i] ** 2 - 1 / 3) * (cy[i] ** 2 - 1 / 3) for i in range(Q)])
    fl, dp, cp, gn = _uniform(f0 + f1s + 1e-4 * h4)
    assert (fl == 4).all()
    assert np.allclose(gn, 1e-4 * np.linalg.norm(h4), rtol=1e-9)


def test_two_level_sensors_leave_interface_nodes_unflagged():
    from paper_2004_11863_amd import inputs as I
    wl = I.vortex_crossing_64(0)
    g0 = wl.geom
    g = O.Grid(O.D2Q9, O.HRR, g0.n[:2], g0.lo[:2], g0.hi[:2], tau_c=0.51)
    for lv in (0, 1):
        g.set_state(lv, *I.fields(wl, lv))
    with pytest.raises(ValueError):
        g.sensors(0, 1e-12)  # no step taken yet
    g.step(3)
    fl0 = g.sensors(0, 1e-10)[0]
    fl1 = g.sensors(1, 1e-10)[0]
    c0, c1 = g.class_map(0), g.class_map(1)
    assert not fl0[(c0 == O.C_TNC) | (c0 == O.C_COVERED)].any()
    assert not fl1[(c1 == O.F_TFF) | (c1 == O.F_IE) | (c1 == O.F_IEFACE)].any()
    assert fl0.any() and fl1.any()
