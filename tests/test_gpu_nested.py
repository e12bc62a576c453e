"""Three nested levels on the GPU (lbm_create_nested) against the oracle's
nested grid: the two-level step applied to each pair, every substep of level
1 a whole step of the pair (1, 2), which with H-RR takes the level-1 ring's
rho and u at its own time.  BGK, RR and H-RR (sigma 0.995 and 0), D2Q9 (the
coarse level in the one-pass H-RR form, level 1 in the two-pass form) and
D3Q19.  FP64 within 1e-12 relative on rho, u and the populations of every
evolved node of the three levels; FP32 deviation storage within the stated
FP32 bars."""

import numpy as np
import pytest

import oracle as O
from oracle_pins import fields_at

pytestmark = pytest.mark.gpu

TAU = 0.8


def _lbm():
    from paper_2004_11863_amd import lbm
    return lbm


def _mesh(coords, D):
    g = np.meshgrid(*coords, indexing="ij")
    return [a.transpose(tuple(range(D))[::-1]).reshape(-1) for a in g]


def _coords(D, n, lo, hi, lo2, hi2, lv):
    if lv == 0:
        return [np.arange(n, dtype=float)] * D
    if lv == 1:
        return [lo + 0.5 * np.arange(2 * (hi - lo) + 1)] * D
    return [lo + 0.5 * (lo2 + 0.5 * np.arange(2 * (hi2 - lo2) + 1))] * D


SIZES = {2: (40, 10, 30, 9, 31), 3: (18, 4, 14, 5, 15)}


def _pair(D, model, prec, kind, sigma=0.995):
    lbm = _lbm()
    lat, olat = (lbm.LBM_D2Q9, O.D2Q9) if D == 2 else (lbm.LBM_D3Q19, O.D3Q19)
    mg, mo = {"BGK": (lbm.LBM_BGK, O.BGK), "RR": (lbm.LBM_RR, O.RR), "HRR": (lbm.LBM_HRR, O.HRR)}[model]
    n, lo, hi, lo2, hi2 = SIZES[D]
    gpu = lbm.Nested(lat, mg, prec, (n,) * D, (lo,) * D, (hi,) * D, (lo2,) * D, (hi2,) * D, tau_coarse=TAU,
                     sigma=sigma)
    ref = O.Nested(olat, mo, (n,) * D, (lo,) * D, (hi,) * D, (lo2,) * D, (hi2,) * D, tau_c=TAU, sigma=sigma)
    for lv in (0, 1, 2):
        rho, u = fields_at(kind, _mesh(_coords(D, n, lo, hi, lo2, hi2, lv), D), n, D)
        gpu.set_state(lv, rho, u)
        ref.set_state(lv, rho, u)
    return gpu, ref


def _evolved(ref):
    """Nodes each level evolves: level 0 not covered by level 1, level 1 not
    covered by level 2, level 2 all."""
    return {0: ref.class_map(0) != O.C_COVERED, 1: ref.child.class_map(0) != O.C_COVERED,
            2: np.ones(ref.nodes(2), bool)}


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("kind", ["shear", "acoustic"])
@pytest.mark.parametrize("model", ["BGK", "RR", "HRR", "HRR0"])
@pytest.mark.parametrize("D", [2, 3])
def test_nested_fp64_matches_oracle(D, model, kind):
    lbm = _lbm()
    sigma = 0.0 if model == "HRR0" else 0.995
    gpu, ref = _pair(D, model[:3] if model.startswith("HRR") else model, lbm.LBM_FP64, kind, sigma)
    steps = 6 if D == 3 else 10
    gpu.step(steps)
    ref.step(steps)
    ev = _evolved(ref)
    worst = {}
    for lv in (0, 1, 2):
        m = ev[lv]
        r1, u1 = gpu.get_macros(lv)
        r0, u0 = ref.get_macros(lv)
        worst[f"rho{lv}"] = _rel(r1[m], r0[m])
        worst[f"u{lv}"] = _rel(u1[:, m], u0[:, m])
        worst[f"f{lv}"] = _rel(gpu.get_populations(lv)[:, m], ref.get_populations(lv)[:, m])
    gpu.close()
    print(D, model, kind, worst)
    assert max(worst.values()) <= 1e-12, worst


@pytest.mark.parametrize("D,model", [(2, "RR"), (2, "HRR"), (3, "RR"), (3, "HRR")])
def test_nested_fp32_within_bars(D, model):
    lbm = _lbm()
    gpu, ref = _pair(D, model, lbm.LBM_FP32_DEV, "acoustic")
    steps = 40 if D == 2 else 12
    gpu.step(steps)
    ref.step(steps)
    ev = _evolved(ref)
    for lv in (0, 1, 2):
        m = ev[lv]
        r1, u1 = gpu.get_macros(lv)
        r0, u0 = ref.get_macros(lv)
        assert np.abs(r1[m] - r0[m]).max() < 1e-5, lv
        assert np.linalg.norm(u1[:, m] - u0[:, m]) / np.linalg.norm(u0[:, m]) < 1e-4, lv
    gpu.close()


def test_nested_levels_and_refusals():
    lbm = _lbm()
    n, lo, hi, lo2, hi2 = SIZES[2]
    g = lbm.Nested(lbm.LBM_D2Q9, lbm.LBM_RR, lbm.LBM_FP64, (n, n), (lo, lo), (hi, hi), (lo2, lo2), (hi2, hi2))
    assert g.dims(1)[:2] == (2 * (hi - lo) + 1,) * 2
    assert g.dims(2)[:2] == (2 * (hi2 - lo2) + 1,) * 2
    assert g.class_map(2).size == g.nodes(2)
    with pytest.raises(lbm.LbmError):
        g.dims(3)
    for call in (lambda: g.totals(), lambda: g.tune(reps=1), lambda: lbm.lbm_sensors_enable(g.h, True)):
        with pytest.raises(lbm.LbmError):
            call()
    g.close()
    with pytest.raises(lbm.LbmError):  # level-2 patch too close to the level-1 ring
        lbm.Nested(lbm.LBM_D2Q9, lbm.LBM_RR, lbm.LBM_FP64, (n, n), (lo, lo), (hi, hi), (1, 1), (hi2, hi2))
