"""Helpers that run the same seeded workload through the HIP library (via
the C ABI binding) and through the CPU oracle."""
from __future__ import annotations

import numpy as np

import oracle as O
from paper_2004_11863_amd import inputs as I

MODELS = {"BGK": (0, O.BGK), "RR": (1, O.RR), "HRR": (2, O.HRR)}


def lat_ids(D):
    from paper_2004_11863_amd import lbm
    return (lbm.LBM_D2Q9, O.D2Q9) if D == 2 else (lbm.LBM_D3Q19, O.D3Q19)


def make_pair(wl: I.Workload, model: str, precision: int, tau_c=0.51, sigma=0.995, with_oracle=True):
    from paper_2004_11863_amd import lbm
    g = wl.geom
    D = g.D
    lg, lo_ = lat_ids(D)
    mg, mo = MODELS[model]
    lo = g.lo[:D] if g.has_fine else None
    hi = g.hi[:D] if g.has_fine else None
    gpu = lbm.Grid(lg, mg, precision, g.n[:D], lo, hi, tau_coarse=tau_c, sigma=sigma)
    ref = O.Grid(lo_, mo, g.n[:D], lo, hi, tau_c=tau_c, sigma=sigma) if with_oracle else None
    levels = (0, 1) if g.has_fine else (0,)
    for lv in levels:
        rho, u = I.fields(wl, lv)
        gpu.set_state(lv, rho, u)
        if ref is not None:
            ref.set_state(lv, rho, u)
    return gpu, ref, levels


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def compare_fp64(gpu, ref, levels):
    """Largest relative deviation over rho, u and populations of all levels."""
    worst = {}
    for lv in levels:
        r1, u1 = gpu.get_macros(lv)
        r0, u0 = ref.get_macros(lv)
        worst[f"rho{lv}"] = rel(r1, r0)
        worst[f"u{lv}"] = rel(u1, u0)
        if lv == 0:
            cls = ref.class_map(0)
            m = cls != O.C_COVERED
            worst["f0"] = rel(gpu.get_populations(0)[:, m], ref.get_populations(0)[:, m])
        else:
            worst["f1"] = rel(gpu.get_populations(1), ref.get_populations(1))
    return worst


def compare_fp32(gpu, ref, levels):
    """Density max-abs error and velocity relative L2 error over all levels."""
    out = {}
    for lv in levels:
        r1, u1 = gpu.get_macros(lv)
        r0, u0 = ref.get_macros(lv)
        out[f"rho_maxabs{lv}"] = float(np.abs(r1 - r0).max())
        out[f"u_relL2{lv}"] = float(np.linalg.norm(u1 - u0) / np.linalg.norm(u0))
    return out
