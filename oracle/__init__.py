"""FP64 CPU oracle of the two-level lattice-Boltzmann scheme.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use it; the product library never imports, links or calls
anything here.  The arithmetic lives in ``lbm_oracle.c`` (plain C, double
precision, no fast-math, contraction off); this module only marshals arrays.

Paper: Astoul et al., "Analysis and reduction of spurious noise generated at
grid refinement interfaces with the lattice Boltzmann method",
arXiv:2004.11863 -- Sec. 3 (lattice, equilibrium, BGK/RR/H-RR collisions),
Sec. 4 (level rescaling, filter, interpolations, two-level schedule).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

D2Q9, D3Q19 = 0, 1
BGK, RR, HRR = 0, 1, 2

# coarse node classes / fine node classes (Fig. Overlap)
C_MIDDLE, C_TFC, C_TNC, C_COVERED = 0, 1, 2, 3
F_MIDDLE, F_TFF, F_IE, F_IEFACE, F_TNF = 0, 1, 2, 3, 4

MUTATIONS = {
    "rescale_swap": 1,
    "temporal_rev": 2,
    "spatial_lin": 3,
    "filter_swap": 4,
    "fd_sign": 5,
    "no_third": 6,
    "sigma_swap": 7,
    "stream_push": 8,
    "sc_half": 9,
    "tauf": 10,
    "feq2": 11,
    "nofilter": 12,
    "filter_zoff": 13,
    "face_axes": 14,
    "nest_sync": 15,
    "nest_ring": 16,
    "nest_inj": 17,
}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
             "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        vp = ctypes.c_void_p
        L.orc_create.restype = vp
        L.orc_create.argtypes = [ctypes.c_int, ctypes.c_int, ip, ip, ip, ctypes.c_double, ctypes.c_double]
        L.orc_create_nested.restype = vp
        L.orc_create_nested.argtypes = [ctypes.c_int, ctypes.c_int, ip, ip, ip, ip, ip, ctypes.c_double,
                                        ctypes.c_double]
        L.orc_child.restype = vp
        L.orc_child.argtypes = [vp]
        L.orc_destroy.argtypes = [vp]
        for name in ("orc_set_state", "orc_get_macros"):
            getattr(L, name).argtypes = [vp, ctypes.c_int, dp, dp]
        for name in ("orc_set_populations", "orc_get_populations"):
            getattr(L, name).argtypes = [vp, ctypes.c_int, dp]
        L.orc_step.argtypes = [vp, ctypes.c_int]
        L.orc_class_map.argtypes = [vp, ctypes.c_int, ctypes.c_void_p]
        L.orc_level_dims.argtypes = [vp, ctypes.c_int, ip]
        L.orc_count.argtypes = [vp, ctypes.c_int]
        L.orc_count.restype = ctypes.c_long
        L.orc_history_nodes.argtypes = [vp, ctypes.c_void_p]
        L.orc_ring_stencils.argtypes = [vp, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.orc_totals.argtypes = [vp, dp, dp]
        L.orc_feq.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp]
        L.orc_collide.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, dp, dp]
        L.orc_lattice_info.argtypes = [ctypes.c_int, ip, ip, ip, dp]
        L.orc_temporal_weights.argtypes = [ctypes.c_int, dp]
        L.orc_temporal_interp.argtypes = [ctypes.c_double] * 3
        L.orc_temporal_interp.restype = ctypes.c_double
        L.orc_cubic_mid.argtypes = [dp]
        L.orc_cubic_mid.restype = ctypes.c_double
        L.orc_filter_weight.argtypes = [ctypes.c_int, ip]
        L.orc_filter_weight.restype = ctypes.c_double
        for name in ("orc_rescale_c2f", "orc_rescale_f2c"):
            getattr(L, name).argtypes = [ctypes.c_double, ctypes.c_double]
            getattr(L, name).restype = ctypes.c_double
        L.orc_tau_fine.argtypes = [ctypes.c_double]
        L.orc_tau_fine.restype = ctypes.c_double
        L.orc_strain_f2c.restype = ctypes.c_double
        L.orc_set_mutation.argtypes = [ctypes.c_int]
        L.orc_threads.restype = ctypes.c_int
        L.orc_sensors.argtypes = [vp, ctypes.c_int, ctypes.c_double, vp, vp, vp, vp]
        L.orc_set_dynamic_sigma.argtypes = [vp, ctypes.c_int, ctypes.c_double, ctypes.c_double]
        L.orc_dynamic_mask.argtypes = [vp, ctypes.c_int, vp]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def set_mutation(name: str | None) -> None:
    """Plant one of a list of plausible mistakes (tests of the pins only)."""
    lib().orc_set_mutation(0 if name is None else MUTATIONS[name])


def threads() -> int:
    return int(lib().orc_threads())


def lattice(lat: int):
    """(D, Q, xi[Q,3] int, w[Q]) of the oracle's lattice table."""
    D = np.zeros(1, np.int32)
    Q = np.zeros(1, np.int32)
    xi = np.zeros(19 * 3, np.int32)
    w = np.zeros(19)
    lib().orc_lattice_info(lat, _ip(D), _ip(Q), _ip(xi), _dp(w))
    q = int(Q[0])
    return int(D[0]), q, xi[: 3 * q].reshape(q, 3).copy(), w[:q].copy()


def feq(lat: int, rho: float, u) -> np.ndarray:
    _, Q, _, _ = lattice(lat)
    uu = np.zeros(3)
    uu[: len(u)] = u
    out = np.zeros(Q)
    lib().orc_feq(lat, float(rho), _dp(uu), _dp(out))
    return out


def collide(lat: int, model: int, tau: float, sigma: float, f, S=None) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros_like(f)
    Sm = np.zeros(9) if S is None else np.ascontiguousarray(np.asarray(S, dtype=np.float64).reshape(9))
    lib().orc_collide(lat, model, float(tau), float(sigma), _dp(f), _dp(Sm), _dp(out))
    return out


def temporal_weights(half: bool = True) -> np.ndarray:
    c = np.zeros(3)
    lib().orc_temporal_weights(1 if half else 0, _dp(c))
    return c


def temporal_interp(gm1: float, g0: float, gp1: float) -> float:
    return float(lib().orc_temporal_interp(gm1, g0, gp1))


def cubic_mid(g) -> float:
    g = np.ascontiguousarray(g, dtype=np.float64)
    return float(lib().orc_cubic_mid(_dp(g)))


def filter_weight(D: int, o) -> float:
    oo = np.zeros(3, np.int32)
    oo[: len(o)] = o
    return float(lib().orc_filter_weight(D, _ip(oo)))


def tau_fine(tau_c: float) -> float:
    return float(lib().orc_tau_fine(tau_c))


def rescale_c2f(tau_c: float, tau_f: float) -> float:
    return float(lib().orc_rescale_c2f(tau_c, tau_f))


def rescale_f2c(tau_c: float, tau_f: float) -> float:
    return float(lib().orc_rescale_f2c(tau_c, tau_f))


def strain_f2c() -> float:
    return float(lib().orc_strain_f2c())


class Grid:
    """Two-level (or, with lo == hi, uniform periodic) grid of the oracle.

    lattice: D2Q9 or D3Q19; model: BGK, RR or HRR; n: coarse nodes per axis;
    lo, hi: fine patch as a box of coarse vertices (ratio 2).
    """

    def __init__(self, lattice_id, model, n, lo=None, hi=None, tau_c=0.51, sigma=0.995):
        D, Q, xi, w = lattice(lattice_id)
        self.D, self.Q, self.xi, self.w = D, Q, xi, w
        self.lattice_id, self.model = lattice_id, model
        nn = np.ones(3, np.int32)
        nn[:D] = n
        lo_ = np.zeros(3, np.int32)
        hi_ = np.zeros(3, np.int32)
        if lo is not None:
            lo_[:D] = lo
            hi_[:D] = hi
        self.n = nn
        self.lo, self.hi = lo_, hi_
        self.has_fine = lo is not None and any(int(a) != int(b) for a, b in zip(lo, hi))
        self.tau_c, self.sigma = tau_c, sigma
        self._h = lib().orc_create(lattice_id, model, _ip(nn), _ip(lo_), _ip(hi_), float(tau_c), float(sigma))
        if not self._h:
            raise ValueError("oracle rejected the grid description")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    def dims(self, level: int):
        d = np.zeros(3, np.int32)
        if lib().orc_level_dims(self._h, level, _ip(d)) != 0:
            raise ValueError("no such level")
        return tuple(int(x) for x in d)

    def nodes(self, level: int) -> int:
        a, b, c = self.dims(level)
        return a * b * c

    def set_state(self, level: int, rho, u):
        N = self.nodes(level)
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(N)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(self.D, N)
        if lib().orc_set_state(self._h, level, _dp(rho), _dp(u)) != 0:
            raise ValueError("set_state failed")

    def set_populations(self, level: int, f):
        N = self.nodes(level)
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(self.Q, N)
        if lib().orc_set_populations(self._h, level, _dp(f)) != 0:
            raise ValueError("set_populations failed")

    def get_populations(self, level: int) -> np.ndarray:
        N = self.nodes(level)
        f = np.zeros((self.Q, N))
        if lib().orc_get_populations(self._h, level, _dp(f)) != 0:
            raise ValueError("get_populations failed")
        return f

    def get_macros(self, level: int):
        N = self.nodes(level)
        rho = np.zeros(N)
        u = np.zeros((self.D, N))
        if lib().orc_get_macros(self._h, level, _dp(rho), _dp(u)) != 0:
            raise ValueError("get_macros failed")
        return rho, u

    def step(self, n: int = 1):
        lib().orc_step(self._h, int(n))

    def class_map(self, level: int) -> np.ndarray:
        out = np.zeros(self.nodes(level), np.uint8)
        if lib().orc_class_map(self._h, level, out.ctypes.data) != 0:
            raise ValueError("no such level")
        return out

    def counts(self):
        L = lib()
        return {"history": int(L.orc_count(self._h, 0)), "ring": int(L.orc_count(self._h, 1)),
                "tn": int(L.orc_count(self._h, 2))}

    def history_nodes(self) -> np.ndarray:
        n = self.counts()["history"]
        out = np.zeros(n, np.int64)
        lib().orc_history_nodes(self._h, out.ctypes.data)
        return out

    def ring_stencils(self):
        n = self.counts()["ring"]
        node = np.zeros(n, np.int64)
        np_ = np.zeros(n, np.int32)
        pts = np.zeros((n, 16), np.int64)
        w = np.zeros((n, 16))
        lib().orc_ring_stencils(self._h, node.ctypes.data, np_.ctypes.data, pts.ctypes.data, w.ctypes.data)
        return node, np_, pts, w

    def sensors(self, level: int, thr: float):
        """NH-sensor flags of a level's last iteration (bit 0 SpuriousAc, bit 1
        SpuriousS, bit 2 SpuriousG; Sec. 7) and the quantities they test: the
        divergence product, the curl product and the norm of the ghost part
        of the non-equilibrium populations."""
        N = self.nodes(level)
        flags = np.zeros(N, np.uint8)
        dp, cp, gn = np.zeros(N), np.zeros(N), np.zeros(N)
        rc = lib().orc_sensors(self._h, level, float(thr), flags.ctypes.data, dp.ctypes.data, cp.ctypes.data,
                               gn.ctypes.data)
        if rc != 0:
            raise ValueError("sensors need a level that exists and a step taken")
        return flags, dp, cp, gn

    def set_dynamic_sigma(self, on: bool, sigma_dyn: float = 0.0, threshold: float = 0.0):
        """H-RR with sigma chosen per node from the SpuriousAc / SpuriousS tests
        between consecutive bulk collisions (sigma_dyn where a product falls
        below -threshold, the grid's sigma elsewhere); a variant Sec. 9.3 and
        Sec. 11 suggest."""
        if lib().orc_set_dynamic_sigma(self._h, 1 if on else 0, float(sigma_dyn), float(threshold)) != 0:
            raise ValueError("dynamic sigma needs H-RR, sigma_dyn in [0, 1] and a threshold >= 0")

    def dynamic_mask(self, level: int):
        """1 on the nodes of a level whose last bulk collision took sigma_dyn."""
        out = np.zeros(self.nodes(level), np.uint8)
        if lib().orc_dynamic_mask(self._h, level, out.ctypes.data) != 0:
            raise ValueError("no such level")
        return out

    def totals(self):
        mass = np.zeros(2)
        mom = np.zeros(6)
        lib().orc_totals(self._h, _dp(mass), _dp(mom))
        return mass, mom.reshape(2, 3)


class _View(Grid):
    """The child pair of a nested grid (owned by its root: never destroyed
    here)."""

    def __init__(self, handle, lattice_id, model, n, lo, hi, tau_c, sigma):
        D, Q, xi, w = lattice(lattice_id)
        self.D, self.Q, self.xi, self.w = D, Q, xi, w
        self.lattice_id, self.model = lattice_id, model
        nn = np.ones(3, np.int32)
        nn[:D] = n
        self.n = nn
        self.lo, self.hi = np.zeros(3, np.int32), np.zeros(3, np.int32)
        self.lo[:D], self.hi[:D] = lo, hi
        self.has_fine = True
        self.tau_c, self.sigma = tau_c, sigma
        self._h = handle

    def __del__(self):
        self._h = None


class Nested:
    """Three nested levels: level 0 the periodic coarse grid, level 1 the
    patch [lo, hi] of coarse vertices, level 2 the patch [lo2, hi2] of level-1
    vertices (ratio 2 at each interface).  The two-level step of Sec. 4.3
    applied to each pair: every substep of level 1 is a whole step of the
    pair (1, 2), which receives the level-1 ring's rho and u at its time.
    BGK, RR and H-RR."""

    def __init__(self, lattice_id, model, n, lo, hi, lo2, hi2, tau_c=0.51, sigma=0.995):
        D, Q, xi, w = lattice(lattice_id)
        self.D, self.Q = D, Q
        self.lattice_id, self.model = lattice_id, model
        a = [np.zeros(3, np.int32) for _ in range(5)]
        a[0][:] = 1
        for arr, v in zip(a, (n, lo, hi, lo2, hi2)):
            arr[:D] = v
        self._h = lib().orc_create_nested(lattice_id, model, _ip(a[0]), _ip(a[1]), _ip(a[2]), _ip(a[3]), _ip(a[4]),
                                          float(tau_c), float(sigma))
        if not self._h:
            raise ValueError("oracle rejected the nested grid description")
        self.root = _View(self._h, lattice_id, model, n, lo, hi, tau_c, sigma)
        nf = [2 * (int(h) - int(l)) + 1 for l, h in zip(lo, hi)]
        self.child = _View(lib().orc_child(self._h), lattice_id, model, nf, lo2, hi2, 2 * tau_c - 0.5, sigma)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    def _at(self, level):
        return {0: (self.root, 0), 1: (self.root, 1), 2: (self.child, 1)}[level]

    def nodes(self, level):
        g, lv = self._at(level)
        return g.nodes(lv)

    def dims(self, level):
        g, lv = self._at(level)
        return g.dims(lv)

    def set_state(self, level, rho, u):
        g, lv = self._at(level)
        g.set_state(lv, rho, u)
        if level == 1:
            self.child.set_state(0, rho, u)

    def step(self, n=1):
        lib().orc_step(self._h, int(n))

    def get_populations(self, level):
        g, lv = self._at(level)
        return g.get_populations(lv)

    def class_map(self, level):
        g, lv = self._at(level)
        return g.class_map(lv)

    def get_macros(self, level):
        """Moments of the current state; nodes a finer level covers take the
        values of its co-located node (output only)."""
        if level == 2:
            return self.child.get_macros(1)
        if level == 1:
            r, u = self.child.get_macros(0)
            ring = np.isin(self.root.class_map(1), [F_TFF, F_IE, F_IEFACE])
            rr, ur = self.root.get_macros(1)
            r[ring], u[:, ring] = rr[ring], ur[:, ring]
            return r, u
        r, u = self.root.get_macros(0)
        cov = self.root.class_map(0) == C_COVERED
        if cov.any():
            r1, u1 = self.get_macros(1)
            nf = self.root.dims(1)
            idx = np.nonzero(cov)[0]
            n = self.root.n
            c = [(idx // int(np.prod(n[:d]))) % n[d] for d in range(self.D)]
            j = [2 * (c[d] - self.root.lo[d]) for d in range(self.D)]
            fi = sum(j[d] * int(np.prod(nf[:d])) for d in range(self.D))
            r[idx], u[:, idx] = r1[fi], u1[:, fi]
        return r, u
