"""Seeded synthetic inputs (initial macroscopic fields) for the two-level solver.

This module holds no part of the scheme's arithmetic: it only samples the
paper's analytic initial fields on the node coordinates of each level, so the
same inputs can be handed to the HIP library and to the CPU oracle.

* Convected barotropic vortex, eq init_COVO (Sec. 9.3): rho0 = 1, U = 0.1 c_s,
  eps = 0.15 U, R_c = 5 coarse cells.
* Gaussian acoustic pulse, eq init_Pulse (Sec. 8.2), taken radially in 2D/3D
  on top of a uniform mean flow.
* The quasi-one-dimensional cases of Sec. 8: the plane convected shear wave
  of eq init_ShearW and the plane upstream-running acoustic wave of eq
  init_Pulse, both invariant along y.
* Uniform flow.

Coordinates are in coarse lattice units; coarse node (i, j, k) sits at
(i, j, k) and fine node j of a patch whose lower coarse corner is ``lo`` sits
at lo + j/2.  Distances use the minimum image on the periodic coarse box.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

CS = 1.0 / math.sqrt(3.0)
CS2 = 1.0 / 3.0


@dataclass
class Geometry:
    """Two-level periodic geometry: coarse nodes per axis and the fine patch
    as a box [lo, hi] of coarse vertices (ratio 2).  lo == hi: no patch."""

    D: int
    n: tuple
    lo: tuple
    hi: tuple

    @property
    def has_fine(self) -> bool:
        return any(a != b for a, b in zip(self.lo, self.hi))

    def coarse_shape(self):
        return tuple(self.n[: self.D])

    def fine_shape(self):
        return tuple(2 * (h - l) + 1 for l, h in zip(self.lo[: self.D], self.hi[: self.D]))

    def coords(self, level: int):
        """Per-axis coordinate vectors (coarse units) of a level, x first."""
        if level == 0:
            return [np.arange(self.n[d], dtype=np.float64) for d in range(self.D)]
        return [self.lo[d] + 0.5 * np.arange(2 * (self.hi[d] - self.lo[d]) + 1, dtype=np.float64)
                for d in range(self.D)]

    def nodes(self, level: int) -> int:
        return int(np.prod(self.coarse_shape() if level == 0 else self.fine_shape()))

    def updates_per_step(self) -> int:
        """Lattice updates per coarse step: evolving coarse nodes + 2 x fine nodes."""
        nc = int(np.prod(self.coarse_shape()))
        if not self.has_fine:
            return nc
        m = [h - l for l, h in zip(self.lo[: self.D], self.hi[: self.D])]
        covered = int(np.prod([mm - 3 for mm in m]))
        return nc - covered + 2 * self.nodes(1)


def _mesh(geom: Geometry, level: int):
    """Coordinate arrays shaped like the level, flattened x-fastest."""
    cs = geom.coords(level)
    grids = np.meshgrid(*cs, indexing="ij")  # axis 0 = x
    # x fastest in memory: transpose to (z, y, x) then flatten
    return [g.transpose(tuple(range(geom.D))[::-1]).reshape(-1) for g in grids]


def _min_image(dx, L):
    return dx - L * np.round(dx / L)


@dataclass
class Vortex:
    """eq init_COVO parameters (coarse units)."""

    center: tuple
    eps: float
    Rc: float = 5.0
    U: tuple = (0.1 * CS, 0.0, 0.0)
    rho0: float = 1.0


@dataclass
class Pulse:
    """Radial Gaussian density pulse, rho = rho0 (1 + A exp(-r^2 / (2 R^2)))."""

    center: tuple
    A: float
    R: float = 5.0


@dataclass
class ShearWave:
    """Plane shear wave of eq init_ShearW (Sec. 8.1): a transverse velocity
    U_y exp(-(x - x_c)^2 / (2 R^2)) on top of the mean flow, invariant along y."""

    xc: float
    Uy: float = 0.1 * CS
    R: float = 5.0


@dataclass
class PlanePulse:
    """Plane acoustic wave of eq init_Pulse (Sec. 8.2): a density excess
    rho' = rho0 A exp(-(x - x_c)^2 / (2 R^2)) with u_x lowered by
    (rho' / rho0) c_s, the acoustic wave that runs towards -x."""

    xc: float
    A: float = 1e-4
    R: float = 5.0


@dataclass
class Workload:
    geom: Geometry
    U: tuple = (0.0, 0.0, 0.0)
    vortices: list = field(default_factory=list)
    pulses: list = field(default_factory=list)
    rho0: float = 1.0
    shear_waves: list = field(default_factory=list)
    plane_pulses: list = field(default_factory=list)


def fields(wl: Workload, level: int):
    """(rho[N], u[D, N]) of a level, float64, x fastest."""
    g = wl.geom
    X = _mesh(g, level)
    N = X[0].size
    rho = np.full(N, wl.rho0)
    u = np.zeros((g.D, N))
    for d in range(g.D):
        u[d] += wl.U[d]
    for v in wl.vortices:
        dx = _min_image(X[0] - v.center[0], g.n[0])
        dy = _min_image(X[1] - v.center[1], g.n[1])
        r2 = dx * dx + dy * dy
        if g.D == 3:  # a vortex tube along z
            pass
        rho *= np.exp(-(v.eps ** 2) / (2.0 * CS2) * np.exp(-r2 / v.Rc ** 2))
        e = np.exp(-r2 / (2.0 * v.Rc ** 2))
        u[0] += -v.eps * (dy / v.Rc) * e
        u[1] += v.eps * (dx / v.Rc) * e
    for p in wl.pulses:
        r2 = np.zeros(N)
        for d in range(g.D):
            dd = _min_image(X[d] - p.center[d], g.n[d])
            r2 += dd * dd
        rho = rho * (1.0 + p.A * np.exp(-r2 / (2.0 * p.R ** 2)))
    for w in wl.shear_waves:
        dx = _min_image(X[0] - w.xc, g.n[0])
        u[1] += w.Uy * np.exp(-dx * dx / (2.0 * w.R ** 2))
    for p in wl.plane_pulses:
        dx = _min_image(X[0] - p.xc, g.n[0])
        drho = wl.rho0 * p.A * np.exp(-dx * dx / (2.0 * p.R ** 2))
        rho = rho + drho
        u[0] -= drho / wl.rho0 * CS
    return np.ascontiguousarray(rho), np.ascontiguousarray(u)


def uniform_flow(geom: Geometry, U=(0.1 * CS, 0.0, 0.0), rho0: float = 1.0) -> Workload:
    return Workload(geom=geom, U=U, rho0=rho0)


# --------------------------------------------------------------------------
# The benchmark workloads (sizes as stated for this hot path).

def vortex_crossing_64(seed: int = 0) -> Workload:
    """D2Q9 periodic 64^2, patch [16,48]^2 (64^2 fine cells), vortex crossing
    the x = 48 edge from fine to coarse."""
    rng = np.random.Generator(np.random.PCG64(seed))
    geom = Geometry(2, (64, 64, 1), (16, 16, 0), (48, 48, 0))
    s = rng.uniform(0.5, 1.5)
    dx, dy = rng.uniform(-1.0, 1.0, size=2)
    U = 0.1 * CS
    v = Vortex(center=(42.0 + dx, 32.0 + dy), eps=0.15 * U * s, U=(U, 0.0, 0.0))
    return Workload(geom=geom, U=(U, 0.0, 0.0), vortices=[v])


def vortex_pulse_4096(seed: int = 0, n: int = 4096) -> Workload:
    """D2Q9 periodic 4096^2, fine band 4096 x 2048 fine cells (patch
    [n/4, 3n/4] x [3n/8, 5n/8]), vortex near the right patch edge plus a
    Gaussian pulse (A = 1e-3) within 200 coarse cells of the interface."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lo = (n // 4, 3 * n // 8, 0)
    hi = (3 * n // 4, 5 * n // 8, 0)
    geom = Geometry(2, (n, n, 1), lo, hi)
    U = 0.1 * CS
    s = rng.uniform(0.5, 1.5)
    v = Vortex(center=(hi[0] - 6.0, 0.5 * (lo[1] + hi[1]) + rng.uniform(-1, 1)), eps=0.15 * U * s,
               U=(U, 0.0, 0.0))
    off = min(200.0, 0.2 * n)
    pc = (hi[0] + rng.uniform(-off, off), lo[1] + rng.uniform(-off, off))
    return Workload(geom=geom, U=(U, 0.0, 0.0), vortices=[v], pulses=[Pulse(center=pc, A=1e-3)])


def pulse_cube_384(seed: int = 0, n: int = 384) -> Workload:
    """D3Q19 periodic n^3, centred fine cube of n^3 fine cells (patch
    [n/4, 3n/4]^3), Gaussian pulse (A = 1e-3) near the interface plus a
    uniform flow at Mach 0.1 along x."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lo = (n // 4,) * 3
    hi = (3 * n // 4,) * 3
    geom = Geometry(3, (n, n, n), lo, hi)
    U = 0.1 * CS
    off = min(10.0, 0.05 * n)
    pc = tuple(float(hi[0]) + rng.uniform(-off, off) if d == 0 else 0.5 * n + rng.uniform(-off, off)
               for d in range(3))
    return Workload(geom=geom, U=(U, 0.0, 0.0), pulses=[Pulse(center=pc, A=1e-3)])


# --------------------------------------------------------------------------
# The quasi-one-dimensional cases of Sec. 8.  The paper runs them one coarse
# cell thick with non-reflecting ends; here the box is periodic and a fine
# band spans the x range of the paper's fine region, `height` coarse cells
# along y (its y edges are interfaces as well).  Nodes farther from those
# edges than the edges' influence has travelled hold the y-invariant
# solution of the paper's one-dimensional case.  Coordinates of the paper's
# set-up are shifted by `shift` along x.

def shear_wave_case(height: int = 256, left: int = 350, right: int = 550, U: float = 0.1 * CS) -> Workload:
    """Eqs init_ShearW / init_ShearW2: rho0 = 1, U_x = U_y = 0.1 c_s, R_c = 5,
    x_c = 150; fine for x < 250 (from -left), coarse beyond (to 250 + right)."""
    shift = left + 50
    n = (shift + 250 + right, height + 10, 1)
    lo = (shift - left, 5, 0)
    hi = (shift + 250, 5 + height, 0)
    geom = Geometry(2, n, lo, hi)
    return Workload(geom=geom, U=(U, 0.0, 0.0), shear_waves=[ShearWave(xc=shift + 150.0, Uy=U)])


def acoustic_wave_case(height: int = 256, left: int = 900, right: int = 400, A: float = 1e-4,
                       U: float = 0.1 * CS) -> Workload:
    """Eqs init_Pulse / init_Pulse2: rho0 = 1, U_x = 0.1 c_s, A = 1e-4,
    R_c = 5, x_c = 750; fine for 500 < x < 1000, coarse below 500 (from
    500 - left) and above 1000 (to 1000 + right)."""
    shift = left - 500
    n = (shift + 1000 + right, height + 10, 1)
    lo = (shift + 500, 5, 0)
    hi = (shift + 1000, 5 + height, 0)
    geom = Geometry(2, n, lo, hi)
    return Workload(geom=geom, U=(U, 0.0, 0.0), plane_pulses=[PlanePulse(xc=shift + 750.0, A=A)])


def batch_instance(seed: int, i: int) -> Workload:
    """One instance of the batched workload: D2Q9, side N = 4 round(exp(U[ln 64,
    ln 1024]) / 4), patch [N/4, 3N/4]^2 (25 % of the area), one vortex at a
    uniform position in the patch with eps = 0.15 U s, s ~ U[0.5, 1.5]."""
    rng = np.random.Generator(np.random.PCG64([seed, i]))
    N = int(4 * round(math.exp(rng.uniform(math.log(64), math.log(1024))) / 4))
    lo = (N // 4, N // 4, 0)
    hi = (3 * N // 4, 3 * N // 4, 0)
    geom = Geometry(2, (N, N, 1), lo, hi)
    U = 0.1 * CS
    c = (rng.uniform(lo[0], hi[0]), rng.uniform(lo[1], hi[1]))
    v = Vortex(center=c, eps=0.15 * U * rng.uniform(0.5, 1.5), U=(U, 0.0, 0.0))
    return Workload(geom=geom, U=(U, 0.0, 0.0), vortices=[v])


def scaled(wl_fn, n: int, seed: int = 0) -> Workload:
    """A configuration generator evaluated at a smaller side length."""
    return wl_fn(seed=seed, n=n)
