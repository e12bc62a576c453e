"""Von Neumann (linear stability) analysis of the LBM schemes, Sec. 5 and
Appendix A of arXiv:2004.11863.

TEST INFRASTRUCTURE ONLY (it pins the oracle's time stepping through
plane-wave runs; the product path never uses it).

The update is linearised about a uniform equilibrium f_bar = f0(rho_bar,
u_bar) (eqs lsa_f, lsa_PhiLin): f'(x + xi_i, t + 1) = J f'(x, t).  With plane
waves f' = F exp(i(omega t - k.x)) (eq LSA_monowaves) this becomes the
eigenproblem exp(i omega) F = M F, M = diag(exp(i k.xi_i)) J (eq
LSA_eigenvalue).  omega_r = arg(lambda) is the dispersion, omega_i =
-ln|lambda| the dissipation.

Everything here is written with NumPy from the definitions in Sec. 3 and
Appendix A; it does not call the C oracle.  The derivatives of the
equilibrium are taken by complex-step differentiation, which is exact to
rounding for this polynomial-and-division map.
"""
from __future__ import annotations

import math

import numpy as np

CS2 = 1.0 / 3.0


def lattice(name: str):
    """Velocities and weights.  D2Q9 in the order of eqs xi_i and w_i;
    D3Q19 standard (rest, 6 axis, 12 face diagonals)."""
    if name == "D2Q9":
        xi = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]], float)
        w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    elif name == "D3Q19":
        v = [[0, 0, 0]]
        for d in range(3):
            for s in (1, -1):
                e = [0, 0, 0]
                e[d] = s
                v.append(e)
        for a, b in ((0, 1), (0, 2), (1, 2)):
            for sa, sb in ((1, 1), (-1, -1), (1, -1), (-1, 1)):
                e = [0, 0, 0]
                e[a], e[b] = sa, sb
                v.append(e)
        xi = np.array(v, float)
        w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    else:
        raise ValueError(name)
    return xi, w


def _hermite2(xi):
    D = xi.shape[1]
    return np.einsum("ia,ib->iab", xi, xi) - CS2 * np.eye(D)[None]


def _hermite3(xi):
    D = xi.shape[1]
    I = np.eye(D)
    H = np.einsum("ia,ib,ic->iabc", xi, xi, xi)
    H = H - CS2 * (np.einsum("ia,bc->iabc", xi, I) + np.einsum("ib,ac->iabc", xi, I)
                   + np.einsum("ic,ab->iabc", xi, I))
    return H


def third_order_basis(xi, w):
    """Third-order polynomials the lattice supports, orthogonalised in the
    lattice inner product: D2Q9 -> H_xxy, H_xyy; D3Q19 -> H_xxy +/- H_yzz,
    H_xzz +/- H_xyy, H_yyz +/- H_xxz.  Returns (P[i, p], coefficient tensors
    C[p, a, b, c] such that a_P = sum C a_abc)."""
    D = xi.shape[1]
    H3 = _hermite3(xi)
    combos = []
    if D == 2:
        combos = [[((0, 0, 1), 1.0)], [((0, 1, 1), 1.0)]]
    else:
        pairs = [((0, 0, 1), (1, 2, 2)), ((0, 2, 2), (0, 1, 1)), ((1, 1, 2), (0, 0, 2))]
        for s in (1.0, -1.0):
            for p, q in pairs:
                combos.append([(p, 1.0), (q, s)])
    P = np.zeros((xi.shape[0], len(combos)))
    C = np.zeros((len(combos), D, D, D))
    for k, cb in enumerate(combos):
        for idx, sgn in cb:
            P[:, k] += sgn * H3[(slice(None),) + idx]
            C[(k,) + idx] += sgn
    return P, C


class Scheme:
    """Linearised LBM operator for a lattice and collision model."""

    def __init__(self, lat: str, model: str, tau: float, sigma: float = 0.995):
        self.xi, self.w = lattice(lat)
        self.Q, self.D = self.xi.shape
        self.model, self.tau, self.sigma = model, tau, sigma
        self.H2 = _hermite2(self.xi)
        self.P, self.C = third_order_basis(self.xi, self.w)
        self.PN = (self.w[:, None] * self.P ** 2).sum(0)

    # equilibrium (eq fEqH truncated at third order), complex-safe
    def feq(self, rho, u):
        u = np.asarray(u)
        a2 = rho * np.outer(u, u)
        a3 = rho * np.einsum("a,b,c->abc", u, u, u)
        aP = np.einsum("pabc,abc->p", self.C, a3)
        t1 = self.xi @ (rho * u)
        t2 = np.einsum("iab,ab->i", self.H2, a2)
        t3 = (self.P * (aP / self.PN)[None]).sum(1)
        return self.w * (rho + t1 / CS2 + t2 / (2 * CS2 ** 2) + t3)

    def jacobian(self, rho, u, k):
        """J(k) of eqs lsa_PhiLin / lsa_PhiRR; k enters only through the
        finite-difference strain rate of H-RR."""
        Q, D = self.Q, self.D
        u = np.asarray(u, float)
        h = 1e-30
        dfe_drho = (self.feq(rho + 1j * h, u.astype(complex))).imag / h
        dfe_du = np.zeros((Q, D))
        for d in range(D):
            uc = u.astype(complex)
            uc[d] += 1j * h
            dfe_du[:, d] = self.feq(complex(rho), uc).imag / h
        # rho' = sum f', u' = (sum xi f' - u sum f') / rho   (eq lsa_uprime)
        drho = np.ones((1, Q))
        du = (self.xi.T - u[:, None] * np.ones((1, Q))) / rho
        F0 = dfe_drho[:, None] * drho + dfe_du @ du  # d f0 / d f'
        I = np.eye(Q)
        om = 1.0 - 1.0 / self.tau
        if self.model == "BGK":
            return F0 + om * (I - F0)
        # a1^(2)' = sum_i H2_i (f' - f0')   (eq a1Proj)
        A2 = np.einsum("iab,ij->abj", self.H2, I - F0)  # [a, b, j]
        if self.model == "HRR":
            # centred differences: d/dx_a <-> -i sin k_a for exp(-i k.x)
            sk = np.sin(np.asarray(k, float))
            G = -1j * sk[:, None, None] * du[None, :, :]  # G[a, b, j] = d_a u_b
            S = 0.5 * (G + G.transpose(1, 0, 2))
            A2 = self.sigma * A2 + (1.0 - self.sigma) * (-2.0 * self.tau * rho * CS2 * S)
        # third order with the mean velocity (eq lsa_a13)
        A3 = (np.einsum("a,bcj->abcj", u, A2) + np.einsum("b,acj->abcj", u, A2)
              + np.einsum("c,abj->abcj", u, A2))
        AP = np.einsum("pabc,abcj->pj", self.C, A3)
        F1 = self.w[:, None] * (np.einsum("iab,abj->ij", self.H2, A2) / (2 * CS2 ** 2)
                                + (self.P / self.PN[None]) @ AP)
        return F0 + om * F1

    def matrix(self, rho, u, k):
        k = np.asarray(k, float)
        return np.diag(np.exp(1j * (self.xi @ k))) @ self.jacobian(rho, u, k)

    def eig(self, rho, u, k):
        lam, V = np.linalg.eig(self.matrix(rho, u, k))
        return lam, V


def omega(lam):
    """(omega_r, omega_i) from lambda = exp(i omega)."""
    return np.angle(lam), -np.log(np.abs(lam))


def macro_content(scheme: Scheme, V):
    """Moments (rho_hat, (rho u)_hat) of each eigenvector (eq momentsF)."""
    return np.vstack([V.sum(0)[None], scheme.xi.T @ V])


def ns_eigenvalues(k, u, nu):
    """Isothermal Navier-Stokes modes, eq eigenvaluesNS (shear, ac+, ac-)."""
    k = np.asarray(k, float)
    kn = np.linalg.norm(k)
    ku = float(k @ np.asarray(u, float))
    cs = math.sqrt(CS2)
    return np.array([ku + 1j * nu * kn ** 2, ku + kn * cs + 1j * nu * kn ** 2, ku - kn * cs + 1j * nu * kn ** 2])
