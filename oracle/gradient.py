"""Gradient of a loss of the density response with respect to the
local-potential amplitudes (oracle, test infrastructure only).

The paper does not treat derivatives; this is the derivation the adjoint
path follows, written out plainly.  With V_loc = sum_a A_a a_a(r) (the
potential is linear in the amplitudes), drho = E^-1 b, E = 1 - chi0 K,
lambda = E^-T dL/d(drho) and u = K drho:

  dL/dA_a = lambda^T (d chi0/dA_a) u + lambda^T chi0 (dK/dA_a) drho
          = sum_r a_a(r) G(r) + sum_r a_a(r) (chi0 s)(r),

  s = (chi0 lambda) * f_x'(rho) * drho   (dK/dA_a = f_x'(rho) chi0 a_a, the
                                          ground state not self-consistent).

The first term is the third derivative of the band energy sum_k w_k
sum_n f e_nk in the directions (a, u, lambda) (rho = (N_g/|Omega|) dE/dV on
the grid), evaluated by the 2n+1 rule with first-order orbitals only
(insulators: equal occupations, parallel-transport gauge):

  E3[x,y,z] = sum over the middle potential y of
              2 Re sum_n f (<psi^x_n, y psi^z_n> - sum_m L^y_mn <psi^x_n, psi^z_m>),
  psi^x_n = -Q (H - e_n)^-1 Q x phi_n,   L^y_mn = <phi_m, y phi_n>.

The terms with psi^a are linear in a through one adjoint Sternheimer
solve per band, eta_n = Q (H - e_n)^-1 Q C_n with
C_n = u psi^l_n + l psi^u_n - sum_m (L^u_mn psi^l_m + L^l_mn psi^u_m), so
that (N_g/|Omega|) E3[a,u,l] = sum_r a(r) G(r) with

  G = sum_k w_k 2 f sum_n [Re(conj psi^u_n psi^l_n)
                           - Re(conj psi_n (eta_n + zeta_n))],
  zeta_n = sum_m <psi^l_m, psi^u_n> phi_m   (all in real space on the right).

Restricted to fixed occupations (no delta f terms).
"""
from __future__ import annotations

from typing import List

import numpy as np

from .groundstate import GroundState
from .response import HxcKernel, chi0_sternheimer, sternheimer_cg
from .system import System


def response_orbitals(sys: System, gs: GroundState, x: np.ndarray, tol: float):
    """psi^x_n = -Q (H - e_n)^-1 Q x phi_n for every occupied (k, n),
    by Sternheimer CG to the absolute tolerance tol * ||x||."""
    xg = x.reshape(sys.n)
    scale = float(np.linalg.norm(xg))
    out = []
    for ik in range(len(sys.bases)):
        nocc = gs.nocc_k[ik]
        phi = gs.phi[ik][:nocc]
        t = sys.to_sphere(ik, xg * sys.to_grid(ik, phi))
        res = np.zeros_like(t)
        for n in range(nocc):
            rhs = -(t[n] - (phi.conj() @ t[n]) @ phi)
            res[n] = sternheimer_cg(sys, gs, ik, n, rhs, tol * max(scale, 1e-300)).x
        out.append(res)
    return out


def third_order_density(sys: System, gs: GroundState, u: np.ndarray,
                        lam: np.ndarray, tol: float) -> np.ndarray:
    """G(r) with sum_r a(r) G(r) = (N_g/|Omega|) E3[a, u, lam] for any a."""
    ug, lg = u.reshape(sys.n), lam.reshape(sys.n)
    psu_all = response_orbitals(sys, gs, ug, tol)
    psl_all = response_orbitals(sys, gs, lg, tol)
    gden = np.zeros(sys.n)
    for ik, kb in enumerate(sys.bases):
        nocc = gs.nocc_k[ik]
        f = gs.occ[ik][:nocc]
        if np.max(np.abs(f - f[0])) > 0:
            raise ValueError("third-order form needs equal occupations")
        phi = gs.phi[ik][:nocc]
        psi = sys.to_grid(ik, phi)
        psu, psl = psu_all[ik], psl_all[ik]
        gu, gl = sys.to_grid(ik, psu), sys.to_grid(ik, psl)
        # L^y_mn = <phi_m, y phi_n>
        tu = sys.to_sphere(ik, ug * psi)
        tl = sys.to_sphere(ik, lg * psi)
        lu = phi.conj() @ tu.T
        ll = phi.conj() @ tl.T
        c = (sys.to_sphere(ik, ug * gl) + sys.to_sphere(ik, lg * gu)
             - lu.T @ psl - ll.T @ psu)
        # eta_n = Q (H - e_n)^-1 Q C_n  (absolute tolerance relative to ||C_n||)
        eta = np.zeros_like(c)
        for n in range(nocc):
            rhs = c[n] - (phi.conj() @ c[n]) @ phi
            eta[n] = sternheimer_cg(sys, gs, ik, n, rhs,
                                    tol * max(np.linalg.norm(rhs), 1e-300)).x
        m = psu.conj() @ psl.T                    # M[n, m] = <psi^u_n, psi^l_m>
        zeta = m.conj() @ phi                     # zeta_n = sum_m conj(M[n,m]) phi_m
        term = np.sum(np.real(gu.conj() * gl), axis=0) - \
            np.sum(np.real(psi.conj() * sys.to_grid(ik, eta + zeta)), axis=0)
        gden += kb.weight * 2.0 * f[0] * term
    return gden


def fx_derivative(rho: np.ndarray) -> np.ndarray:
    """d f_x / d rho for f_x = -(1/3)(3/pi)^{1/3} max(rho, 1e-10)^{-2/3}."""
    return np.where(rho > 1e-10,
                    (2.0 / 9.0) * (3.0 / np.pi) ** (1.0 / 3.0) *
                    np.maximum(rho, 1e-10) ** (-5.0 / 3.0), 0.0)


def amplitude_gradient(sys: System, gs: GroundState, kern: HxcKernel,
                       drho: np.ndarray, lam: np.ndarray, tol: float = 1e-12) -> np.ndarray:
    """dL/dA for every atom, given drho = E^-1 b and lam = E^-T dL/d(drho)."""
    drho = drho.reshape(sys.n)
    lam = lam.reshape(sys.n)
    u = kern.apply(drho)
    gden = third_order_density(sys, gs, u, lam, tol)
    if kern.xc:
        nl = float(np.linalg.norm(lam))
        chil = nl * chi0_sternheimer(sys, gs, lam / nl, tol)
        s = chil * fx_derivative(gs.rho) * drho
        ns = float(np.linalg.norm(s))
        gden = gden + (ns * chi0_sternheimer(sys, gs, s / ns, tol) if ns > 0 else 0.0)
    return np.array([float(np.sum(sys.local_potential_derivative(a) * gden))
                     for a in range(sys.spec.natoms)])
