"""Atom-displacement perturbation (oracle, test infrastructure only).

The paper's test problems perturb the ground state by displacing atoms
(Sec. 4.1.2, "Implementation and computational setup"): the perturbing
potential dV0 is the derivative of the external potential with respect to
an atomic position, and the right-hand side of the Dyson equation
(eq. dyson_discretised) is chi0 dV0.  For the model here both parts of the
pseudopotential move with atom a:

  * local part: dV_loc / dR_a,beta has Fourier coefficients
    (-i G_beta) (1/|Omega|) (-A_a) exp(-s^2 |G|^2 / 2) exp(-i G.R_a) on the
    FFT cube (the derivative of the local-potential coefficients of the
    system module); on the grid it is the real part of their inverse sum;
  * nonlocal part: p_a(q) carries exp(-i q.R_a), so dp_a/dR_a,beta =
    -i q_beta p_a(q) (q = G + k) and
    dV_nl = D (|dp_a><p_a| + |p_a><dp_a|).

drho0 = chi0 dV0 is formed three independent ways: by the sum over states
with the nonlocal matrix elements added to M_mn, by the Sternheimer route
with dV_nl phi_n added to the right-hand sides, and by a central finite
difference of the density in the atom's position (the ground state
recomputed by dense diagonalisation; the model's potential is fixed, not
self-consistent, so d rho / dR = chi0 dV0 exactly).
"""
from __future__ import annotations

import numpy as np

from .groundstate import ground_state
from .system import System


def local_potential_derivative_position(sys: System, atom: int, direction: int) -> np.ndarray:
    """dV_loc / dR_{atom, direction} on the real-space grid."""
    spec = sys.spec
    g = sys.cube_g()
    gg = g[0] ** 2 + g[1] ** 2 + g[2] ** 2
    r = sys.pos[atom]
    phase = np.exp(-1j * (g[0] * r[0] + g[1] * r[1] + g[2] * r[2]))
    vt = (-1j * g[direction]) * (-spec.amp[atom]) * \
        np.exp(-spec.sigma_loc ** 2 * gg / 2.0) * phase / sys.volume
    return np.ascontiguousarray((np.fft.ifftn(vt) * sys.ng).real)


def projector_pair(sys: System, ik: int, atom: int, direction: int):
    """(p_a, dp_a / dR_{a,direction}) on the sphere of k-point ik."""
    p = sys.projectors(ik)[atom]
    q = sys.bases[ik].q[:, direction]
    return p, -1j * q * p


def nonlocal_action(sys: System, atom: int, direction: int):
    """dv_nl(ik, coeffs) -> dV_nl applied to coefficient rows [n, nb]."""
    d = sys.spec.d_proj

    def act(ik, c):
        p, dp = projector_pair(sys, ik, atom, direction)
        return d * (np.outer(c @ p.conj(), dp) + np.outer(c @ dp.conj(), p))
    return act


def density_fd(spec, atom: int, direction: int, h: float = 1e-4) -> np.ndarray:
    """Central difference of the ground-state density in R_{atom,direction}
    (dense eigenpairs, occupations and Fermi level recomputed at R +- h)."""
    rhos = []
    for sgn in (1.0, -1.0):
        pos = np.array(spec.frac_pos, float)
        pos[atom, direction] += sgn * h / spec.lattice[direction]
        sys = System(spec.with_(frac_pos=pos))
        rhos.append(ground_state(sys, dense=True).rho)
    return (rhos[0] - rhos[1]) / (2.0 * h)
