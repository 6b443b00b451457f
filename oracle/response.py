"""Independent-particle response, Hxc kernel and dielectric adjoint
(oracle, test infrastructure only).

Three independent routes to chi0 (Sec. 2.2):
  * ``chi0_sos``      : plain sum over all eigenpairs of the dense H_k
                        (the Adler-Wiser form implied by eq. chi0 and
                        eq. delta_phi_P with the exact orbital response);
  * ``chi0_fd``       : central finite difference of the potential-to-density
                        map F_KS (eq. potdensmap), chi0 = F_KS';
  * ``Sternheimer``   : the method itself -- eq. delta_phi_P for the occupied
                        part, preconditioned CG on eq. sternheimer_equation
                        for the unoccupied part, eq. delta_f for occupations,
                        accumulated as in eq. kchi0.

Readings (paper silent / inconsistent):
  * delta_phi_P coefficient: the printed f_n^2 / (f_n^2 + f_m^2) weight
    does not reproduce eq. chi0 for fractional occupations; the weight used
    is f_n / (f_n^2 + f_m^2) (the minimal-norm split of the pair term, which
    reproduces the sum over states).  Terms m = n are excluded (carried by
    delta_f).  For |e_n - e_m| < 1e-8 Ha the divided difference is
    f'((e_n + e_m)/2).
  * the CG preconditioner is diag(|G+k|^2/2 + c_nk) with
    c_nk = max(<phi_nk, |G+k|^2/2 phi_nk>, 0.1 Ha) (the floor keeps a G = 0
    free-electron band from dividing by zero); z = Q M^-1 r and A p are re-projected
    onto range Q (Remark after Lemma cgtol_E); at least one CG iteration; the
    stopping test uses the recursively updated residual norm, absolute.
  * the Hxc kernel is K_H (4 pi / |G|^2 on the grid, 0 at G = 0) plus the
    Slater-exchange kernel f_x(rho) = -(1/3)(3/pi)^{1/3} max(rho,1e-10)^{-2/3}.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np
import scipy.fft as sfft

from .groundstate import GroundState, f_fd, f_fd_deriv, ground_state
from .system import WORKERS, System

DEGEN_TOL = 1e-8
PRECOND_FLOOR = 0.1     # Ha; floor of the preconditioner shift c_nk


# ---------------------------------------------------------------- helpers
def divided_difference(sys: System, gs: GroundState, ik: int, n: int, m: int) -> float:
    """(f_n - f_m)/(e_n - e_m), -> f' at the midpoint when near-degenerate
    (eq. fprime convention)."""
    e, f = gs.eps[ik], gs.occ[ik]
    de = e[n] - e[m]
    if abs(de) < DEGEN_TOL:
        T = sys.spec.temperature
        if T <= 0.0:
            return 0.0
        x = (0.5 * (e[n] + e[m]) - gs.fermi) / T
        return float(f_fd_deriv(x) / T)
    return float((f[n] - f[m]) / de)


def inner(a: np.ndarray, b: np.ndarray) -> complex:
    return complex(np.vdot(a, b))


# ---------------------------------------------------------------- kernel K
@dataclass
class HxcKernel:
    """K = K_H + K_xc on real grid vectors (eq. dyson_equation; Hartree
    diagonal 4 pi/|G|^2 with G = 0 -> 0 as in Sec. 3.4.3)."""
    sys: System
    rho: np.ndarray
    xc: int

    def __post_init__(self):
        g1, g2, g3 = self.sys.cube_g()
        gg = g1 ** 2 + g2 ** 2 + g3 ** 2
        with np.errstate(divide="ignore"):
            kh = np.where(gg > 0, 4.0 * np.pi / np.where(gg > 0, gg, 1.0), 0.0)
        self.kh = kh
        if self.xc:
            self.fx = -(1.0 / 3.0) * (3.0 / np.pi) ** (1.0 / 3.0) * \
                np.maximum(self.rho, 1e-10) ** (-2.0 / 3.0)
        else:
            self.fx = np.zeros(self.sys.n)

    def apply(self, v: np.ndarray) -> np.ndarray:
        v = v.reshape(self.sys.n)
        vh = sfft.ifftn(self.kh * sfft.fftn(v, workers=WORKERS),
                        workers=WORKERS).real
        return vh + self.fx * v

    def norm2_bound(self) -> float:
        """||K||_2 <= max 4 pi/|G|^2 + max |f_x| (used by the adjoint grt)."""
        return float(self.kh.max() + np.abs(self.fx).max())


# ---------------------------------------------------------------- SOS chi0
class SumOverStates:
    """chi0 by the plain sum over ALL eigenpairs of the dense H_k (tiny cells).

    (chi0 dV)(r) = sum_k w_k sum_{n,m} D_nm conj(psi_n) psi_m M_mn
                   - dEF sum_k w_k sum_n f'_n |psi_n|^2,
    M_mn = <psi_m, dV psi_n>, D_nm the divided difference with f_m = 0 for
    unoccupied bands, dEF = sum w f' M_nn / sum w f' (0 if the sum is 0).
    """

    def __init__(self, sys: System, gs: GroundState):
        import scipy.linalg
        self.sys = sys
        self.gs = gs
        self.full = []
        self.vecs = []
        T = sys.spec.temperature
        for ik, kb in enumerate(sys.bases):
            e, v = scipy.linalg.eigh(sys.dense_h(ik))
            nocc = gs.nocc_k[ik]
            # occupations of all states; f = 0 beyond the occupied set
            f = np.zeros(len(e))
            f[:nocc] = gs.occ[ik][:nocc]
            if T > 0:
                fp = np.zeros(len(e))
                fp[:nocc] = f_fd_deriv((e[:nocc] - gs.fermi) / T) / T
            else:
                fp = np.zeros(len(e))
            psi = sys.to_grid(ik, v.T).reshape(len(e), -1)   # [nall, ng]
            self.full.append((e, f, fp, psi))
            self.vecs.append(np.ascontiguousarray(v.T))

    def _dd(self, e, f, fp, n, m):
        de = e[n] - e[m]
        T = self.sys.spec.temperature
        if abs(de) < DEGEN_TOL:
            if T <= 0:
                return 0.0
            x = (0.5 * (e[n] + e[m]) - self.gs.fermi) / T
            return float(f_fd_deriv(x) / T)
        return (f[n] - f[m]) / de

    def apply(self, dv: np.ndarray, dv_nl=None) -> np.ndarray:
        """chi0 dV; ``dv_nl(ik, coeffs)`` optionally adds a non-multiplicative
        part of the perturbation (its action on coefficient rows), whose
        matrix elements join M_mn."""
        sys = self.sys
        dvf = dv.reshape(-1)
        out = np.zeros(sys.ng)
        num, den = 0.0, 0.0
        diag_terms = []
        for ik, kb in enumerate(sys.bases):
            e, f, fp, psi = self.full[ik]
            nocc = self.gs.nocc_k[ik]
            # M_mn for n occupied, all m
            mm = (psi.conj() * dvf) @ psi[:nocc].T * (sys.volume / sys.ng)  # [nall, nocc]
            if dv_nl is not None:
                vecs = self.vecs[ik]                                   # [nall, nb]
                mm = mm + vecs.conj() @ dv_nl(ik, vecs[:nocc]).T
            acc = np.zeros(sys.ng, complex)
            for n in range(nocc):
                for m in range(len(e)):
                    if m == n:
                        continue
                    d = self._dd(e, f, fp, n, m)
                    if d == 0.0:
                        continue
                    if m < nocc:
                        # both occupied: ordered pair counted once here
                        acc += d * psi[n].conj() * psi[m] * mm[m, n]
                    else:
                        # (n occ, m unocc) + (m, n) = 2 Re(...)
                        acc += 2.0 * d * (psi[n].conj() * psi[m] * mm[m, n]).real
            out += kb.weight * acc.real
            # diagonal m = n: f'_n (M_nn - dEF) |psi_n|^2
            for n in range(nocc):
                diag_terms.append((kb.weight, fp[n], mm[n, n].real,
                                   np.abs(psi[n]) ** 2))
                num += kb.weight * fp[n] * mm[n, n].real
                den += kb.weight * fp[n]
        def_ = num / den if den != 0.0 else 0.0
        for w, fpn, mnn, dens in diag_terms:
            out += w * fpn * (mnn - def_) * dens
        return out.reshape(sys.n)

    def dense_matrix(self) -> np.ndarray:
        """chi0 as an N_g x N_g real matrix.

        Each ordered pair (n occupied, m) contributes
        (|Omega|/N_g) D_nm a_nm a_nm^H with a_nm(r) = conj(psi_n) psi_m; pairs
        with m unoccupied also stand for their mirror (m, n), hence the real
        part; the Fermi-level term is the rank-one correction
        -(|Omega|/N_g) g g^T / sum w f', g = sum w f' |psi_n|^2.
        """
        sys = self.sys
        ng = sys.ng
        out = np.zeros((ng, ng))
        gvec = np.zeros(ng)
        den = 0.0
        for ik, kb in enumerate(sys.bases):
            e, f, fp, psi = self.full[ik]
            nocc = self.gs.nocc_k[ik]
            cols, wts = [], []
            for n in range(nocc):
                for m in range(len(e)):
                    d = fp[n] if m == n else self._dd(e, f, fp, n, m)
                    if d == 0.0:
                        continue
                    cols.append(psi[n].conj() * psi[m])
                    wts.append(d * (2.0 if m >= nocc else 1.0))
            if cols:
                a = np.array(cols).T                       # [ng, npairs]
                c = np.array(wts)
                out += kb.weight * (sys.volume / ng) * np.real((a * c) @ a.conj().T)
            for n in range(nocc):
                gvec += kb.weight * fp[n] * np.abs(psi[n]) ** 2
                den += kb.weight * fp[n]
        if den != 0.0:
            out -= (sys.volume / ng) * np.outer(gvec, gvec) / den
        return out


def chi0_fd(sys: System, dv: np.ndarray, h: float = 1e-4) -> np.ndarray:
    """chi0 dV = d/dh F_KS(V + h dV) by a central difference (eq. potdensmap).

    F_KS recomputes eigenpairs (dense), occupations and the Fermi level at
    the perturbed potential.
    """
    def rho_at(v):
        gs = ground_state(sys, dense=True, vloc=v)
        return gs.rho
    vp = sys.vloc + h * dv
    vm = sys.vloc - h * dv
    return (rho_at(vp) - rho_at(vm)) / (2.0 * h)


# ---------------------------------------------------------------- Sternheimer
@dataclass
class CGResult:
    x: np.ndarray
    iterations: int
    resnorm: float
    converged: bool


def sternheimer_cg(sys: System, gs: GroundState, ik: int, n: int,
                   rhs: np.ndarray, tol: float, maxiter: int = 1000,
                   miniter: int = 1) -> CGResult:
    """Solve Q (H_k - e_n) Q x = rhs, rhs in range Q, by preconditioned CG
    (eq. discretised_sternheimer; Remark after Lemma cgtol_E; Sec. 4.1.2)."""
    kb = sys.bases[ik]
    nocc = gs.nocc_k[ik]
    phi = gs.phi[ik][:nocc]                       # [nocc, nb]
    en = gs.eps[ik][n]

    def proj_q(y):
        return y - (phi.conj() @ y) @ phi

    def apply_a(y):
        return proj_q(sys.apply_h(ik, y) - en * y)

    ckin = float(np.real(np.vdot(gs.phi[ik][n], kb.kin * gs.phi[ik][n])))
    minv = 1.0 / (kb.kin + max(ckin, PRECOND_FLOOR))

    x = np.zeros_like(rhs)
    r = rhs.copy()
    z = proj_q(minv * r)
    p = z.copy()
    rz = np.real(np.vdot(r, z))
    it = 0
    rn = np.linalg.norm(r)
    while it < maxiter:
        if it >= miniter and rn <= tol:
            break
        ap = apply_a(p)
        alpha = rz / np.real(np.vdot(p, ap))
        x = x + alpha * p
        r = r - alpha * ap
        it += 1
        rn = np.linalg.norm(r)
        if it >= miniter and rn <= tol:
            break
        z = proj_q(minv * r)
        rz_new = np.real(np.vdot(r, z))
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
    return CGResult(x=x, iterations=it, resnorm=rn, converged=rn <= tol)


@dataclass
class Chi0Stats:
    n_ham: int = 0
    iterations: List[List[int]] = field(default_factory=list)


def chi0_sternheimer(sys: System, gs: GroundState, dv: np.ndarray,
                     tol, stats: Optional[Chi0Stats] = None,
                     maxiter: int = 1000, dv_nl=None) -> np.ndarray:
    """chi0 dV through the Sternheimer route (eq. kchi0, eq. delta_phi_P,
    eq. sternheimer_equation, eq. delta_f).

    ``tol`` is a scalar or a per-(k, n) list of absolute CG tolerances.
    ``dv_nl(ik, phi)`` optionally adds a non-multiplicative part of the
    perturbation: it returns (dV_nl phi_n) as coefficients [nocc, nb], added
    to t_n = F(dV psi_n) (the Sternheimer right-hand side and every matrix
    element of the perturbation only use dV phi_n).
    """
    dvg = dv.reshape(sys.n)
    rho1 = np.zeros(sys.n)
    per_band = []           # (k, n, w_k, f, f', de_n, psi_n)
    num, den = 0.0, 0.0
    for ik, kb in enumerate(sys.bases):
        nocc = gs.nocc_k[ik]
        phi = gs.phi[ik][:nocc]
        f = gs.occ[ik]
        fp = gs.focc_deriv[ik]
        psi = sys.to_grid(ik, phi)                          # [nocc, grid]
        t = sys.to_sphere(ik, dvg * psi)                    # F(dV psi_n)
        if dv_nl is not None:
            t = t + dv_nl(ik, phi)
        iters = []
        for n in range(nocc):
            tn = t[n]
            den_n = float(np.real(np.vdot(phi[n], tn)))    # delta eps_n
            # occupied part, minimal gauge (reading on the coefficient)
            dphi_p = np.zeros_like(tn)
            for m in range(nocc):
                if m == n:
                    continue
                d = divided_difference(sys, gs, ik, n, m)
                if d == 0.0:
                    continue
                alpha = f[n] * d / (f[n] ** 2 + f[m] ** 2)
                dphi_p += alpha * np.vdot(phi[m], tn) * phi[m]
            # unoccupied part: Sternheimer
            rhs = -(tn - (phi.conj() @ tn) @ phi)
            tau = tol if np.isscalar(tol) else tol[ik][n]
            res = sternheimer_cg(sys, gs, ik, n, rhs, tau, maxiter=maxiter)
            iters.append(res.iterations)
            if stats is not None:
                stats.n_ham += res.iterations
            dphi = dphi_p + res.x
            rho1 += kb.weight * 2.0 * f[n] * np.real(
                psi[n].conj() * sys.to_grid(ik, dphi))
            per_band.append((kb.weight, fp[n], den_n, psi[n]))
            num += kb.weight * fp[n] * den_n
            den += kb.weight * fp[n]
        if stats is not None:
            stats.iterations.append(iters)
    def_ = num / den if den != 0.0 else 0.0
    for w, fpn, den_n, psin in per_band:
        rho1 += w * fpn * (den_n - def_) * np.abs(psin) ** 2
    return rho1


# ---------------------------------------------------------------- dielectric
def apply_dielectric(sys: System, gs: GroundState, kern: HxcKernel,
                     v: np.ndarray, tol_fn, stats: Optional[Chi0Stats] = None):
    """E v = v - ||K v|| chi0(K v / ||K v||)  (eq. op_discretised).

    ``tol_fn(knorm)`` returns the CG tolerances (scalar or per (k, n)) for the
    normalised Sternheimer right-hand sides, given ||K v||.
    Returns (E v, ||K v||).
    """
    kv = kern.apply(v)
    nu = float(np.linalg.norm(kv))
    if nu == 0.0:
        return v.reshape(sys.n).copy(), 0.0
    chi = chi0_sternheimer(sys, gs, kv / nu, tol_fn(nu), stats=stats)
    return v.reshape(sys.n) - nu * chi, nu


def apply_dielectric_adjoint(sys: System, gs: GroundState, kern: HxcKernel,
                             v: np.ndarray, tol_fn, stats: Optional[Chi0Stats] = None):
    """E^T v = v - ||v|| K chi0(v / ||v||).

    The transpose of eq. op_discretised's operator: K and chi0 are symmetric
    in the Euclidean grid inner product, so (1 - chi0 K)^T = 1 - K chi0.  Not
    in the paper; used for dL/db = E^-T dL/d(drho).  ``tol_fn`` receives
    ||K||_2 ||v|| (the CG error reaches the result through K).
    Returns (E^T v, ||v||).
    """
    v = v.reshape(sys.n)
    nu = float(np.linalg.norm(v))
    if nu == 0.0:
        return v.copy(), 0.0
    chi = chi0_sternheimer(sys, gs, v / nu, tol_fn(kern.norm2_bound() * nu), stats=stats)
    return v - nu * kern.apply(chi), nu


def orbital_row_norm(sys: System, gs: GroundState, ik: int, real_part: bool = True) -> float:
    """||F_k^-1 Phi_k||_{2,inf} (max over grid points of the row norm), or of
    its real part (Sec. 3.4.1, used by the grt strategy).

    The real part depends on the phase of each orbital, which the eigensolver
    leaves arbitrary.  Sec. 3.4.1 takes it where a real representation of the
    orbitals can be chosen; each orbital is therefore first multiplied by the
    phase that makes sum_r psi(r)^2 real and positive (this is the real
    representation whenever one exists), and the result is floored at
    ||F_k^-1 Phi_k||_{2,inf} / sqrt(2), the largest loss the section allows."""
    nocc = gs.nocc_k[ik]
    psi = sys.to_grid(ik, gs.phi[ik][:nocc]).reshape(nocc, -1)
    full = float(np.sqrt(np.max(np.sum(np.abs(psi) ** 2, axis=0))))
    if not real_part:
        return full
    theta = -0.5 * np.angle(np.sum(psi * psi, axis=1))
    re = (psi * np.exp(1j * theta)[:, None]).real
    return max(float(np.sqrt(np.max(np.sum(re ** 2, axis=0)))), full / np.sqrt(2.0))


# ---------------------------------------------------------------- Kerker
def kerker_symbol(sys: System, alpha: float) -> np.ndarray:
    """D(G) = |G|^2 / (|G|^2 + alpha^2) on the FFT cube (numpy FFT order,
    |G| from the signed index) -- the Fourier representation of the
    discretised Kerker preconditioner (Sec. 3.3)."""
    g1, g2, g3 = sys.cube_g()
    gg = g1 ** 2 + g2 ** 2 + g3 ** 2
    return gg / (gg + alpha * alpha)


def kerker_apply(sys: System, v: np.ndarray, alpha: float) -> np.ndarray:
    """T v with T of eq. (kerker): (1 - 1 1^T / N_g) W^-1 D W + 1 1^T / N_g,
    the charge-conserving form of W^-1 D W (W the unitary grid DFT of
    eq. fft_ifft; W^-1 D W is applied through numpy's FFT pair, whose
    normalisations cancel).  Real grid vectors in, real out."""
    vg = v.reshape(sys.n)
    t = sfft.ifftn(kerker_symbol(sys, alpha) * sfft.fftn(vg, workers=WORKERS),
                   workers=WORKERS).real
    return t - t.mean() + vg.mean()
