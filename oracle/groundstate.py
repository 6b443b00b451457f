"""Ground state of the fixed model Hamiltonian (oracle, test infrastructure only).

Eigenpairs (eq. KS / eq. discretised_KS, Bloch form of Sec. 4.1.1),
occupations and Fermi level (eq. density with f_FD(x) = 2/(1+e^x)),
occupation derivatives (eq. fprime) and the density (eq. bzdensity).

Reading: the potential is fixed (no self-consistency); "insulator" means
f = 2 for the first nocc bands of every k-point and f = 0 otherwise, so
f' = 0.  With smearing, the Fermi level is found by bisection so that
sum_k w_k sum_n f_nk = 2 nocc over the computed bands only, and a band
counts as occupied when f_nk > 1e-10 (the paper's epsilon_occ threshold,
value chosen here).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional

import numpy as np
import scipy.linalg
import scipy.sparse.linalg as spla

from .system import System

EPS_OCC = 1e-10


@dataclass
class GroundState:
    eps: List[np.ndarray]       # per k: [nbands] eigenvalues
    phi: List[np.ndarray]       # per k: [nbands, nb] orthonormal coefficients
    occ: List[np.ndarray]       # per k: [nbands] f_nk in [0, 2]
    focc_deriv: List[np.ndarray]  # per k: [nbands] f'_nk (eq. fprime)
    fermi: float
    nocc_k: List[int]           # occupied bands per k (f > EPS_OCC)
    rho: np.ndarray             # density on the grid


def f_fd(x):
    """Fermi-Dirac occupation 2 / (1 + e^x), evaluated without overflow."""
    x = np.asarray(x, float)
    return 2.0 * np.where(x > 0, np.exp(-np.abs(x)) / (1.0 + np.exp(-np.abs(x))),
                          1.0 / (1.0 + np.exp(-np.abs(x))))


def f_fd_deriv(x):
    """d/dx of 2/(1+e^x) = -2 e^x / (1+e^x)^2, evaluated without overflow."""
    e = np.exp(-np.abs(np.asarray(x, float)))
    return -2.0 * e / (1.0 + e) ** 2


def eigenpairs(sys: System, ik: int, nbands: int, dense: Optional[bool] = None,
               tol: float = 1e-10, vloc=None):
    """Lowest nbands eigenpairs of H_k (dense eigh, or block LOBPCG)."""
    nb = sys.bases[ik].nb
    if dense is None:
        dense = nb <= 3000
    if dense:
        h = sys.dense_h(ik, vloc=vloc)
        e, v = scipy.linalg.eigh(h, subset_by_index=[0, nbands - 1])
        return e, np.ascontiguousarray(v.T)
    # Block LOBPCG with the kinetic preconditioner 1/(|G+k|^2/2 + 0.1),
    # followed by a Rayleigh-Ritz polish; results are checked by residual.
    kin = sys.bases[ik].kin
    nblk = nbands + 4

    def matmat(X):
        return sys.apply_h(ik, np.asarray(X).T, vloc=vloc).T

    op = spla.LinearOperator((nb, nb), dtype=complex,
                             matvec=lambda x: matmat(x.reshape(nb, 1)).ravel(),
                             matmat=matmat)
    prec = spla.LinearOperator(
        (nb, nb), dtype=complex,
        matvec=lambda x: x.ravel() / (kin + 0.1),
        matmat=lambda X: X / (kin[:, None] + 0.1))
    rng = np.random.default_rng(1234 + ik)
    x0 = rng.standard_normal((nb, nblk)) + 1j * rng.standard_normal((nb, nblk))
    x0 *= np.exp(-kin)[:, None]
    e, v = spla.lobpcg(op, x0, M=prec, largest=False, tol=tol * 0.1,
                       maxiter=1000)
    q, _ = np.linalg.qr(v)
    hs = q.conj().T @ matmat(q)
    e2, c = np.linalg.eigh(0.5 * (hs + hs.conj().T))
    v = q @ c[:, :nbands]
    return e2[:nbands], np.ascontiguousarray(v.T)


def occupations(sys: System, eps: List[np.ndarray]):
    """f_nk, f'_nk and the Fermi level (eq. density, eq. fprime)."""
    spec = sys.spec
    nk = len(eps)
    if spec.temperature <= 0.0:
        occ = [np.where(np.arange(len(e)) < spec.nocc, 2.0, 0.0) for e in eps]
        dfo = [np.zeros(len(e)) for e in eps]
        homo = max(e[spec.nocc - 1] for e in eps)
        lumo = min(e[spec.nocc] for e in eps) if len(eps[0]) > spec.nocc else homo
        return occ, dfo, 0.5 * (homo + lumo)
    T = spec.temperature
    nel = 2.0 * spec.nocc
    w = np.array([kb.weight for kb in sys.bases])

    def count(ef):
        return sum(w[k] * np.sum(f_fd((eps[k] - ef) / T)) for k in range(nk))

    lo = min(e.min() for e in eps) - 50 * T
    hi = max(e.max() for e in eps) + 50 * T
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if count(mid) < nel:
            lo = mid
        else:
            hi = mid
        if hi - lo < 1e-15:
            break
    ef = 0.5 * (lo + hi)
    occ = [f_fd((e - ef) / T) for e in eps]
    dfo = [f_fd_deriv((e - ef) / T) / T for e in eps]
    return occ, dfo, ef


def density(sys: System, phi: List[np.ndarray], occ: List[np.ndarray]) -> np.ndarray:
    """rho = sum_k w_k sum_n f_nk |F_k^-1 phi_nk|^2 (eq. bzdensity)."""
    rho = np.zeros(sys.n)
    for ik, kb in enumerate(sys.bases):
        psi = sys.to_grid(ik, phi[ik])
        rho += kb.weight * np.einsum("n,nxyz->xyz", occ[ik], np.abs(psi) ** 2)
    return rho


def ground_state(sys: System, dense: Optional[bool] = None, vloc=None) -> GroundState:
    nbands = sys.spec.nbands
    eps, phi = [], []
    for ik in range(len(sys.bases)):
        e, v = eigenpairs(sys, ik, nbands, dense=dense, vloc=vloc)
        eps.append(e)
        phi.append(v)
    occ, dfo, ef = occupations(sys, eps)
    nocc_k = [int(np.max(np.nonzero(o > EPS_OCC)[0]) + 1) for o in occ]
    rho = density(sys, phi, occ)
    return GroundState(eps=eps, phi=phi, occ=occ, focc_deriv=dfo, fermi=ef,
                       nocc_k=nocc_k, rho=rho)
