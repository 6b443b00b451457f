"""Discretisation and model Hamiltonian (oracle, test infrastructure only).

Follows the paper's Sec. 2.3.1 (plane-wave bases, eq. fourier_bases and
eq. fft_ifft), eq. (Hamiltonian) and its Bloch form in Sec. 4.1.1.

Readings where the paper is silent or garbled, taken here:
  * orthorhombic cells only; reciprocal vectors b_i = 2 pi / a_i;
  * the k-grid is Gamma-centred and unshifted, k_j = (i_j / l_j) folded
    into [-1/2, 1/2), weights 1/N_k, no symmetry reduction (the printed
    Monkhorst-Pack definition repeats b_1 three times);
  * the local potential has Fourier coefficients
    (1/|Omega|) sum_a (-A_a) exp(-sigma^2 |G|^2 / 2) exp(-i G.R_a) on the
    whole FFT cube and V(r) is the real part of its inverse grid sum
    (keeps index -N/2);
  * projectors p_a(q) = (4 pi s^2)^{3/4} exp(-s^2 |q|^2 / 2) exp(-i q.R_a)
    / sqrt|Omega|, q = G + k, the Fourier coefficients of an L2-normalised
    Gaussian; V_nl = D sum_a |p_a><p_a|;
  * the operator is exactly the FFT-on-the-stated-grid operator, aliasing
    included (the stated grids are smaller than the paper's density cube).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List

import os

import numpy as np
import scipy.fft as sfft

from workloads import SystemSpec

WORKERS = max(1, len(os.sched_getaffinity(0)))


@dataclass
class KBasis:
    """Plane-wave sphere for one k-point: {G : |G + k|^2 <= 2 Ecut}."""
    kfrac: np.ndarray        # k in units of b_i
    kcart: np.ndarray        # k in bohr^-1
    weight: float
    miller: np.ndarray       # [nb, 3] signed integer G indices
    q: np.ndarray            # [nb, 3] G + k (cartesian)
    kin: np.ndarray          # [nb] |G + k|^2 / 2
    grid_index: np.ndarray   # [nb] flat C-order index of G mod N on the cube

    @property
    def nb(self) -> int:
        return int(self.miller.shape[0])


class System:
    """Everything the oracle derives from a SystemSpec."""

    def __init__(self, spec: SystemSpec):
        self.spec = spec
        self.a = np.array(spec.lattice, float)
        self.b = 2.0 * np.pi / self.a
        self.n = tuple(int(x) for x in spec.fft)
        self.ng = int(np.prod(self.n))
        self.volume = float(np.prod(self.a))
        # w = sqrt(|Omega| / N_g)  (Sec. 2.3.1, eq. fft_ifft)
        self.w = np.sqrt(self.volume / self.ng)
        self.pos = np.asarray(spec.frac_pos, float) * self.a    # cartesian
        self.kpoints = self._kgrid()
        self.bases: List[KBasis] = [self._sphere(kf, wk)
                                    for kf, wk in self.kpoints]
        self.vloc = self._local_potential()

    # -- k-points (Sec. 4.1.1; reading: Gamma-centred, folded to [-1/2,1/2))
    def _kgrid(self):
        l1, l2, l3 = self.spec.kgrid
        nk = l1 * l2 * l3
        out = []
        for i in range(l1):
            for j in range(l2):
                for k in range(l3):
                    f = np.array([i / l1, j / l2, k / l3])
                    f = np.where(f >= 0.5, f - 1.0, f)
                    out.append((f, 1.0 / nk))
        return out

    # -- sphere basis (eq. fourier_bases with |G + k| <= sqrt(2 Ecut))
    def _sphere(self, kfrac, wk) -> KBasis:
        kc = kfrac * self.b
        rng = [np.arange(-m // 2, m // 2) for m in self.n]     # cube indices
        i1, i2, i3 = np.meshgrid(*rng, indexing="ij")
        mill = np.stack([i1.ravel(), i2.ravel(), i3.ravel()], axis=1)
        q = mill * self.b + kc
        qq = np.sum(q * q, axis=1)
        keep = qq <= 2.0 * self.spec.ecut
        mill = mill[keep]
        q = q[keep]
        n = np.array(self.n)
        wrapped = np.mod(mill, n)
        flat = (wrapped[:, 0] * n[1] + wrapped[:, 1]) * n[2] + wrapped[:, 2]
        return KBasis(kfrac=kfrac, kcart=kc, weight=wk, miller=mill, q=q,
                      kin=0.5 * np.sum(q * q, axis=1), grid_index=flat)

    # -- cube G vectors in numpy FFT order (signed indices)
    def cube_g(self):
        idx = [np.fft.fftfreq(m, 1.0 / m) for m in self.n]
        g1, g2, g3 = np.meshgrid(idx[0] * self.b[0], idx[1] * self.b[1],
                                 idx[2] * self.b[2], indexing="ij")
        return g1, g2, g3

    # -- local potential on the real-space grid (reading S16/S18)
    def _local_potential(self, amp=None) -> np.ndarray:
        spec = self.spec
        amp = np.asarray(spec.amp if amp is None else amp, float)
        g1, g2, g3 = self.cube_g()
        gg = g1 ** 2 + g2 ** 2 + g3 ** 2
        vt = np.zeros(self.n, complex)
        for a in range(spec.natoms):
            r = self.pos[a]
            phase = np.exp(-1j * (g1 * r[0] + g2 * r[1] + g3 * r[2]))
            vt += -amp[a] * np.exp(-spec.sigma_loc ** 2 * gg / 2.0) * phase
        vt /= self.volume
        # V(r) = Re sum_G Vt(G) e^{iG.r}: numpy's ifftn carries 1/N_g.
        return np.ascontiguousarray((np.fft.ifftn(vt) * self.ng).real)

    def local_potential_derivative(self, atom: int) -> np.ndarray:
        """dV_loc / dA_atom on the grid (the potential is linear in A)."""
        amp = np.zeros(self.spec.natoms)
        amp[atom] = 1.0
        return self._local_potential(amp)

    def with_amplitudes(self, amp) -> "System":
        spec = self.spec.with_(amp=np.asarray(amp, float))
        return System(spec)

    # -- projectors (reading S17)
    def projectors(self, ik: int) -> np.ndarray:
        """[natoms, nb] projector coefficients p_a(G + k)."""
        s = self.spec.sigma_proj
        kb = self.bases[ik]
        qq = 2.0 * kb.kin
        radial = (4.0 * np.pi * s * s) ** 0.75 * np.exp(-s * s * qq / 2.0)
        radial /= np.sqrt(self.volume)
        ph = np.exp(-1j * (kb.q @ self.pos.T)).T        # [natoms, nb]
        return radial[None, :] * ph

    # -- F^-1 and F of eq. fft_ifft (literal: w^-1 W^-1 Z and w Z^T W)
    def to_grid(self, ik: int, coef: np.ndarray) -> np.ndarray:
        """F^-1: sphere coefficients [..., nb] -> grid values [..., N1,N2,N3]."""
        kb = self.bases[ik]
        lead = coef.shape[:-1]
        full = np.zeros(lead + (self.ng,), complex)
        full[..., kb.grid_index] = coef
        full = full.reshape(lead + self.n)
        axes = tuple(range(len(lead), len(lead) + 3))
        return sfft.ifftn(full, axes=axes, norm="ortho", workers=WORKERS) / self.w

    def to_sphere(self, ik: int, vals: np.ndarray) -> np.ndarray:
        """F: grid values [..., N1,N2,N3] -> sphere coefficients [..., nb]."""
        kb = self.bases[ik]
        lead = vals.shape[:-3]
        axes = tuple(range(len(lead), len(lead) + 3))
        full = sfft.fftn(vals, axes=axes, norm="ortho", workers=WORKERS) * self.w
        return full.reshape(lead + (self.ng,))[..., kb.grid_index]

    # -- Hamiltonian (eq. Hamiltonian, Bloch form): FFT-applied
    def apply_h(self, ik: int, x: np.ndarray, vloc=None) -> np.ndarray:
        """H_k x for x [..., nb]: kinetic + F(V F^-1 x) + nonlocal."""
        kb = self.bases[ik]
        v = self.vloc if vloc is None else vloc
        y = kb.kin * x
        y = y + self.to_sphere(ik, v * self.to_grid(ik, x))
        p = self.projectors(ik)
        c = x @ p.conj().T                                 # [..., natoms]
        y = y + self.spec.d_proj * (c @ p)
        return y

    # -- Hamiltonian: dense matrix (tiny cells only)
    def dense_h(self, ik: int, vloc=None) -> np.ndarray:
        """H_k[G, G'] = |G+k|^2/2 d + Vhat(G - G') + D sum_a p_a(G) p_a(G')^*.

        Vhat is the grid DFT (1/N_g) sum_r V(r) e^{-iG.r}, indexed with the
        difference of Miller indices folded onto the grid, so the dense matrix
        is the same operator as the FFT-applied one, aliasing included.
        """
        kb = self.bases[ik]
        v = self.vloc if vloc is None else vloc
        vhat = np.fft.fftn(v) / self.ng
        n = np.array(self.n)
        d = kb.miller[:, None, :] - kb.miller[None, :, :]
        d = np.mod(d, n)
        h = vhat[d[..., 0], d[..., 1], d[..., 2]].astype(complex)
        h[np.diag_indices(kb.nb)] += kb.kin
        p = self.projectors(ik)
        h += self.spec.d_proj * (p.T @ p.conj())
        return h
