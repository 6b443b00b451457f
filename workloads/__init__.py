"""Seeded synthetic workloads shared by the oracle and the HIP path.

This module only *describes* inputs: cell geometry, atom positions, model
parameters, and seeded random real-space fields (perturbations dV, right-hand
sides b).  It contains none of the response method's arithmetic (no
Hamiltonian, no Fourier bases, no response, no solver); both the CPU oracle
(`oracle/`) and the HIP library consume exactly these arrays.

Model (the potential model the paper's experiments replace; see the paper's
Section 2.1 for the Hamiltonian form):
  * orthorhombic cell of side lengths ``lattice`` (bohr);
  * per atom a Gaussian local potential of integral ``-amp`` (Ha bohr^3)
    and width ``sigma_loc``;
  * per atom one s-type Gaussian separable projector of width
    ``sigma_proj`` and strength ``d_proj`` (Ha);
  * plane-wave cutoff ``ecut`` (Ha), real-space grid ``fft``;
  * Gamma-centred unshifted k-grid ``kgrid`` (no symmetry reduction);
  * ``nocc`` doubly occupied bands plus ``nextra`` empty bands
    (``temperature`` = 0), or Fermi-Dirac smearing of ``2*nocc`` electrons
    over ``nocc + nextra`` bands (``temperature`` > 0);
  * ``xc`` = 1 adds the Slater-exchange kernel to the Hartree kernel.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Dict, Tuple

import numpy as np

__all__ = ["SystemSpec", "config", "CONFIGS", "random_field", "diamond_sites",
           "DV_SEED", "B_SEED", "BPRIME_SEED", "THROUGHPUT_B_SEEDS"]

DV_SEED = 1
B_SEED = 2
BPRIME_SEED = 3
THROUGHPUT_B_SEEDS = (2, 12, 22)


@dataclass(frozen=True)
class SystemSpec:
    name: str
    lattice: Tuple[float, float, float]
    frac_pos: np.ndarray            # [natoms, 3] fractional coordinates
    amp: np.ndarray                 # [natoms] local-potential amplitudes A
    sigma_loc: float = 0.8
    sigma_proj: float = 0.8
    d_proj: float = 1.0
    ecut: float = 8.0
    fft: Tuple[int, int, int] = (20, 20, 20)
    kgrid: Tuple[int, int, int] = (1, 1, 1)
    nocc: int = 4
    nextra: int = 2
    temperature: float = 0.0
    xc: int = 1

    @property
    def natoms(self) -> int:
        return int(self.frac_pos.shape[0])

    @property
    def ng(self) -> int:
        return int(np.prod(self.fft))

    @property
    def nbands(self) -> int:
        return self.nocc + self.nextra

    @property
    def volume(self) -> float:
        return float(np.prod(self.lattice))

    def with_(self, **kw) -> "SystemSpec":
        return replace(self, **kw)


# Fractional positions of the 8 sites of a conventional diamond cube.
_DIAMOND = np.array([
    [0.0, 0.0, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0],
    [0.25, 0.25, 0.25], [0.25, 0.75, 0.75], [0.75, 0.25, 0.75],
    [0.75, 0.75, 0.25]])


def diamond_sites(reps: Tuple[int, int, int], a: float, jitter: float,
                  seed: int = 0) -> np.ndarray:
    """Fractional positions of ``reps`` diamond cubes of side ``a``.

    Every atom is displaced independently by U(-jitter, jitter)*a per
    Cartesian component, drawn atom-major from ``default_rng(seed)``.
    """
    cells = []
    for i in range(reps[0]):
        for j in range(reps[1]):
            for k in range(reps[2]):
                cells.append(_DIAMOND + np.array([i, j, k], float))
    pos = np.concatenate(cells, axis=0)            # in units of a
    rng = np.random.default_rng(seed)
    pos = pos + rng.uniform(-jitter, jitter, size=pos.shape)
    lat = np.array(reps, float)
    frac = (pos / lat) % 1.0
    return frac


def _make_configs() -> Dict[str, SystemSpec]:
    c: Dict[str, SystemSpec] = {}
    # cfg1 is stated with 4 occupied bands, but at Gamma bands 4 and 5 of
    # this cell are degenerate (no gap); the smallest occupied count with a
    # gap >= 1e-4 Ha is 5 (gap 0.0316 Ha), which is used instead.
    a1 = 10.26
    c["cfg1"] = SystemSpec(
        name="cfg1", lattice=(a1, a1, a1),
        frac_pos=np.array([[0.0, 0.0, 0.0], [0.25, 0.25, 0.25]]),
        amp=np.array([4.0, 4.0]), ecut=8.0, fft=(20, 20, 20),
        kgrid=(1, 1, 1), nocc=5, nextra=2, temperature=0.0, xc=1)
    a = 20.52
    f2 = diamond_sites((1, 1, 1), a, 0.05, seed=0)
    c["cfg2"] = SystemSpec(
        name="cfg2", lattice=(a, a, a), frac_pos=f2, amp=np.full(8, 4.0),
        ecut=15.0, fft=(48, 48, 48), kgrid=(2, 2, 2), nocc=16, nextra=4,
        temperature=0.0, xc=1)
    f3 = diamond_sites((1, 1, 2), a, 0.05, seed=0)
    c["cfg3"] = SystemSpec(
        name="cfg3", lattice=(a, a, 2 * a), frac_pos=f3,
        amp=np.full(16, 4.0), ecut=20.0, fft=(48, 48, 96), kgrid=(2, 2, 2),
        nocc=32, nextra=6, temperature=0.0, xc=1)
    f4 = diamond_sites((1, 2, 2), a, 0.05, seed=0)
    c["cfg4"] = SystemSpec(
        name="cfg4", lattice=(a, 2 * a, 2 * a), frac_pos=f4,
        amp=np.full(32, 4.0), ecut=25.0, fft=(60, 108, 108),
        kgrid=(3, 3, 3), nocc=64, nextra=8, temperature=0.01, xc=1)
    c["cfg5"] = c["cfg3"].with_(name="cfg5")
    # Small variants (same model) used by parity tests: several k-points,
    # smearing, odd cell shapes, at sizes the oracle handles in seconds.
    c["small_k"] = c["cfg1"].with_(name="small_k", kgrid=(1, 1, 2), nocc=1,
                                   nextra=2)
    c["small_metal"] = c["cfg1"].with_(
        name="small_metal", kgrid=(1, 1, 2), nocc=3, nextra=7,
        temperature=0.002)
    c["small_rect"] = SystemSpec(
        name="small_rect", lattice=(a1, a1, 2 * a1),
        frac_pos=np.array([[0.0, 0.0, 0.0], [0.25, 0.25, 0.125],
                           [0.5, 0.5, 0.5], [0.75, 0.75, 0.625]]),
        amp=np.full(4, 4.0), ecut=5.0, fft=(20, 20, 36), kgrid=(1, 1, 2),
        nocc=8, nextra=4, temperature=0.0, xc=1)
    # More than 64 projection rows on a small grid (natoms + 2 N_occ = 68, or
    # 80 with the extra bands): closed free-electron shells at 33 bands.
    c["wide"] = c["cfg1"].with_(name="wide", nocc=33, nextra=6)
    c["wide_k"] = c["wide"].with_(name="wide_k", kgrid=(1, 1, 2))
    # 116 rows (57 occupied bands, the next closed shell; 128 with the extras)
    c["wider"] = c["cfg1"].with_(name="wider", nocc=57, nextra=6)
    # Tiny cells (N_g = 12^3) on which chi0 and E are formed as dense
    # matrices by the oracle.
    c["tiny"] = c["cfg1"].with_(name="tiny", ecut=3.0, fft=(12, 12, 12))
    c["tiny_k"] = c["tiny"].with_(name="tiny_k", kgrid=(1, 1, 2), nocc=1,
                                  nextra=2)
    c["tiny_metal"] = c["tiny"].with_(name="tiny_metal", kgrid=(1, 1, 2),
                                      nocc=3, nextra=7, temperature=0.002)
    # A 48 x 48 plane (the smallest on which the plane kernel is built at
    # both 256 and 512 threads) with the few bands of the tiny cell.
    c["tiny48"] = c["tiny"].with_(name="tiny48", fft=(48, 48, 48))
    return c


CONFIGS: Dict[str, SystemSpec] = _make_configs()


def config(name: str) -> SystemSpec:
    return CONFIGS[name]


def random_field(spec: SystemSpec, seed: int, gmax: float = 2.0) -> np.ndarray:
    """Seeded smooth real field on the real-space grid, C-order [N1][N2][N3].

    Fourier coefficients on 0 < |G| < gmax are complex N(0,1) times
    exp(-|G|^2/2); the coefficient at G = 0 is zero (zero mean).  Taking the
    real part of the inverse grid transform is the Hermitian symmetrisation.
    The result is scaled to unit Euclidean norm over grid values.
    """
    n = np.array(spec.fft)
    recip = 2.0 * np.pi / np.array(spec.lattice)
    idx = [np.fft.fftfreq(int(m), 1.0 / int(m)) for m in n]   # signed ints
    g1, g2, g3 = np.meshgrid(idx[0] * recip[0], idx[1] * recip[1],
                             idx[2] * recip[2], indexing="ij")
    gg = g1 ** 2 + g2 ** 2 + g3 ** 2
    rng = np.random.default_rng(seed)
    coef = rng.standard_normal(gg.shape) + 1j * rng.standard_normal(gg.shape)
    mask = (gg > 0) & (gg < gmax ** 2)
    coef = np.where(mask, coef * np.exp(-gg / 2.0), 0.0)
    field = np.fft.ifftn(coef).real
    nrm = np.linalg.norm(field)
    return np.ascontiguousarray(field / nrm)
