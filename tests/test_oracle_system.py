"""Pins of the oracle's discretisation and Hamiltonian against facts that do
not come from the oracle itself (closed forms, real-space sums, invariants).
"""
import numpy as np
import pytest

from oracle.system import System
from workloads import config


def _periodic_gaussians(sys, pts):
    """Direct real-space sum of -A (2 pi s^2)^{-3/2} exp(-|r-R-L|^2/2s^2)."""
    s = sys.spec.sigma_loc
    out = np.zeros(len(pts))
    shifts = [np.array([i, j, k]) * sys.a for i in (-1, 0, 1)
              for j in (-1, 0, 1) for k in (-1, 0, 1)]
    for a in range(sys.spec.natoms):
        for L in shifts:
            d = pts - sys.pos[a] - L
            out += -sys.spec.amp[a] * (2 * np.pi * s * s) ** -1.5 * \
                np.exp(-np.sum(d * d, axis=1) / (2 * s * s))
    return out


def test_local_potential_is_sum_of_gaussians():
    # cfg2's grid truncates the Gaussian's Fourier series at exp(-17): the
    # grid values equal the real-space lattice sum to ~1e-8.
    sys = System(config("cfg2"))
    rng = np.random.default_rng(0)
    idx = rng.integers(0, 48, size=(200, 3))
    pts = idx / np.array(sys.n) * sys.a
    ref = _periodic_gaussians(sys, pts)
    got = sys.vloc[idx[:, 0], idx[:, 1], idx[:, 2]]
    assert np.max(np.abs(got - ref)) < 1e-6 * np.max(np.abs(ref))


def test_local_potential_integral():
    for name in ("cfg1", "small_rect"):
        sys = System(config(name))
        integral = sys.vloc.sum() * sys.volume / sys.ng
        assert abs(integral + np.sum(sys.spec.amp)) < 1e-10


@pytest.mark.parametrize("name", ["tiny", "cfg1", "small_metal", "small_rect"])
def test_dense_h_hermitian_and_equals_fft_apply(name):
    sys = System(config(name))
    rng = np.random.default_rng(3)
    for ik in range(len(sys.bases)):
        h = sys.dense_h(ik)
        assert np.max(np.abs(h - h.conj().T)) < 1e-14
        x = rng.standard_normal((3, sys.bases[ik].nb)) + \
            1j * rng.standard_normal((3, sys.bases[ik].nb))
        y1 = (h @ x.T).T
        y2 = sys.apply_h(ik, x)
        assert np.linalg.norm(y1 - y2) < 1e-12 * np.linalg.norm(y1)


def test_free_electron_hamiltonian_is_kinetic_diagonal():
    spec = config("small_metal").with_(amp=np.zeros(2), d_proj=0.0)
    sys = System(spec)
    for ik, kb in enumerate(sys.bases):
        h = sys.dense_h(ik)
        assert np.max(np.abs(h - np.diag(kb.kin))) < 1e-17
        # kinetic energies are |G + k|^2 / 2 with k folded into [-1/2, 1/2)
        assert np.allclose(kb.kin, 0.5 * np.sum(
            (kb.miller * sys.b + kb.kfrac * sys.b) ** 2, axis=1), rtol=0, atol=1e-15)


def test_parseval_weight_convention():
    """(|Omega|/N_g) sum_r |F^-1 phi|^2 = sum_G |phi_G|^2 (Sec. 2.3.1)."""
    sys = System(config("small_rect"))
    rng = np.random.default_rng(1)
    for ik, kb in enumerate(sys.bases):
        c = rng.standard_normal(kb.nb) + 1j * rng.standard_normal(kb.nb)
        u = sys.to_grid(ik, c)
        assert abs(np.sum(np.abs(u) ** 2) * sys.volume / sys.ng
                   - np.sum(np.abs(c) ** 2)) < 1e-11 * np.sum(np.abs(c) ** 2)
        # a single plane wave is e^{iG.r}/sqrt|Omega| on the grid
        e = np.zeros(kb.nb, complex)
        e[7] = 1.0
        u = sys.to_grid(ik, e)
        r = np.stack(np.meshgrid(*[np.arange(m) / m * a for m, a in
                                  zip(sys.n, sys.a)], indexing="ij"), -1)
        g = kb.miller[7] * sys.b
        ref = np.exp(1j * r @ g) / np.sqrt(sys.volume)
        assert np.max(np.abs(u - ref)) < 1e-12
        back = sys.to_sphere(ik, u)
        assert np.max(np.abs(back - e)) < 1e-13


def test_projector_is_normalised_gaussian():
    """sum_G |p(G+k)|^2 -> int |p|^2 = 1 once the sphere covers the Gaussian."""
    spec = config("cfg1").with_(ecut=30.0, fft=(40, 40, 40))
    sys = System(spec)
    p = sys.projectors(0)
    assert np.allclose(np.sum(np.abs(p) ** 2, axis=1), 1.0, atol=1e-6)


def test_sphere_size_matches_paper_estimate():
    """N_b ~ sqrt(2)/(3 pi^2) Ecut^{3/2} |Omega| (eq. Nb_Ng_definition)."""
    for name in ("cfg1", "cfg2", "cfg3"):
        sys = System(config(name))
        est = np.sqrt(2) / (3 * np.pi ** 2) * sys.spec.ecut ** 1.5 * sys.volume
        for kb in sys.bases:
            assert abs(kb.nb - est) / est < 0.03


def test_kgrid_folding_and_weights():
    sys = System(config("cfg2"))
    kf = np.array([k for k, _ in sys.kpoints])
    assert len(kf) == 8 and set(np.unique(kf)) == {-0.5, 0.0}
    assert abs(sum(w for _, w in sys.kpoints) - 1.0) < 1e-15


@pytest.mark.parametrize("name,ik", [("cfg1", 0), ("small_k", 0), ("small_k", 1)])
def test_projector_real_space_centre(name, ik):
    """F_k^-1 p_a on the grid is the L2-normalised Gaussian
    (pi s^2)^{-3/4} exp(-|r - R_a - L|^2 / 2 s^2) centred on the atom, summed over
    lattice vectors L with the Bloch phase e^{-ik.(r - L)} left by F^-1 (the
    e^{ik.r} factor is dropped, Sec. 4.1.1): the Poisson summation of the
    projector's Fourier coefficients.  A sign slip in e^{-iq.R} moves every
    projector to -R, which this fails (the atoms here are not centrosymmetric
    about the origin: R = (a/4, a/4, a/4) and -R differ by a/2 per axis)."""
    spec = config(name).with_(ecut=30.0, fft=(40, 40, 40))
    sys = System(spec)
    kb = sys.bases[ik]
    p = sys.projectors(ik)
    grid = sys.to_grid(ik, p)                      # [natoms, N1, N2, N3]
    s = spec.sigma_proj
    r = np.stack(np.meshgrid(*[np.arange(m) / m * a for m, a in zip(sys.n, sys.a)],
                             indexing="ij"), -1)
    shifts = [np.array([i, j, k]) * sys.a for i in (-1, 0, 1)
              for j in (-1, 0, 1) for k in (-1, 0, 1)]
    for a in range(spec.natoms):
        ref = np.zeros(sys.n, complex)
        for L in shifts:
            d = r - sys.pos[a] - L
            ref += (np.pi * s * s) ** -0.75 * np.exp(-np.sum(d * d, -1) / (2 * s * s)) * \
                np.exp(-1j * ((r - L) @ kb.kcart))
        assert np.max(np.abs(grid[a] - ref)) < 1e-6 * np.max(np.abs(ref))
        # the mirrored centre is far off: the test is not blind to the sign
        mir = np.zeros(sys.n, complex)
        for L in shifts:
            d = r + sys.pos[a] - L
            mir += (np.pi * s * s) ** -0.75 * np.exp(-np.sum(d * d, -1) / (2 * s * s)) * \
                np.exp(-1j * ((r - L) @ kb.kcart))
        if np.linalg.norm(sys.pos[a]) > 0:
            assert np.max(np.abs(grid[a] - mir)) > 0.1 * np.max(np.abs(ref))
