"""Pins of the oracle's ground state: eigen-residuals, orthonormality, the
electron count, the Fermi-Dirac derivative, and two independent eigensolvers
agreeing."""
import numpy as np
import pytest

from oracle.groundstate import (eigenpairs, f_fd, f_fd_deriv, ground_state,
                                occupations)
from oracle.system import System
from workloads import config


@pytest.mark.parametrize("name", ["tiny", "cfg1", "small_metal", "small_rect"])
def test_eigenpairs_residual_orthonormal_count(name, oracle_case):
    sys, gs = oracle_case(name)
    for ik in range(len(sys.bases)):
        phi = gs.phi[ik]
        res = sys.apply_h(ik, phi) - gs.eps[ik][:, None] * phi
        assert np.max(np.linalg.norm(res, axis=1)) < 1e-10
        assert np.max(np.abs(phi.conj() @ phi.T - np.eye(len(phi)))) < 1e-12
        assert np.all(np.diff(gs.eps[ik]) >= -1e-14)
    nel = gs.rho.sum() * sys.volume / sys.ng
    assert abs(nel - 2 * sys.spec.nocc) < 1e-10
    wsum = sum(kb.weight * np.sum(gs.occ[ik]) for ik, kb in enumerate(sys.bases))
    assert abs(wsum - 2 * sys.spec.nocc) < 1e-10


def test_iterative_and_dense_eigensolvers_agree():
    sys = System(config("cfg1"))
    e_d, v_d = eigenpairs(sys, 0, 7, dense=True)
    e_i, v_i = eigenpairs(sys, 0, 7, dense=False)
    assert np.max(np.abs(e_d - e_i)) < 1e-10
    # same occupied subspace (5 bands below the gap)
    p_d = v_d[:5].T @ v_d[:5].conj()
    p_i = v_i[:5].T @ v_i[:5].conj()
    assert np.max(np.abs(p_d - p_i)) < 1e-8


def test_free_electron_spectrum():
    spec = config("cfg1").with_(amp=np.zeros(2), d_proj=0.0, nocc=7, nextra=2)
    sys = System(spec)
    e, _ = eigenpairs(sys, 0, 9, dense=True)
    ref = np.sort(sys.bases[0].kin)[:9]
    assert np.max(np.abs(e - ref)) < 1e-14
    # shells 0, (2 pi/a)^2/2 x6, 2 (2 pi/a)^2 / 2 ...
    g = 2 * np.pi / 10.26
    assert abs(e[1] - 0.5 * g * g) < 1e-14 and abs(e[6] - 0.5 * g * g) < 1e-14


def test_fermi_dirac_derivative_and_count():
    x = np.linspace(-30, 30, 601)
    h = 1e-5
    fd = (f_fd(x + h) - f_fd(x - h)) / (2 * h)
    assert np.max(np.abs(fd - f_fd_deriv(x))) < 1e-9
    assert abs(f_fd(0.0) - 1.0) < 1e-15 and f_fd(-800.0) == 2.0 and f_fd(800.0) == 0.0


def test_metal_fermi_level_and_occupied_counts(oracle_case):
    sys, gs = oracle_case("small_metal")
    T = sys.spec.temperature
    for ik in range(len(sys.bases)):
        f = f_fd((gs.eps[ik] - gs.fermi) / T)
        assert np.max(np.abs(f - gs.occ[ik])) < 1e-14
        nocc = gs.nocc_k[ik]
        assert np.all(gs.occ[ik][:nocc] > 1e-10)
        assert np.all(gs.occ[ik][nocc:] <= 1e-10)
    assert gs.nocc_k == [7, 8]
