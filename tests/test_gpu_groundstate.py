"""GPU parity of the library's own ground state (Chebyshev-filtered subspace
iteration on the GPU) against the oracle's eigensolvers, and the response
computed end to end from it."""
import numpy as np
import pytest

from gpu_common import gpu_system, rel, to_dev, to_host
from workloads import random_field

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["tiny", "cfg1", "small_rect", "small_metal", "tiny_k"])
def test_eigenvalues_and_subspace(name):
    rs, osys, ogs, perms = gpu_system(name, ground_state="compute")
    eps, occ, cf, fermi = rs.ground_state()
    info = rs.setup_info()
    print(name, "eigensolver outer steps", info["gs_iters"], "residual", info["gs_residual"])
    assert info["gs_residual"] <= 1e-10
    for k in range(len(ogs.eps)):
        assert np.max(np.abs(eps[k] - ogs.eps[k])) < 1e-10
        # occupied projector agrees (gauge-invariant)
        no = ogs.nocc_k[k]
        nb = len(perms[k])
        phi = np.zeros((no, nb), complex)
        phi[:, perms[k]] = cf[k, :no, :nb]
        p_gpu = phi.T @ phi.conj()
        p_ora = ogs.phi[k][:no].T @ ogs.phi[k][:no].conj()
        assert np.max(np.abs(p_gpu - p_ora)) < 1e-8
    rho = to_host(rs.density())
    assert rel(rho, ogs.rho) < 1e-9


@pytest.mark.parametrize("name", ["cfg1", "small_metal"])
def test_chi0_from_library_ground_state(name):
    from oracle.response import SumOverStates
    rs, osys, ogs, perms = gpu_system(name, ground_state="compute")
    dv = random_field(osys.spec, 1)
    got, st = rs.apply_chi0(to_dev(dv), cg_tol=1e-12)
    sos = SumOverStates(osys, ogs).apply(dv)
    assert rel(to_host(got), sos) < 1e-8
