"""GPU parity of the operators under the response path against the oracle:
H_k psi (pruned FFT + nonlocal), the ground-state density, and the Hxc
kernel, element by element on the same seeded inputs."""
import numpy as np
import pytest

from gpu_common import gpu_system, rel, to_dev, to_host
from workloads import random_field

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["tiny", "cfg1", "small_rect", "small_metal"])
def test_hamiltonian_matches_dense(name):
    rs, osys, ogs, perms = gpu_system(name)
    inf = rs.info()
    rng = np.random.default_rng(11)
    for k in range(inf.nk):
        nb = len(perms[k])
        nvec = 19                     # > one tile of 16, ragged tail
        x = np.zeros((nvec, inf.nb_max), np.complex128)
        x[:, :nb] = rng.standard_normal((nvec, nb)) + 1j * rng.standard_normal((nvec, nb))
        y = to_host(rs.apply_hamiltonian(k, to_dev(x)))
        h = osys.dense_h(k)
        xo = np.zeros((nvec, nb), np.complex128)
        xo[:, perms[k]] = x[:, :nb]
        yo = (h @ xo.T).T
        got = y[:, :nb]
        ref = yo[:, perms[k]]
        assert rel(got, ref) < 1e-12, (name, k, rel(got, ref))


def test_hamiltonian_cfg2_sampled_rows():
    """Full-size cfg2 grid: sampled rows of H_k x computed one by one."""
    from oracle.system import System
    from paper_2505_02319_amd import ResponseSystem
    from workloads import config
    spec = config("cfg2")
    osys = System(spec)
    rs = ResponseSystem(spec, ground_state=None)
    inf = rs.info()
    rng = np.random.default_rng(5)
    vhat = np.fft.fftn(osys.vloc) / osys.ng
    n = np.array(osys.n)
    for k in (0, 7):
        m_lib = rs.basis(k)
        nb = len(m_lib)
        x = np.zeros((3, inf.nb_max), np.complex128)
        x[:, :nb] = rng.standard_normal((3, nb)) + 1j * rng.standard_normal((3, nb))
        y = to_host(rs.apply_hamiltonian(k, to_dev(x)))
        kb = osys.bases[k]
        kin = 0.5 * np.sum((m_lib * osys.b + kb.kcart) ** 2, axis=1)
        q = m_lib * osys.b + kb.kcart
        s = osys.spec.sigma_proj
        p = (4 * np.pi * s * s) ** 0.75 * np.exp(-s * s * np.sum(q * q, 1) / 2) / np.sqrt(osys.volume)
        proj = p[None, :] * np.exp(-1j * (q @ osys.pos.T)).T
        for row in rng.integers(0, nb, size=24):
            d = np.mod(m_lib[row] - m_lib, n)
            hrow = vhat[d[:, 0], d[:, 1], d[:, 2]] + osys.spec.d_proj * proj[:, row] @ proj.conj()
            hrow[row] += kin[row]
            ref = x[:, :nb] @ hrow
            assert np.max(np.abs(y[:, row] - ref)) < 1e-12 * np.max(np.abs(ref)) + 1e-13


@pytest.mark.parametrize("name", ["cfg1", "small_rect", "small_metal"])
def test_density_and_kernel(name):
    from oracle.response import HxcKernel
    rs, osys, ogs, perms = gpu_system(name)
    rho = to_host(rs.density())
    assert rel(rho, ogs.rho) < 1e-11
    kern = HxcKernel(osys, ogs.rho, xc=osys.spec.xc)
    v = random_field(osys.spec, 2)
    kv = to_host(rs.apply_kernel(to_dev(v)))
    assert rel(kv, kern.apply(v)) < 1e-11
    eps, occ, cf, fermi = rs.ground_state()
    for k in range(len(ogs.eps)):
        assert np.max(np.abs(eps[k] - ogs.eps[k])) == 0.0
        # both sides bisect the Fermi level to ~1e-15 Ha; |f'| <= 2/(4T) = 250
        assert np.max(np.abs(occ[k] - ogs.occ[k])) < 1e-11
