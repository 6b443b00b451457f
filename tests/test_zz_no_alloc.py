"""The entry point that allocates no device memory (ikr_apply_hamiltonian_noalloc)
against ikr_apply_hamiltonian, through the C ABI: two calls in a row, the
second with fewer vectors (the shared work space keeps the first call's
contents), each compared with the allocating entry point and with the oracle's
dense H_k; sizes beyond the fixed work space are rejected."""
import numpy as np
import pytest

from gpu_common import gpu_system, rel, to_dev, to_host

pytestmark = pytest.mark.gpu


def _vectors(rng, nvec, nb, nb_max):
    x = np.zeros((nvec, nb_max), np.complex128)
    x[:, :nb] = rng.standard_normal((nvec, nb)) + 1j * rng.standard_normal((nvec, nb))
    return x


@pytest.mark.parametrize("name", ["small_rect", "small_metal"])
def test_noalloc_matches_allocating_entry_point(name):
    print(f"no-alloc H apply: {name}", flush=True)
    rs, osys, ogs, perms = gpu_system(name)
    inf = rs.info()
    rng = np.random.default_rng(23)
    for k in range(min(inf.nk, 2)):
        nb = len(perms[k])
        h = osys.dense_h(k)
        for nvec in (37, 5):          # a ragged tile tail, then a smaller call
            x = _vectors(rng, nvec, nb, inf.nb_max)
            xd = to_dev(x)
            y_ref = to_host(rs.apply_hamiltonian(k, xd))
            y_na = to_host(rs.apply_hamiltonian_noalloc(k, xd))
            assert rel(y_na[:, :nb], y_ref[:, :nb]) < 1e-14, (name, k, nvec)
            xo = np.zeros((nvec, nb), np.complex128)
            xo[:, perms[k]] = x[:, :nb]
            yo = (h @ xo.T).T
            assert rel(y_na[:, :nb], yo[:, perms[k]]) < 1e-12, (name, k, nvec)
    rs.close()


def test_noalloc_rejects_sizes_beyond_the_work_space():
    from paper_2505_02319_amd import IkrError
    print("no-alloc H apply: size limit on cfg2", flush=True)
    import torch
    from paper_2505_02319_amd import ResponseSystem
    from workloads import config
    rs = ResponseSystem(config("cfg2"), ground_state=None)   # no ground state needed
    inf = rs.info()
    g = torch.Generator(device="cuda").manual_seed(5)
    x = torch.randn((4096, inf.nb_max), dtype=torch.complex128, device="cuda", generator=g)
    with pytest.raises(IkrError) as e:
        rs.apply_hamiltonian_noalloc(0, x)
    assert e.value.code == 1 and "MiB" in str(e.value)
    # a size that fits still works on the same handle, and matches
    nb0 = rs.basis(0).shape[0]
    y = rs.apply_hamiltonian_noalloc(0, x[:3].contiguous())
    y2 = rs.apply_hamiltonian(0, x[:3].contiguous())
    assert torch.equal(y[:, :nb0], y2[:, :nb0])
    rs.close()
