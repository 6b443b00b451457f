"""Helpers shared by the GPU parity tests: build a library system from a
workload, import the oracle's ground state in the library's basis order, and
move grid vectors between numpy and the device."""
import numpy as np

from conftest import cached


def reorder_map(lib_miller, oracle_miller):
    """perm with lib_basis[i] == oracle_basis[perm[i]] (by Miller index)."""
    index = {tuple(m): i for i, m in enumerate(oracle_miller)}
    return np.array([index[tuple(m)] for m in lib_miller])


def oracle_state(name):
    from oracle.groundstate import ground_state
    from oracle.system import System
    from workloads import config

    def make():
        s = System(config(name))
        return s, ground_state(s)
    return cached(("gs", name), make)


def gpu_system(name, ground_state="oracle"):
    """(ResponseSystem, oracle System, oracle GroundState, perms)."""
    from paper_2505_02319_amd import ResponseSystem
    from workloads import config
    spec = config(name)
    osys, ogs = oracle_state(name)
    if ground_state == "oracle":
        rs = ResponseSystem(spec, ground_state=None)
        inf = rs.info()
        perms = [reorder_map(rs.basis(k), osys.bases[k].miller) for k in range(inf.nk)]
        eps = np.array([ogs.eps[k] for k in range(inf.nk)])
        cf = np.zeros((inf.nk, inf.nbands, inf.nb_max), np.complex128)
        for k in range(inf.nk):
            cf[k, :, :len(perms[k])] = ogs.phi[k][:, perms[k]]
        rs.import_ground_state(eps, cf)
    else:
        rs = ResponseSystem(spec, ground_state="compute")
        inf = rs.info()
        perms = [reorder_map(rs.basis(k), osys.bases[k].miller) for k in range(inf.nk)]
    return rs, osys, ogs, perms


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def to_host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))
