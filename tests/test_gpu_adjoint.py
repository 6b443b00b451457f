"""GPU parity of the adjoint path: E^T v against the dense transpose, the
adjoint inexact GMRES against a dense solve with E^T, and dL/db through the
torch.autograd.Function against the dense gradient and a finite difference."""
import numpy as np
import pytest

from gpu_common import gpu_system, rel, to_dev, to_host
from workloads import random_field

pytestmark = pytest.mark.gpu


def _dense(name):
    from oracle.response import HxcKernel, SumOverStates
    rs, osys, ogs, perms = gpu_system(name)
    kern = HxcKernel(osys, ogs.rho, xc=1)
    chi = SumOverStates(osys, ogs).dense_matrix()
    kmat = np.zeros((osys.ng, osys.ng))
    for j in range(osys.ng):
        e = np.zeros(osys.ng)
        e[j] = 1
        kmat[:, j] = kern.apply(e.reshape(osys.n)).ravel()
    return rs, osys, np.eye(osys.ng) - chi @ kmat


@pytest.fixture(scope="module")
def tiny_dense():
    return _dense("tiny")


@pytest.mark.parametrize("name", ["tiny", "tiny_metal"])
def test_dielectric_adjoint_matches_dense_transpose(name):
    from paper_2505_02319_amd import default_opts
    rs, osys, emat = _dense(name)
    v = random_field(osys.spec, 5)
    ev, st = rs.apply_dielectric_adjoint(to_dev(v), 1e-13, default_opts(strategy="fixed"))
    assert rel(to_host(ev), emat.T @ v.ravel()) < 1e-9
    assert abs(st["knorm_last"] - np.linalg.norm(v)) < 1e-12 * np.linalg.norm(v)


@pytest.mark.parametrize("strategy", ["bal", "grt", "thm2"])
def test_solve_adjoint_matches_dense(tiny_dense, strategy):
    from paper_2505_02319_amd import default_opts
    rs, osys, emat = tiny_dense
    g = random_field(osys.spec, 4)
    lam, st = rs.solve_adjoint(to_dev(g), default_opts(strategy=strategy, tol=1e-8,
                                                      want_true_residual=1))
    lam = to_host(lam).ravel()
    tau = 1e-8 * np.linalg.norm(g)
    true_r = np.linalg.norm(g.ravel() - emat.T @ lam)
    assert abs(true_r - st["true_res"]) < 1e-3 * tau + 1e-13
    if strategy in ("grt", "thm2"):
        assert true_r <= tau
    assert true_r <= 3 * tau
    assert rel(lam, np.linalg.solve(emat.T, g.ravel())) < 1e-7


def test_solve_adjoint_mixed_precision(tiny_dense):
    from paper_2505_02319_amd import default_opts
    rs, osys, emat = tiny_dense
    g = random_field(osys.spec, 4)
    lam, st = rs.solve_adjoint(to_dev(g), default_opts(strategy="grt", tol=1e-8, precision=1))
    lam = to_host(lam).ravel()
    assert np.linalg.norm(g.ravel() - emat.T @ lam) <= 1e-8 * np.linalg.norm(g)
    assert st["n_ham_fp32"] > 0


def test_autograd_gradient_of_quadratic_loss(tiny_dense):
    """L = ||drho - t||^2: dL/db = 2 E^-T (E^-1 b - t) (dense), and the
    directional derivative equals the central difference (exact for a
    quadratic up to the solve tolerance)."""
    import torch
    from paper_2505_02319_amd import default_opts, dyson_solve
    rs, osys, emat = tiny_dense
    b = to_dev(random_field(osys.spec, 2)).requires_grad_(True)
    t = to_dev(random_field(osys.spec, 3))
    opts = default_opts(strategy="grt", tol=1e-11)
    x = dyson_solve(b, rs, opts)
    loss = torch.sum((x - t) ** 2)
    loss.backward()
    grad = to_host(b.grad).ravel()
    bh, th = to_host(b.detach()).ravel(), to_host(t).ravel()
    ref = 2 * np.linalg.solve(emat.T, np.linalg.solve(emat, bh) - th)
    assert rel(grad, ref) < 1e-8
    d = random_field(osys.spec, 7).ravel()
    h = 1e-2

    def lossval(bv):
        xv, _ = rs.solve(to_dev(bv.reshape(osys.n)), opts)
        return float(np.sum((to_host(xv).ravel() - th) ** 2))
    fd = (lossval(bh + h * d) - lossval(bh - h * d)) / (2 * h)
    assert abs(fd - grad @ d) < 1e-7 * abs(fd)


def test_solve_adjoint_cfg1_against_oracle_gmres():
    from oracle.gmres import inexact_gmres
    from oracle.response import HxcKernel
    from paper_2505_02319_amd import default_opts
    rs, osys, ogs, perms = gpu_system("cfg1")
    kern = HxcKernel(osys, ogs.rho, xc=1)
    g = random_field(osys.spec, 4)
    tau = 1e-10 * np.linalg.norm(g)
    ref = inexact_gmres(osys, ogs, kern, g, tau, strategy="grt", adjoint=True)
    lam, st = rs.solve_adjoint(to_dev(g), default_opts(strategy="grt", tol=1e-10))
    assert rel(to_host(lam), ref.x) < 1e-8
    assert st["gmres_iters"] > 0


def _gpu_system_for(spec):
    """Library system for an arbitrary spec with the oracle's ground state."""
    from gpu_common import reorder_map
    from oracle.groundstate import ground_state
    from oracle.system import System
    from paper_2505_02319_amd import ResponseSystem
    osys = System(spec)
    ogs = ground_state(osys)
    rs = ResponseSystem(spec, ground_state=None)
    inf = rs.info()
    perms = [reorder_map(rs.basis(k), osys.bases[k].miller) for k in range(inf.nk)]
    eps = np.array([ogs.eps[k] for k in range(inf.nk)])
    cf = np.zeros((inf.nk, inf.nbands, inf.nb_max), np.complex128)
    for k in range(inf.nk):
        cf[k, :, :len(perms[k])] = ogs.phi[k][:, perms[k]]
    rs.import_ground_state(eps, cf)
    return rs, osys, ogs


@pytest.mark.parametrize("name", ["tiny", "tiny_k"])
def test_grad_amplitudes_matches_oracle(name):
    """The library's dL/dA (third-order form + f_x' term) against the oracle's,
    both from the same drho and lambda (dense solves)."""
    from oracle.gradient import amplitude_gradient
    from oracle.response import HxcKernel
    rs, osys, emat = _dense(name)
    from gpu_common import oracle_state
    _, ogs = oracle_state(name)
    b = random_field(osys.spec, 2)
    t = random_field(osys.spec, 3)
    x = np.linalg.solve(emat, b.ravel())
    lam = np.linalg.solve(emat.T, 2 * (x - t.ravel()))
    got, st = rs.grad_amplitudes(to_dev(x.reshape(osys.n)), to_dev(lam.reshape(osys.n)), 1e-13)
    kern = HxcKernel(osys, ogs.rho, xc=osys.spec.xc)
    ref = amplitude_gradient(osys, ogs, kern, x, lam, tol=1e-13)
    assert rel(got, ref) < 1e-8, (got, ref)
    assert st["n_ham"] > 0


def test_autograd_amplitude_gradient_matches_fd():
    """dL/dA through the autograd Function (adjoint GMRES + amplitude
    gradient) against central differences of the library's own loss with the
    ground state recomputed at A +- h (L = ||drho - t||^2)."""
    import torch
    from paper_2505_02319_amd import default_opts, dyson_solve
    from workloads import config
    spec = config("tiny")
    rs, osys, ogs = _gpu_system_for(spec)
    b = to_dev(random_field(spec, 2))
    t = to_dev(random_field(spec, 3))
    opts = default_opts(strategy="grt", tol=1e-12)
    amp = torch.tensor(np.asarray(spec.amp, float), requires_grad=True)
    x = dyson_solve(b, rs, opts, amplitudes=amp)
    loss = torch.sum((x - t) ** 2)
    loss.backward()
    grad = amp.grad.numpy()
    h = 1e-4
    for atom in range(spec.natoms):
        vals = []
        for sgn in (1, -1):
            a2 = np.array(spec.amp, float)
            a2[atom] += sgn * h
            rs2, _, _ = _gpu_system_for(spec.with_(amp=a2))
            x2, _ = rs2.solve(b, opts)
            vals.append(float(torch.sum((x2 - t) ** 2)))
            rs2.close()
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(grad[atom] - fd) < 1e-5 * abs(fd), (atom, grad[atom], fd)


def test_grad_amplitudes_rejects_smeared_occupations():
    from paper_2505_02319_amd import IkrError
    rs, osys, ogs, perms = gpu_system("tiny_metal")
    v = to_dev(random_field(osys.spec, 2))
    with pytest.raises(IkrError):
        rs.grad_amplitudes(v, v, 1e-12)


@pytest.mark.parametrize("name", ["small_rect", "cfg1"])
def test_grad_amplitudes_matches_oracle_mid_size(name):
    """dL/dA on larger cells (small_rect: 20 x 20 x 36 grid, 2 k, 4 atoms; cfg1:
    20^3), from the library's own drho = E^-1 b and lambda = E^-T 2 (drho - t)
    (grt, 1e-11): the library's gradient against the oracle's third-order form
    on the same drho and lambda (Sternheimer CG at 1e-13 on both sides)."""
    from oracle.gradient import amplitude_gradient
    from oracle.response import HxcKernel
    from paper_2505_02319_amd import default_opts
    print(f"amplitude gradient vs oracle: {name}", flush=True)
    rs, osys, ogs, perms = gpu_system(name)
    b = random_field(osys.spec, 2)
    t = random_field(osys.spec, 3)
    opts = default_opts(strategy="grt", tol=1e-11)
    x, _ = rs.solve(to_dev(b), opts)
    lam, _ = rs.solve_adjoint(2 * (x - to_dev(t)), opts)
    got, st = rs.grad_amplitudes(x, lam, 1e-13)
    kern = HxcKernel(osys, ogs.rho, xc=osys.spec.xc)
    ref = amplitude_gradient(osys, ogs, kern, to_host(x), to_host(lam), tol=1e-13)
    assert rel(got, ref) < 1e-8, (got, ref)
