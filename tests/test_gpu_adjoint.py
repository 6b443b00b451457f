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
