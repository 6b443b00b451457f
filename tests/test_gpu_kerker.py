"""GPU parity of the Kerker preconditioner (Sec. 3.3, eq. kerker) and of the
Kerker-preconditioned inexact GMRES (eq. precond_dyson) against the oracle:
T v element by element, the Lemma's facts (symmetric, positive, ||T|| = 1,
charge kept), and the preconditioned solve against a dense LU solve of
E drho = b and against the oracle's preconditioned Alg. 1."""
import numpy as np
import pytest

from gpu_common import gpu_system, rel, to_dev, to_host
from workloads import random_field

pytestmark = pytest.mark.gpu
ALPHA = 0.8


@pytest.mark.parametrize("name", ["tiny", "small_rect", "cfg2"])
def test_kerker_apply_matches_oracle(name):
    from oracle.response import kerker_apply
    from oracle.system import System
    from paper_2505_02319_amd import ResponseSystem
    from workloads import config
    print(f"kerker apply: {name}", flush=True)
    spec = config(name)
    osys = System(spec)
    rs = ResponseSystem(spec, ground_state=None)     # T needs no ground state
    u, v = random_field(spec, 4), random_field(spec, 5)
    for alpha in (ALPHA, 0.3):
        tv = to_host(rs.apply_kerker(to_dev(v), alpha))
        assert rel(tv, kerker_apply(osys, v, alpha)) < 1e-13
        tu = to_host(rs.apply_kerker(to_dev(u), alpha))
        assert abs(np.sum(u * tv) - np.sum(tu * v)) < 1e-13 * np.linalg.norm(u) * np.linalg.norm(v)
        assert 0 < np.sum(v * tv) <= np.sum(v * v)
        assert np.linalg.norm(tv) <= np.linalg.norm(v)
    one = np.ones(osys.n)
    assert np.max(np.abs(to_host(rs.apply_kerker(to_dev(one), ALPHA)) - 1.0)) < 1e-13
    rs.close()


@pytest.fixture(scope="module")
def metal_dense():
    from oracle.response import HxcKernel, SumOverStates, kerker_apply
    rs, osys, ogs, perms = gpu_system("tiny_metal")
    kern = HxcKernel(osys, ogs.rho, xc=1)
    chi = SumOverStates(osys, ogs).dense_matrix()
    kmat = np.zeros((osys.ng, osys.ng))
    tmat = np.zeros((osys.ng, osys.ng))
    for j in range(osys.ng):
        e = np.zeros(osys.ng)
        e[j] = 1
        kmat[:, j] = kern.apply(e.reshape(osys.n)).ravel()
        tmat[:, j] = kerker_apply(osys, e.reshape(osys.n), ALPHA).ravel()
    emat = np.eye(osys.ng) - chi @ kmat
    return rs, osys, ogs, kern, emat, tmat


@pytest.mark.parametrize("strategy", ["bal", "grt", "thm2", "D10n"])
@pytest.mark.parametrize("precision", [0, 1])
def test_kerker_solve_matches_dense(metal_dense, strategy, precision):
    """Pbal / Pgrt / Pthm2 / PD10n on the smeared two-k cell: the solution of
    T E x = T b equals the dense E^-1 b; the estimated (preconditioned)
    residual meets tau, and for the guaranteed strategies so does the true
    preconditioned residual ||T (b - E x)||."""
    from paper_2505_02319_amd import default_opts
    rs, osys, ogs, kern, emat, tmat = metal_dense
    print(f"kerker solve: {strategy} precision {precision}", flush=True)
    b = random_field(osys.spec, 2)
    x, st = rs.solve(to_dev(b), default_opts(strategy=strategy, tol=1e-8, kerker=1,
                                             kerker_alpha=ALPHA, precision=precision,
                                             want_true_residual=1))
    x = to_host(x).ravel()
    tau = 1e-8 * np.linalg.norm(b)
    r = b.ravel() - emat @ x
    assert st["est_res"] <= tau / 3
    assert abs(np.linalg.norm(r) - st["true_res"]) < 1e-3 * tau + 1e-13   # unpreconditioned
    if strategy in ("grt", "thm2"):
        assert np.linalg.norm(tmat @ r) <= tau
    if strategy != "D10n":
        assert rel(x, np.linalg.solve(emat, b.ravel())) < 1e-6


def test_kerker_solve_against_oracle_gmres():
    """small_metal (smeared, two k): the library's and the oracle's
    Kerker-preconditioned Alg. 1 (grt, tau = 1e-10 ||b||) reach the same drho."""
    from oracle.gmres import inexact_gmres
    from oracle.response import HxcKernel
    from paper_2505_02319_amd import default_opts
    print("kerker solve vs oracle Alg. 1: small_metal", flush=True)
    rs, osys, ogs, perms = gpu_system("small_metal")
    kern = HxcKernel(osys, ogs.rho, xc=osys.spec.xc)
    b = random_field(osys.spec, 2)
    tau = 1e-10 * np.linalg.norm(b)
    ref = inexact_gmres(osys, ogs, kern, b, tau, strategy="grt", kerker_alpha=ALPHA)
    x, st = rs.solve(to_dev(b), default_opts(strategy="grt", tol=1e-10, kerker=1,
                                             kerker_alpha=ALPHA))
    assert rel(to_host(x), ref.x) < 1e-8
    print(f"GMRES steps gpu {st['gmres_iters']} oracle {ref.iterations}; "
          f"N_ham gpu {st['n_ham']} oracle {ref.n_ham}")


def test_kerker_rejected_for_adjoint(metal_dense):
    from paper_2505_02319_amd import IkrError, default_opts
    rs = metal_dense[0]
    g = to_dev(random_field(metal_dense[1].spec, 3))
    with pytest.raises(IkrError) as e:
        rs.solve_adjoint(g, default_opts(kerker=1))
    assert e.value.code == 1
