"""Pins of the oracle's Hxc kernel and inexact GMRES (Alg. 1): closed-form
Hartree action, dense LU solve of E drho = b on a tiny cell, the guarantee of
Theorem 2 for the grt strategy, Lemma 2, the monotone estimated residual,
and the forced extra restart of Alg. 1."""
import numpy as np
import pytest

from oracle.gmres import STRATEGIES, inexact_gmres, true_residual
from oracle.response import HxcKernel, SumOverStates, apply_dielectric
from workloads import random_field


def _dense_k(kern, ng, shape):
    kmat = np.zeros((ng, ng))
    for j in range(ng):
        e = np.zeros(ng)
        e[j] = 1.0
        kmat[:, j] = kern.apply(e.reshape(shape)).ravel()
    return kmat


def test_hartree_closed_form(oracle_case):
    sys, gs = oracle_case("small_rect")
    kern = HxcKernel(sys, gs.rho, xc=0)
    idx = np.meshgrid(*[np.arange(m) / m for m in sys.n], indexing="ij")
    for q in [(1, 0, 0), (0, 2, 1), (1, -1, 3)]:
        phase = 2 * np.pi * sum(qi * xi for qi, xi in zip(q, idx))
        qq = sum((qi * bi) ** 2 for qi, bi in zip(q, sys.b))
        got = kern.apply(np.cos(phase))
        assert np.max(np.abs(got - 4 * np.pi / qq * np.cos(phase))) < 1e-12 * 4 * np.pi / qq
    assert np.max(np.abs(kern.apply(np.ones(sys.n)))) < 1e-12


@pytest.fixture(scope="module")
def tiny_dense():
    from oracle.groundstate import ground_state
    from oracle.system import System
    from workloads import config
    sys = System(config("tiny"))
    gs = ground_state(sys)
    kern = HxcKernel(sys, gs.rho, xc=1)
    chi = SumOverStates(sys, gs).dense_matrix()
    kmat = _dense_k(kern, sys.ng, sys.n)
    emat = np.eye(sys.ng) - chi @ kmat
    return sys, gs, kern, kmat, emat


def test_kernel_symmetric(tiny_dense):
    sys, gs, kern, kmat, emat = tiny_dense
    assert np.max(np.abs(kmat - kmat.T)) < 1e-12 * np.max(np.abs(kmat))


@pytest.mark.parametrize("strategy", STRATEGIES)
def test_gmres_matches_dense_solve(tiny_dense, strategy):
    sys, gs, kern, kmat, emat = tiny_dense
    b = random_field(sys.spec, 2)
    tau = 1e-8 * np.linalg.norm(b)
    ref = np.linalg.solve(emat, b.ravel())
    res = inexact_gmres(sys, gs, kern, b, tau, strategy=strategy, m=20)
    x = res.x.ravel()
    true_r = np.linalg.norm(b.ravel() - emat @ x)
    # the Sternheimer-applied operator equals the dense one
    assert abs(true_r - true_residual(sys, gs, kern, b, res.x)) < 1e-12
    cond = np.linalg.cond(emat)
    assert np.linalg.norm(x - ref) <= cond * 10 * true_r + 1e-14
    if strategy in ("grt", "thm2"):
        assert true_r <= tau                      # Theorem 2 guarantee
    if strategy in ("bal", "grt", "thm2"):
        assert true_r <= 3 * tau
    # estimated residual decreases monotonically inside a cycle
    for a_, b_ in zip(res.history, res.history[1:]):
        if a_["cycle"] == b_["cycle"]:
            assert b_["est_res"] <= a_["est_res"] * (1 + 1e-12)


def test_lemma2_and_zero_mean_solution(tiny_dense):
    sys, gs, kern, kmat, emat = tiny_dense
    b = random_field(sys.spec, 2)
    tau = 1e-10 * np.linalg.norm(b)
    res = inexact_gmres(sys, gs, kern, b, tau, strategy="grt", m=20)
    h = res.hessenberg
    sig = np.linalg.svd(h, compute_uv=False)[-1]
    m = h.shape[1]
    # residual history of the last cycle: ||r~_0|| = beta, then est_res
    last = [res.beta] + [x["est_res"] for x in res.history[-m:]]
    for i in range(m):
        assert abs(res.y[i]) <= last[i] / sig * (1 + 1e-10)
    # charge conservation: b has zero mean and so has drho
    assert abs(res.x.sum()) < 1e-9 * np.abs(res.x).sum()


def test_overestimated_s_forces_restart(tiny_dense):
    sys, gs, kern, kmat, emat = tiny_dense
    b = random_field(sys.spec, 2)
    tau = 1e-8 * np.linalg.norm(b)
    res = inexact_gmres(sys, gs, kern, b, tau, strategy="bal", m=20, s0=1e6)
    assert res.restarts >= 1
    assert res.s_final < 1e6
    assert np.linalg.norm(b.ravel() - emat @ res.x.ravel()) <= 3 * tau


def test_static_tolerance_loses_accuracy(tiny_dense):
    """With a loose static tolerance the estimated residual reaches tau while
    the true residual does not (the failure mode of Sec. 3.1)."""
    sys, gs, kern, kmat, emat = tiny_dense
    b = random_field(sys.spec, 2)
    tau = 1e-9 * np.linalg.norm(b)
    res = inexact_gmres(sys, gs, kern, b, tau * 1e4, strategy="D10", m=20)
    res_small = inexact_gmres(sys, gs, kern, b, tau, strategy="D10", m=20)
    true_r = np.linalg.norm(b.ravel() - emat @ res_small.x.ravel())
    assert res_small.est_res <= tau / 3
    assert true_r > res_small.est_res
