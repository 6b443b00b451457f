"""Pins of the oracle's Kerker preconditioner (Sec. 3.3, eq. kerker, Lemma
kerker_properties), the Kerker-preconditioned inexact GMRES
(eq. precond_dyson), and the atom-displacement perturbation (Sec. 4.1.2):
closed forms, the Lemma's spectral facts on the dense matrix, dense solves,
and finite differences in the atom position."""
import numpy as np
import pytest

from oracle.displacement import (density_fd, local_potential_derivative_position,
                                 nonlocal_action, projector_pair)
from oracle.gmres import inexact_gmres
from oracle.response import (HxcKernel, SumOverStates, chi0_sternheimer, kerker_apply,
                             kerker_symbol)
from oracle.system import System
from workloads import config, random_field

ALPHA = 0.8


def _dense(op, sys):
    m = np.zeros((sys.ng, sys.ng))
    for j in range(sys.ng):
        e = np.zeros(sys.ng)
        e[j] = 1.0
        m[:, j] = op(e.reshape(sys.n)).ravel()
    return m


@pytest.fixture(scope="module")
def tiny_t():
    sys = System(config("tiny"))
    return sys, _dense(lambda v: kerker_apply(sys, v, ALPHA), sys)


def test_kerker_lemma_properties(tiny_t):
    """T is symmetric positive definite with largest eigenvalue 1 and
    ||T|| = 1 (Lemma kerker_properties); the constant vector is its
    eigenvector for 1 (charge conservation)."""
    sys, t = tiny_t
    assert np.max(np.abs(t - t.T)) < 1e-14
    lam = np.linalg.eigvalsh(0.5 * (t + t.T))
    assert lam.min() > 0
    assert abs(lam.max() - 1.0) < 1e-13
    assert abs(np.linalg.norm(t, 2) - 1.0) < 1e-13
    one = np.ones(sys.ng)
    assert np.max(np.abs(t @ one - one)) < 1e-13
    # smallest eigenvalue = D at the smallest nonzero |G| (= min b_i)
    bmin = np.min(sys.b)
    assert abs(lam.min() - bmin ** 2 / (bmin ** 2 + ALPHA ** 2)) < 1e-13


def test_kerker_plane_wave_closed_form():
    """T cos(G.r) = |G|^2/(|G|^2 + alpha^2) cos(G.r) for G != 0: the plane
    waves are T's eigenvectors, with the eigenvalues of D."""
    sys = System(config("small_rect"))
    idx = np.meshgrid(*[np.arange(m) / m for m in sys.n], indexing="ij")
    for q in [(1, 0, 0), (0, 2, 1), (1, -1, 3)]:
        v = np.cos(2 * np.pi * sum(qi * xi for qi, xi in zip(q, idx)))
        qq = sum((qi * bi) ** 2 for qi, bi in zip(q, sys.b))
        assert np.max(np.abs(kerker_apply(sys, v, ALPHA) - qq / (qq + ALPHA ** 2) * v)) < 1e-13


def test_kerker_equals_symbol_with_unit_zero_mode(tiny_t):
    """The proof of the Lemma: eq. kerker equals W^-1 D' W with D'(0) = 1 and
    D' = D elsewhere (the form a GPU applies as one FFT pair)."""
    sys, t = tiny_t
    d = kerker_symbol(sys, ALPHA)
    assert d.flat[0] == 0.0
    d1 = d.copy()
    d1.flat[0] = 1.0
    v = random_field(sys.spec, 9) + 0.3
    alt = np.fft.ifftn(d1 * np.fft.fftn(v)).real
    assert np.max(np.abs(alt.ravel() - t @ v.ravel())) < 1e-14


@pytest.fixture(scope="module")
def metal_dense():
    from oracle.groundstate import ground_state
    sys = System(config("tiny_metal"))
    gs = ground_state(sys)
    kern = HxcKernel(sys, gs.rho, xc=1)
    chi = SumOverStates(sys, gs).dense_matrix()
    kmat = _dense(kern.apply, sys)
    emat = np.eye(sys.ng) - chi @ kmat
    tmat = _dense(lambda v: kerker_apply(sys, v, ALPHA), sys)
    return sys, gs, kern, emat, tmat


@pytest.mark.parametrize("strategy", ["grt", "bal", "thm2"])
def test_kerker_gmres_meets_preconditioned_tolerance(metal_dense, strategy):
    """Alg. 1 on T E drho = T b: since ||T|| = 1, Theorem 2's strategies bound
    the preconditioned true residual ||T (b - E x)|| by tau (grt, thm2; bal
    within its 3 tau), and the solution is that of the dense system."""
    sys, gs, kern, emat, tmat = metal_dense
    b = random_field(sys.spec, 2)
    tau = 1e-9 * np.linalg.norm(b)
    res = inexact_gmres(sys, gs, kern, b, tau, strategy=strategy, m=20, kerker_alpha=ALPHA)
    x = res.x.ravel()
    pres = np.linalg.norm(tmat @ (b.ravel() - emat @ x))
    assert pres <= (tau if strategy != "bal" else 3 * tau)
    ref = np.linalg.solve(emat, b.ravel())
    assert np.linalg.norm(x - ref) <= np.linalg.cond(tmat @ emat) * 10 * pres + 1e-14
    # the preconditioner changes the Krylov space: fewer GMRES steps than
    # without it on this metal
    plain = inexact_gmres(sys, gs, kern, b, tau, strategy=strategy, m=20)
    assert res.iterations <= plain.iterations


# ---------------------------------------------------------------- displacement
def test_local_potential_position_derivative_is_fd():
    spec = config("small_rect")
    sys = System(spec)
    h = 1e-5
    for atom, d in [(0, 0), (1, 2), (3, 1)]:
        got = local_potential_derivative_position(sys, atom, d)
        vals = []
        for sgn in (1.0, -1.0):
            pos = np.array(spec.frac_pos, float)
            pos[atom, d] += sgn * h / spec.lattice[d]
            vals.append(System(spec.with_(frac_pos=pos)).vloc)
        fd = (vals[0] - vals[1]) / (2 * h)
        assert np.max(np.abs(got - fd)) < 1e-7 * np.max(np.abs(got))


def test_projector_position_derivative_is_fd():
    spec = config("small_k")
    sys = System(spec)
    h = 1e-5
    for ik in range(len(sys.bases)):
        p, dp = projector_pair(sys, ik, 1, 2)
        vals = []
        for sgn in (1.0, -1.0):
            pos = np.array(spec.frac_pos, float)
            pos[1, 2] += sgn * h / spec.lattice[2]
            vals.append(System(spec.with_(frac_pos=pos)).projectors(ik)[1])
        fd = (vals[0] - vals[1]) / (2 * h)
        assert np.max(np.abs(dp - fd)) < 1e-8 * np.max(np.abs(dp))


@pytest.mark.parametrize("name,atom,d", [("tiny", 1, 0), ("tiny_metal", 0, 2)])
def test_displacement_response_three_routes(name, atom, d, oracle_case):
    """chi0 dV0 by sum over states = by Sternheimer = d rho / dR_a by finite
    differences of the recomputed ground state."""
    sys, gs = oracle_case(name)
    dv = local_potential_derivative_position(sys, atom, d)
    nl = nonlocal_action(sys, atom, d)
    sos = SumOverStates(sys, gs).apply(dv, dv_nl=nl)
    st = chi0_sternheimer(sys, gs, dv, 1e-12, dv_nl=nl)
    fd = density_fd(sys.spec, atom, d)
    nrm = np.linalg.norm(sos)
    assert np.linalg.norm(st - sos) < 1e-9 * nrm
    assert np.linalg.norm(fd - sos) < 2e-8 * nrm
    # the nonlocal part matters: dropping it misses the finite difference
    loc_only = SumOverStates(sys, gs).apply(dv)
    assert np.linalg.norm(fd - loc_only) > 1e-3 * nrm
    # a displacement moves charge but does not create it
    assert abs(sos.sum()) < 1e-10 * np.abs(sos).sum()
