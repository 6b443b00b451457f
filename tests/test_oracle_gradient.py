"""Pins of the oracle's amplitude gradient: the 2n+1 third-order form against
a central finite difference of the (sum-over-states) chi0 in the amplitude,
and the full dL/dA against a central difference of the loss with dense
dielectric solves and the ground state recomputed at each amplitude."""
import numpy as np
import pytest

from oracle.gradient import amplitude_gradient, third_order_density
from oracle.groundstate import ground_state
from oracle.response import HxcKernel, SumOverStates
from oracle.system import System
from workloads import config, random_field

H = 1e-4


def _case(name):
    sys = System(config(name))
    return sys, ground_state(sys)


def _shifted(sys, atom, h):
    amp = np.array(sys.spec.amp, float)
    amp[atom] += h
    s2 = sys.with_amplitudes(amp)
    return s2, ground_state(s2)


@pytest.mark.parametrize("name", ["tiny", "tiny_k"])
def test_third_order_form_matches_fd_of_chi0(name):
    sys, gs = _case(name)
    u = random_field(sys.spec, 11)
    lam = random_field(sys.spec, 12)
    gden = third_order_density(sys, gs, u, lam, tol=1e-13)
    for atom in range(sys.spec.natoms):
        got = float(np.sum(sys.local_potential_derivative(atom) * gden))
        sp, gp = _shifted(sys, atom, H)
        sm, gm = _shifted(sys, atom, -H)
        cp = SumOverStates(sp, gp).apply(u)
        cm = SumOverStates(sm, gm).apply(u)
        fd = float(np.sum(lam * (cp - cm))) / (2 * H)
        assert abs(got - fd) < 1e-6 * max(abs(fd), 1e-12), (atom, got, fd)


def _loss_dense(sys, gs, b, t):
    kern = HxcKernel(sys, gs.rho, xc=sys.spec.xc)
    chi = SumOverStates(sys, gs).dense_matrix()
    kmat = np.zeros((sys.ng, sys.ng))
    for j in range(sys.ng):
        e = np.zeros(sys.ng)
        e[j] = 1
        kmat[:, j] = kern.apply(e.reshape(sys.n)).ravel()
    emat = np.eye(sys.ng) - chi @ kmat
    x = np.linalg.solve(emat, b.ravel())
    return float(np.sum((x - t.ravel()) ** 2)), x, emat, kern


def test_amplitude_gradient_matches_fd_of_loss():
    sys, gs = _case("tiny")
    assert sys.spec.xc == 1            # the f_x' term is exercised
    b = random_field(sys.spec, 2)
    t = random_field(sys.spec, 3)
    loss, x, emat, kern = _loss_dense(sys, gs, b, t)
    lam = np.linalg.solve(emat.T, 2 * (x - t.ravel()))
    grad = amplitude_gradient(sys, gs, kern, x, lam, tol=1e-13)
    for atom in range(sys.spec.natoms):
        sp, gp = _shifted(sys, atom, H)
        sm, gm = _shifted(sys, atom, -H)
        lp = _loss_dense(sp, gp, b, t)[0]
        lm = _loss_dense(sm, gm, b, t)[0]
        fd = (lp - lm) / (2 * H)
        assert abs(grad[atom] - fd) < 1e-6 * max(abs(fd), 1e-12), (atom, grad[atom], fd)
