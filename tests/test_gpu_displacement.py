"""GPU parity of the atom-displacement right-hand side b = chi0 dV0 (Sec. 4.1.2)
against the oracle: the local part of dV0 element by element, and b against
the oracle's sum over states with the nonlocal matrix elements added, its
Sternheimer route, and a central finite difference of the density in the
atom's position."""
import numpy as np
import pytest

from gpu_common import gpu_system, rel, to_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,atom,direction", [("tiny", 1, 0), ("cfg1", 0, 2),
                                                 ("small_metal", 1, 1), ("small_rect", 2, 2)])
def test_displacement_rhs_matches_oracle(name, atom, direction):
    from oracle.displacement import local_potential_derivative_position, nonlocal_action
    from oracle.response import SumOverStates
    print(f"displacement rhs: {name} atom {atom} dir {direction}", flush=True)
    rs, osys, ogs, perms = gpu_system(name)
    b, dv0, st = rs.displacement_rhs(atom, direction, cg_tol=1e-12)
    dvo = local_potential_derivative_position(osys, atom, direction)
    assert rel(to_host(dv0), dvo) < 1e-12
    ref = SumOverStates(osys, ogs).apply(dvo, dv_nl=nonlocal_action(osys, atom, direction))
    assert rel(to_host(b), ref) < 1e-9, rel(to_host(b), ref)
    assert st["n_ham"] > 0 and st["cg_unconverged"] == 0
    got = to_host(b)
    assert abs(got.sum()) < 1e-10 * np.abs(got).sum()   # the displacement moves no charge


def test_displacement_rhs_against_density_difference():
    """chi0 dV0 = d rho / dR for the fixed (non-self-consistent) potential:
    central difference of the oracle's dense ground-state density."""
    from oracle.displacement import density_fd
    from workloads import config
    rs, osys, ogs, perms = gpu_system("tiny")
    b, _, _ = rs.displacement_rhs(0, 1, cg_tol=1e-12)
    fd = density_fd(config("tiny"), 0, 1, h=1e-4)
    assert rel(to_host(b), fd) < 1e-6


def test_displacement_rhs_rejects_bad_arguments():
    from paper_2505_02319_amd import IkrError
    rs, osys, ogs, perms = gpu_system("tiny")
    for atom, d, tol in ((5, 0, 1e-8), (0, 3, 1e-8), (0, 0, 0.0), (-1, 0, 1e-8)):
        with pytest.raises(IkrError) as e:
            rs.displacement_rhs(atom, d, cg_tol=tol)
        assert e.value.code == 1
    b, _, _ = rs.displacement_rhs(0, 0, cg_tol=1e-10)   # the handle still works
    assert np.all(np.isfinite(to_host(b)))
