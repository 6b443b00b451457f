"""Edge cases and error paths through the C ABI, and properties of the
response at the full size of the 48^3 cell in the bench's configuration
(properties that hold at any size, where the oracle cannot follow)."""
import ctypes as C

import numpy as np
import pytest

from gpu_common import gpu_system, rel, to_dev, to_host
from workloads import config, random_field

pytestmark = pytest.mark.gpu


def test_zero_right_hand_side():
    """b = 0: drho = 0 with no GMRES step and no H application (and the same
    for the adjoint)."""
    from paper_2505_02319_amd import default_opts
    rs, osys, ogs, perms = gpu_system("tiny")
    z = to_dev(np.zeros(osys.n))
    for solve in (rs.solve, rs.solve_adjoint):
        x, st = solve(z, default_opts(strategy="grt", tol=1e-8, want_true_residual=1))
        assert np.all(to_host(x) == 0)
        assert st["gmres_iters"] == 0 and st["n_ham"] == 0


def test_dielectric_when_the_kernel_annihilates_v():
    """nu = ||K v|| = 0 gives E v = v with no CG work: v = 0, and a constant
    field under the Hartree-only kernel (its G = 0 entry is zero)."""
    from paper_2505_02319_amd import ResponseSystem, default_opts
    rs, osys, ogs, perms = gpu_system("tiny")
    z = to_dev(np.zeros(osys.n))
    ev, st = rs.apply_dielectric(z, 1e-10, default_opts(strategy="fixed"))
    assert np.all(to_host(ev) == 0) and st["n_ham"] == 0
    rh = ResponseSystem(config("tiny").with_(name="tiny_hartree", xc=0), ground_state="compute")
    try:
        c = np.full(osys.n, 0.25)
        ev, st = rh.apply_dielectric(to_dev(c), 1e-10, default_opts(strategy="fixed"))
        assert np.array_equal(to_host(ev), c)
        assert st["n_ham"] == 0 and st["knorm_last"] == 0
    finally:
        rh.close()


def test_invalid_arguments_are_rejected():
    from paper_2505_02319_amd import IkrError, default_opts
    from paper_2505_02319_amd.binding import Stats, lib
    rs, osys, ogs, perms = gpu_system("tiny")
    b = random_field(osys.spec, 2)
    bad = b.copy()
    bad[0, 0, 0] = np.nan
    with pytest.raises(IkrError) as e:
        rs.solve(to_dev(bad), default_opts(strategy="grt"))
    assert e.value.code == 5                                   # IKR_E_NAN
    with pytest.raises(IkrError) as e:
        rs.apply_dielectric(to_dev(bad), 1e-8, default_opts(strategy="fixed"))
    assert e.value.code == 5
    for kw in (dict(restart_m=0), dict(tol=-1.0), dict(precision=2), dict(cg_max_iter=0),
               dict(strategy=99), dict(s0=0.0)):
        with pytest.raises(IkrError) as e:
            rs.solve(to_dev(b), default_opts(**kw))
        assert e.value.code == 1, kw                           # IKR_E_ARG
    o, st = default_opts(), Stats()
    assert lib().ikr_solve_response(rs.h, None, None, C.byref(o), C.byref(st)) == 1
    assert lib().ikr_apply_chi0(rs.h, None, None, 1e-8, None, C.byref(st)) == 1
    assert lib().ikr_solve_response(None, None, None, C.byref(o), C.byref(st)) == 1
    # the handle still works after the rejected calls
    x, st2 = rs.solve(to_dev(b), default_opts(strategy="grt", tol=1e-8))
    assert np.all(np.isfinite(to_host(x))) and st2["gmres_iters"] > 0


@pytest.fixture(scope="module")
def cfg2_system():
    from paper_2505_02319_amd import ResponseSystem
    rs = ResponseSystem(config("cfg2"), ground_state="compute")
    yield rs
    rs.close()


def test_cfg2_chi0_symmetric_negative_and_charge_conserving(cfg2_system):
    """chi0 at full size: <u, chi0 v> = <chi0 u, v>, <v, chi0 v> < 0, and
    sum_r chi0 v = 0 (an insulator conserves charge)."""
    rs = cfg2_system
    spec = config("cfg2")
    u, v = random_field(spec, 4), random_field(spec, 5)
    cu, st_u = rs.apply_chi0(to_dev(u), cg_tol=1e-12)
    cv, st_v = rs.apply_chi0(to_dev(v), cg_tol=1e-12)
    cu, cv = to_host(cu), to_host(cv)
    assert st_u["cg_unconverged"] == 0 and st_v["cg_unconverged"] == 0
    lhs, rhs_ = float(np.sum(u * cv)), float(np.sum(cu * v))
    assert abs(lhs - rhs_) <= 1e-8 * np.linalg.norm(u) * np.linalg.norm(cv)
    assert float(np.sum(v * cv)) < 0
    assert abs(float(np.sum(cv))) <= 1e-10 * float(np.sum(np.abs(cv)))


def test_cfg2_solve_meets_tolerance_mixed_and_fp64(cfg2_system):
    """The bench's solve (grt, tau = 1e-8 ||b||, mixed precision, extra-band
    split) keeps the grt guarantee at full size and agrees with the FP64-CG
    solve; the graph-replayed solve agrees too."""
    from paper_2505_02319_amd import default_opts
    from workloads import B_SEED
    rs = cfg2_system
    b = to_dev(random_field(config("cfg2"), B_SEED))
    bnorm = float(np.linalg.norm(to_host(b)))
    kw = dict(strategy="grt", tol=1e-8, tol_is_relative=1, schur=1, want_true_residual=1)
    xm, stm = rs.solve(b, default_opts(precision=1, **kw))
    x64, st64 = rs.solve(b, default_opts(precision=0, **kw))
    xg, stg = rs.solve(b, default_opts(precision=1, batching=1, **kw))
    for st in (stm, st64, stg):
        assert st["true_res"] <= 1e-8 * bnorm
    assert stm["n_ham_fp32"] > 0 and st64["n_ham_fp32"] == 0
    assert rel(to_host(xm), to_host(x64)) < 1e-7
    assert rel(to_host(xg), to_host(xm)) < 1e-7


def test_cfg3_chi0_properties_two_launch_iteration_end():
    """chi0 on the 16-atom cell at full size (8 k x 32 bands, spheres of
    ~74k coefficients): the batch has more per-slot partials than one block
    of the fused iteration end takes, so every CG iteration ends with the
    separate finish and compaction launches.  Checked by the properties that
    hold at any size: symmetry, negativity and charge conservation."""
    from paper_2505_02319_amd import ResponseSystem
    spec = config("cfg3")
    rs = ResponseSystem(spec, ground_state="compute")
    try:
        u, v = random_field(spec, 4), random_field(spec, 5)
        cu, st_u = rs.apply_chi0(to_dev(u), cg_tol=1e-11)
        cv, st_v = rs.apply_chi0(to_dev(v), cg_tol=1e-11)
        cu, cv = to_host(cu), to_host(cv)
        assert st_u["cg_unconverged"] == 0 and st_v["cg_unconverged"] == 0
        lhs, rhs_ = float(np.sum(u * cv)), float(np.sum(cu * v))
        assert abs(lhs - rhs_) <= 1e-7 * np.linalg.norm(u) * np.linalg.norm(cv)
        assert float(np.sum(v * cv)) < 0
        assert abs(float(np.sum(cv))) <= 1e-9 * float(np.sum(np.abs(cv)))
    finally:
        rs.close()
