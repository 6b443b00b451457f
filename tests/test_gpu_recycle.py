"""Sternheimer warm starts across dielectric applications (solver option
recycle): each band's CG starts from the least-squares combination of its
solutions for the earlier right-hand sides of the same solve.  The operator
of every band is the same at each GMRES step, so the converged result must
not change beyond the tolerances: checked against dense LU solves and the
oracle's Alg. 1, in FP64 and mixed precision, with and without Kerker."""
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
def dense_cells():
    return {name: _dense(name) for name in ("tiny", "tiny_metal")}


@pytest.mark.parametrize("name,strategy,precision,kerker",
                         [("tiny", "grt", 0, 0), ("tiny", "bal", 1, 0),
                          ("tiny_metal", "grt", 1, 1), ("tiny_metal", "thm2", 0, 0)])
def test_recycled_solve_matches_dense(dense_cells, name, strategy, precision, kerker):
    from paper_2505_02319_amd import default_opts
    print(f"recycle: {name} {strategy} precision {precision} kerker {kerker}", flush=True)
    rs, osys, emat = dense_cells[name]
    b = random_field(osys.spec, 2)
    kw = dict(strategy=strategy, tol=1e-8, precision=precision, kerker=kerker,
              want_true_residual=1)
    x0, st0 = rs.solve(to_dev(b), default_opts(recycle=0, **kw))
    x1, st1 = rs.solve(to_dev(b), default_opts(recycle=4, **kw))
    x1 = to_host(x1).ravel()
    tau = 1e-8 * np.linalg.norm(b)
    true_r = np.linalg.norm(b.ravel() - emat @ x1)
    assert abs(true_r - st1["true_res"]) < 1e-3 * tau + 1e-13
    if strategy in ("grt", "thm2") and not kerker:
        assert true_r <= tau
    assert rel(x1, np.linalg.solve(emat, b.ravel())) < 1e-6
    print(f"N_ham without {st0['n_ham']}, with warm starts {st1['n_ham']} "
          f"({st1['warm_started']} warm band solves)")


@pytest.mark.parametrize("name,precision", [("tiny", 0), ("tiny_metal", 1), ("small_rect", 1)])
def test_repeated_dielectric_apply_starts_warm(name, precision):
    """The same E v applied twice with warm starts on: the second application's
    right-hand sides equal the stored ones, so every band starts from its stored
    solution and needs about one CG iteration; the result matches the first
    application and an application without warm starts to the CG tolerance."""
    from paper_2505_02319_amd import default_opts
    print(f"repeated apply: {name}", flush=True)
    rs, osys, ogs, perms = gpu_system(name)
    v = to_dev(random_field(osys.spec, 2))
    o = default_opts(strategy="fixed", precision=precision, recycle=2)
    e1, st1 = rs.apply_dielectric(v, 1e-11, o)
    e2, st2 = rs.apply_dielectric(v, 1e-11, o)
    e0, st0 = rs.apply_dielectric(v, 1e-11, default_opts(strategy="fixed", precision=precision))
    nslots = sum(rs.nocc_k())
    assert st1["warm_started"] == 0 and st2["warm_started"] == nslots
    assert st2["n_ham"] <= 3 * nslots < st1["n_ham"]
    assert rel(to_host(e2), to_host(e1)) < 1e-8
    assert rel(to_host(e2), to_host(e0)) < 1e-8


def test_recycled_solve_against_oracle_and_repeatable():
    """cfg1 (grt, 1e-10): the oracle's Alg. 1 and the library's solve with warm
    starts agree; two solves in a row give the same result (the stored pairs
    are reset at the start of each solve)."""
    from oracle.gmres import inexact_gmres
    from oracle.response import HxcKernel
    from paper_2505_02319_amd import default_opts
    import torch
    rs, osys, ogs, perms = gpu_system("cfg1")
    kern = HxcKernel(osys, ogs.rho, xc=1)
    b = random_field(osys.spec, 2)
    ref = inexact_gmres(osys, ogs, kern, b, 1e-10 * np.linalg.norm(b), strategy="grt")
    o = default_opts(strategy="grt", tol=1e-10, recycle=3)
    x1, st1 = rs.solve(to_dev(b), o)
    x2, st2 = rs.solve(to_dev(b), o)
    assert rel(to_host(x1), ref.x) < 1e-8
    assert torch.equal(x1, x2) and st1["n_ham"] == st2["n_ham"]


def test_recycle_option_is_validated():
    from paper_2505_02319_amd import IkrError, default_opts
    rs, osys, ogs, perms = gpu_system("tiny")
    with pytest.raises(IkrError):
        rs.solve(to_dev(random_field(osys.spec, 2)), default_opts(recycle=9))
