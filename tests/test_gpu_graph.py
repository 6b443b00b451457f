"""The graph-replayed Sternheimer CG iteration (batching = 1) against the
plain launches and the dense operator.  Every replay is checked: solves run
several times in a row with eager work on the caller's stream in between."""
import numpy as np
import pytest

from gpu_common import gpu_system, rel, to_dev, to_host
from workloads import random_field

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,precision", [("tiny", 0), ("tiny", 1), ("tiny_k", 1),
                                            ("tiny_metal", 0), ("cfg1", 1)])
def test_graph_solve_matches_plain_launches(name, precision):
    from paper_2505_02319_amd import default_opts
    rs, osys, ogs, perms = gpu_system(name)
    b = to_dev(random_field(osys.spec, 2))
    bnorm = float(np.linalg.norm(to_host(b)))
    kw = dict(strategy="grt", tol=1e-9, precision=precision, want_true_residual=1)
    x0, st0 = rs.solve(b, default_opts(**kw))
    xs, sts = [], []
    for _ in range(3):
        x, st = rs.solve(b, default_opts(batching=1, **kw))
        xs.append(to_host(x))
        sts.append(st)
        rs.apply_kernel(b)            # eager work between the replays
    assert rel(xs[0], to_host(x0)) < 1e-8
    for x, st in zip(xs, sts):
        assert np.array_equal(x, xs[0])          # replays are bitwise reproducible
        assert st["n_ham"] == sts[0]["n_ham"]
        assert st["true_res"] <= 1e-9 * bnorm    # the grt guarantee
    assert abs(sts[0]["n_ham"] - st0["n_ham"]) <= 0.02 * st0["n_ham"]


def test_graph_dielectric_matches_dense():
    from oracle.response import HxcKernel, SumOverStates
    from paper_2505_02319_amd import default_opts
    rs, osys, ogs, perms = gpu_system("tiny_k")
    kern = HxcKernel(osys, ogs.rho, xc=1)
    chi = SumOverStates(osys, ogs).dense_matrix()
    v = random_field(osys.spec, 3)
    ref = v.ravel() - chi @ kern.apply(v).ravel()
    for _ in range(2):
        ev, _ = rs.apply_dielectric(to_dev(v), 1e-13, default_opts(strategy="fixed", batching=1))
        assert rel(to_host(ev), ref) < 1e-9


def test_graph_mode_with_profiling_falls_back_to_launches():
    from paper_2505_02319_amd import (default_opts, profile_enable, profile_query,
                                      profile_reset)
    rs, osys, ogs, perms = gpu_system("tiny")
    b = to_dev(random_field(osys.spec, 2))
    kw = dict(strategy="grt", tol=1e-9)
    x0, _ = rs.solve(b, default_opts(**kw))
    profile_reset()
    profile_enable(True)
    try:
        x1, _ = rs.solve(b, default_opts(batching=1, **kw))
        prof = profile_query()
    finally:
        profile_enable(False)
    assert prof["gram"][0] > 0
    assert np.array_equal(to_host(x1), to_host(x0))


def test_batching_option_is_validated():
    from paper_2505_02319_amd import IkrError, default_opts
    rs, osys, ogs, perms = gpu_system("tiny")
    b = to_dev(random_field(osys.spec, 2))
    with pytest.raises(IkrError):
        rs.solve(b, default_opts(batching=3))
