"""Every kernel path against the oracle.  Which path a launch takes depends on
its size: the gram runs on the matrix cores per tile of 16 bands up to 64
projection rows, on the matrix cores for all bands of a k-point at once
above (the k-wide gram, while a k-point's bands and rows fit it), else by
vector FMA; a CG iteration ends in one block while the batch has few
partials and in two launches above.  The large cells take the k-wide gram
and the two-launch end, so the same sum-over-states and dense-solve parity
tests run here with each path forced on the small cells, and on cells with
more than 64 projection rows where the size itself selects them ("wide": 33
occupied bands, 68 rows, 80 with the extra bands; "wider": 57 bands, 116
rows)."""
import numpy as np
import pytest

from gpu_common import gpu_system, rel, to_dev, to_host
from workloads import random_field

pytestmark = pytest.mark.gpu

FORCED = 3   # PATH_VECTOR_GRAM | PATH_SPLIT_END


@pytest.fixture
def paths():
    from paper_2505_02319_amd import kernel_paths, set_kernel_paths
    old = kernel_paths()

    def use(mask):
        set_kernel_paths(mask)
        assert kernel_paths() == mask
    yield use
    set_kernel_paths(old)


KWIDE = 4    # PATH_KWIDE


@pytest.mark.parametrize("name,mask", [("cfg1", FORCED), ("small_rect", FORCED),
                                       ("small_metal", FORCED), ("tiny_k", 1), ("tiny_k", 2),
                                       ("cfg1", KWIDE), ("small_rect", KWIDE),
                                       ("small_metal", KWIDE | 2), ("tiny_k", KWIDE),
                                       ("wide", 0), ("wide", 1), ("wide", 2), ("wide_k", 0),
                                       ("wider", 0), ("wider", 1)])
def test_chi0_sum_over_states_on_each_path(paths, name, mask):
    from oracle.response import SumOverStates
    print(f"chi0 paths: {name} mask {mask}", flush=True)
    paths(mask)
    rs, osys, ogs, perms = gpu_system(name)
    dv = random_field(osys.spec, 1)
    for precision_tol in (1e-12,):
        got, st = rs.apply_chi0(to_dev(dv), cg_tol=precision_tol)
        got = to_host(got)
        sos = SumOverStates(osys, ogs).apply(dv)
        assert rel(got, sos) < 1e-9, (name, mask, rel(got, sos))
        assert st["cg_unconverged"] == 0
        assert abs(got.sum()) < 1e-10 * np.abs(got).sum()


@pytest.fixture(scope="module")
def tiny_dense_paths():
    from oracle.response import HxcKernel, SumOverStates
    rs, osys, ogs, perms = gpu_system("tiny")
    kern = HxcKernel(osys, ogs.rho, xc=1)
    chi = SumOverStates(osys, ogs).dense_matrix()
    kmat = np.zeros((osys.ng, osys.ng))
    for j in range(osys.ng):
        e = np.zeros(osys.ng)
        e[j] = 1
        kmat[:, j] = kern.apply(e.reshape(osys.n)).ravel()
    return rs, osys, np.eye(osys.ng) - chi @ kmat


@pytest.mark.parametrize("strategy,precision,batching", [("grt", 0, 0), ("bal", 0, 0),
                                                         ("grt", 1, 0), ("thm2", 1, 1)])
def test_dense_solve_on_forced_paths(paths, tiny_dense_paths, strategy, precision, batching):
    from paper_2505_02319_amd import default_opts
    print(f"dense solve forced paths: {strategy} {precision} {batching}", flush=True)
    paths(FORCED)
    rs, osys, emat = tiny_dense_paths
    b = random_field(osys.spec, 2)
    x, st = rs.solve(to_dev(b), default_opts(strategy=strategy, tol=1e-8, precision=precision,
                                             batching=batching, want_true_residual=1))
    x = to_host(x).ravel()
    tau = 1e-8 * np.linalg.norm(b)
    true_r = np.linalg.norm(b.ravel() - emat @ x)
    assert true_r <= (tau if strategy != "bal" else 3 * tau)
    assert rel(x, np.linalg.solve(emat, b.ravel())) < 1e-7


@pytest.mark.parametrize("name,precision", [("wide", 0), ("wide", 1), ("wider", 1)])
def test_wide_solve_against_oracle_gmres(paths, name, precision):
    """More than 64 projection rows: the library's Alg. 1 (grt, tau = 1e-10
    ||b||) and the oracle's reach the same drho, by size-selected paths and
    with the two-launch end forced."""
    from oracle.gmres import inexact_gmres
    from oracle.response import HxcKernel
    from paper_2505_02319_amd import default_opts
    print(f"wide solve vs oracle: {name} precision {precision}", flush=True)
    rs, osys, ogs, perms = gpu_system(name)
    kern = HxcKernel(osys, ogs.rho, xc=osys.spec.xc)
    b = random_field(osys.spec, 2)
    tau = 1e-10 * np.linalg.norm(b)
    ref = inexact_gmres(osys, ogs, kern, b, tau, strategy="grt")
    for mask in (0, 2, 1):
        paths(mask)
        x, st = rs.solve(to_dev(b), default_opts(strategy="grt", tol=1e-10, precision=precision))
        assert rel(to_host(x), ref.x) < 1e-8, (mask, rel(to_host(x), ref.x))


@pytest.mark.parametrize("mask", [FORCED, KWIDE | 2])
def test_graph_replay_matches_launches_on_forced_paths(paths, mask):
    from paper_2505_02319_amd import default_opts
    paths(mask)
    rs, osys, ogs, perms = gpu_system("small_metal")
    b = to_dev(random_field(osys.spec, 2))
    kw = dict(strategy="grt", tol=1e-8, precision=1)
    x0, _ = rs.solve(b, default_opts(batching=0, **kw))
    x1, _ = rs.solve(b, default_opts(batching=1, **kw))
    x2, _ = rs.solve(b, default_opts(batching=1, **kw))
    assert rel(to_host(x1), to_host(x0)) < 1e-8
    import torch
    assert torch.equal(x1, x2)


def test_kernel_path_mask_is_checked():
    from paper_2505_02319_amd import IkrError, set_kernel_paths
    with pytest.raises(IkrError):
        set_kernel_paths(16)


@pytest.mark.parametrize("name", ["small_metal", "wide_k"])
def test_plain_fp64_reference_path(name):
    """batching = 2, the plain FP64 path (the k-points one after the other, a
    host read of the live count every CG iteration): the same drho as the
    batched solve and the oracle's Alg. 1 (insulator: grt at 1e-10 ||b||)."""
    from oracle.gmres import inexact_gmres
    from oracle.response import HxcKernel
    from paper_2505_02319_amd import default_opts
    print(f"plain fp64 path: {name}", flush=True)
    rs, osys, ogs, perms = gpu_system(name)
    b = random_field(osys.spec, 2)
    kw = dict(strategy="grt", tol=1e-10)
    xp, stp = rs.solve(to_dev(b), default_opts(batching=2, precision=1, **kw))
    xb, stb = rs.solve(to_dev(b), default_opts(batching=0, precision=0, **kw))
    assert stp["n_ham_fp32"] == 0
    assert rel(to_host(xp), to_host(xb)) < 1e-9
    kern = HxcKernel(osys, ogs.rho, xc=osys.spec.xc)
    ref = inexact_gmres(osys, ogs, kern, b, 1e-10 * np.linalg.norm(b), strategy="grt")
    assert rel(to_host(xp), ref.x) < 1e-8
