"""Launch shapes picked by measurement at the first CG run of a precision:
the gram's kernel and block count, the CG update's band group and the plane
kernel's block size.  Each candidate computes the same quantities, so every
one of them, pinned by hand, must give the oracle's chi0 (sum over states,
Sec. 2) and Alg. 1's solution; the measured picks must be among the
candidates and give the same solution as the size rules (PATH_FIXED)."""
import numpy as np
import pytest

from conftest import cached
from gpu_common import gpu_system, rel, to_dev, to_host
from workloads import random_field

pytestmark = pytest.mark.gpu

PATH_FIXED = 8


@pytest.fixture
def paths():
    from paper_2505_02319_amd import kernel_paths, set_kernel_paths
    old = kernel_paths()
    yield set_kernel_paths
    set_kernel_paths(old)


def _oracle_solution(name, osys, ogs, b):
    from oracle.gmres import inexact_gmres
    from oracle.response import HxcKernel

    def make():
        kern = HxcKernel(osys, ogs.rho, xc=osys.spec.xc)
        return inexact_gmres(osys, ogs, kern, b, 1e-10 * np.linalg.norm(b), strategy="grt").x
    return cached(("gmres_grt_1e-10_seed2", name), make)


def _valid(entry):
    assert entry["gram"] in ("size_rule", "per_tile_mfma", "kwide_mfma", "vector")
    assert entry["gram_scale"] in (0.5, 1.0, 2.0)
    assert entry["update_bands_per_block"] in (0, 4, 8, 16)
    assert entry["plane_threads"] in (0, 256, 512)
    assert entry["gram_us"] > 0


def test_tuning_measured_and_matches_size_rules(paths):
    """wide_k: 2 k-points x 33 bands = 3 tiles per k, so the first FP64 run
    measures both batch classes; mixed precision adds the FP32 ones.  The
    solution equals that of the size rules and of the oracle's Alg. 1."""
    from paper_2505_02319_amd import default_opts
    print("tuning: wide_k", flush=True)
    paths(0)
    rs, osys, ogs, perms = gpu_system("wide_k")
    assert rs.tuning() == {}
    b = random_field(osys.spec, 2)
    x64, _ = rs.solve(to_dev(b), default_opts(strategy="grt", tol=1e-10, precision=0))
    t = rs.tuning()
    assert ("fp64", "thick") in t and ("fp64", "thin") in t, t
    x32, st = rs.solve(to_dev(b), default_opts(strategy="grt", tol=1e-10, precision=1))
    t = rs.tuning()
    assert st["n_ham_fp32"] == 0 or ("fp32", "thin") in t, t
    for e in t.values():
        _valid(e)
    print(t, flush=True)
    paths(PATH_FIXED)
    rs2, _, _, _ = gpu_system("wide_k")
    xf, _ = rs2.solve(to_dev(b), default_opts(strategy="grt", tol=1e-10, precision=0))
    assert rs2.tuning() == {}
    ref = _oracle_solution("wide_k", osys, ogs, b)
    for x in (x64, x32, xf):
        assert rel(to_host(x), ref) < 1e-8
    assert rel(to_host(x64), to_host(xf)) < 1e-8


# every candidate value at least once, on cells where the size rules would
# take another: cfg1 (16 projection rows), wide (68 rows, 3 tiles on one
# k-point), tiny48 (48 x 48 planes)
PINS = [
    ("cfg1", dict(gram=1, gram_scale=0.5, update_bands_per_block=16)),
    ("cfg1", dict(gram=2, gram_scale=2.0, update_bands_per_block=4)),
    ("cfg1", dict(gram=3, gram_scale=2.0, update_bands_per_block=8)),
    ("wide", dict(gram=2, gram_scale=0.5, update_bands_per_block=16)),
    ("wide", dict(gram=3, gram_scale=0.5, update_bands_per_block=4)),
    ("tiny48", dict(gram=1, gram_scale=1.0, update_bands_per_block=8, plane_threads=256)),
    ("tiny48", dict(gram=2, gram_scale=2.0, update_bands_per_block=16, plane_threads=512)),
    ("wide", dict(gram=0, gram_scale=1.0, update_bands_per_block=0, plane_threads=0)),
]


@pytest.mark.parametrize("name,pin", PINS)
def test_pinned_shapes_against_oracle(paths, name, pin):
    """chi0 by the library's Sternheimer CG with the shapes pinned = the
    oracle's sum over states; a mixed-precision solve = the oracle's Alg. 1."""
    from oracle.response import SumOverStates
    from paper_2505_02319_amd import default_opts
    print(f"pinned shapes: {name} {pin}", flush=True)
    paths(0)
    rs, osys, ogs, perms = gpu_system(name)
    rs.pin_tuning(**pin)
    dv = random_field(osys.spec, 1)
    got, st = rs.apply_chi0(to_dev(dv), cg_tol=1e-12)
    sos = SumOverStates(osys, ogs).apply(dv)
    assert rel(to_host(got), sos) < 1e-9, rel(to_host(got), sos)
    assert st["cg_unconverged"] == 0
    b = random_field(osys.spec, 2)
    ref = _oracle_solution(name, osys, ogs, b)
    x, _ = rs.solve(to_dev(b), default_opts(strategy="grt", tol=1e-10, precision=1))
    assert rel(to_host(x), ref) < 1e-8
    # still pinned (a pinned entry is never measured over)
    t = rs.tuning()
    assert all(e["gram_us"] == 0 for e in t.values()) and len(t) == 4


def test_tuning_at_setup(paths):
    """ikr_tune_launches measures both precisions' classes before any solve
    and the first solve keeps them."""
    from paper_2505_02319_amd import default_opts
    paths(0)
    rs, osys, ogs, perms = gpu_system("wide_k")
    rs.tune_launches(precision=1, schur=1)
    t = rs.tuning()
    assert set(t) == {("fp64", "thick"), ("fp64", "thin"), ("fp32", "thick"), ("fp32", "thin")}
    for e in t.values():
        _valid(e)
    b = random_field(osys.spec, 2)
    x, _ = rs.solve(to_dev(b), default_opts(strategy="grt", tol=1e-10, precision=1))
    assert rs.tuning() == t
    assert rel(to_host(x), _oracle_solution("wide_k", osys, ogs, b)) < 1e-8


def test_tuning_input_is_checked():
    from paper_2505_02319_amd import IkrError
    rs, osys, ogs, perms = gpu_system("tiny")
    for bad in (dict(gram=4), dict(gram=-1), dict(gram=1, gram_scale=3.0),
                dict(gram=1, update_bands_per_block=5),
                dict(gram=1, plane_threads=128)):
        with pytest.raises(IkrError):
            rs.pin_tuning(**bad)
    rs.pin_tuning(gram=3)
    assert len(rs.tuning()) == 4
    rs.pin_tuning(None)
    assert rs.tuning() == {}
