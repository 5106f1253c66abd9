"""Forward-product tile autotuner (sadmm_autotune): it picks one of the
supported widths, leaves the solve's result unchanged up to summation order,
and hands its choice to later handles of the same storage, rows and
pixel-count bucket.  The shapes here (K M = 180 and 132 rows) are used by no other
test, so the widths recorded for them change no other test's handles."""

import numpy as np
import pytest

import oracle
from scenegen import make_geometry, make_scene, steering

pytestmark = pytest.mark.gpu

WIDTHS = (64, 128, 256, 512, 1024)


def problem(Q, M, K, n_side, seed):
    g = make_geometry(Q, M, K, n_side)
    sc = make_scene(g, seed, 8, 20.0)
    A = [steering(g, q) for q in range(Q)]
    lam = 0.2 * oracle.lambda_max(A, sc.y, 1.0, 1.0)
    return g, sc, A, lam


def solver(lib, g, A, lam, storage, **kw):
    s = lib.Solver(g.Q, g.K, g.M, g.N, storage=storage, lam=lam, **kw)
    for q in range(g.Q):
        s.set_operator(q, A[q])
    return s


@pytest.mark.parametrize("storage,rtol", [("fp32", 1e-4), ("bf16", 1e-3)])
def test_tuned_width_keeps_result_and_is_shared(gpu_lib, storage, rtol):
    g, sc, A, lam = problem(4, 3, 60, 70, 11)          # N = 4900: every width fits
    s = solver(gpu_lib, g, A, lam, storage, max_iter=40, stop=False)
    w0 = s.autotune(sc.y, 0)
    assert w0 in WIDTHS
    s.solve(sc.y)
    z0 = s.image()
    w = s.autotune(sc.y, 6)
    print(f"{storage}: default width {w0}, tuned {w}", flush=True)
    assert w in WIDTHS and s.autotune(sc.y, 0) == w
    info = s.solve(sc.y)
    assert info["iters"] == 40                          # parameters restored
    z1 = s.image()
    assert np.linalg.norm(z1 - z0) <= rtol * np.linalg.norm(z0)
    # a later handle with the same key starts from the tuned width
    s2 = solver(gpu_lib, g, A, lam, storage, max_iter=40, stop=False)
    assert s2.autotune(sc.y, 0) == w
    s2.solve(sc.y)
    assert np.array_equal(s2.image(), z1)


def test_tuned_fp64_matches_oracle(gpu_lib):
    """After tuning, the FP64 solve still meets the oracle at 1e-8."""
    g, sc, A, lam = problem(3, 3, 44, 40, 12)
    s = solver(gpu_lib, g, A, lam, "fp64", max_iter=300, eps_rel=1e-5, prune=True)
    assert s.autotune(sc.y, 4) in WIDTHS
    info = s.solve(sc.y)
    ref = oracle.solve(A, sc.y, oracle.Params(lam=lam, max_iter=300, eps_rel=1e-5, prune=True))
    assert info["iters"] == ref.iters
    assert np.linalg.norm(s.image() - ref.z) <= 1e-8 * np.linalg.norm(ref.z)


def test_small_image_takes_narrow_widths_and_bad_counts_fail(gpu_lib):
    g, sc, A, lam = problem(2, 2, 16, 12, 13)           # N = 144: widths 64 and 128
    s = solver(gpu_lib, g, A, lam, "fp32", max_iter=10)
    assert s.autotune(sc.y, 3) in (64, 128)
    with pytest.raises(gpu_lib.SadmmError):
        s.autotune(sc.y, 1)
