"""Matrix-free operator (entries regenerated from per-pixel phase records in
every product) vs the FP64 oracle and vs stored operators.  Arithmetic is
FP32 with FP64 phase fractions, so the bar is the FP32 one: NMSE <= 1e-6
against the FP64 optimum."""

import numpy as np
import pytest

import oracle
from scenegen import make_geometry, make_scene, steering

pytestmark = pytest.mark.gpu


def nmse(a, b):
    return float(np.linalg.norm(a - b) ** 2 / np.linalg.norm(b) ** 2)


def setup(Q=4, M=4, K=64, n_side=32, seed=1, n_targets=10):
    g = make_geometry(Q, M, K, n_side)
    sc = make_scene(g, seed, n_targets, 20.0)
    A = [steering(g, q) for q in range(Q)]
    lam = 0.2 * oracle.lambda_max(A, sc.y, 1.0, 1.0)
    return g, sc, A, lam


def mf_solver(lib, g, lam, **kw):
    s = lib.Solver(g.Q, g.K, g.M, g.N, storage="mf", lam=lam, **kw)
    for q in range(g.Q):
        s.set_operator_geometry(q, g.tx[q], g.rx[q], g.pix, g.f0, g.bw)
    return s


def test_matrix_free_plain_matches_oracle(gpu_lib):
    g, sc, A, lam = setup()
    opt = oracle.solve(A, sc.y, oracle.Params(lam=lam, max_iter=3000, eps_rel=1e-10))
    s = mf_solver(gpu_lib, g, lam, max_iter=100, stop=False)
    s.solve(sc.y)
    assert nmse(s.image(), opt.z) <= 1e-6


def test_matrix_free_factor_matches_dense(gpu_lib):
    """The factor built from regenerated columns equals the one built from the
    stored FP64 operator to FP32 entry accuracy."""
    g, sc, A, lam = setup(Q=2, M=4, K=32, n_side=16, n_targets=4)
    s = mf_solver(gpu_lib, g, lam, max_iter=1, stop=False)
    s.solve(sc.y)
    d = gpu_lib.Solver(g.Q, g.K, g.M, g.N, storage="fp64", lam=lam, max_iter=1, stop=False)
    for q in range(g.Q):
        d.set_operator(q, A[q])
    d.solve(sc.y)
    for q in range(g.Q):
        W1, W2 = s.factor(q), d.factor(q)
        assert np.linalg.norm(W1 - W2) <= 1e-4 * np.linalg.norm(W2)


def test_matrix_free_pruned_with_kkt(gpu_lib):
    """Accelerated solve (SSC elimination, compaction of the phase records,
    low-rank factor updates, optimality re-check) on the matrix-free operator."""
    g, sc, A, lam = setup(seed=3)
    kw = dict(max_iter=60, stop=False, eps_rel=1e-4, prune=True, Kp=5, eps_p=1e-5)
    ref = oracle.solve(A, sc.y, oracle.Params(lam=lam, **kw))
    s = mf_solver(gpu_lib, g, lam, **kw)
    info = s.solve(sc.y)
    assert ref.prune_events > 0 and info["prune_events"] > 0
    assert nmse(s.image(), ref.z) <= 1e-6


def test_matrix_free_matched_filter(gpu_lib):
    g, sc, A, lam = setup(Q=3, M=4, K=32, n_side=16, n_targets=4)
    s = mf_solver(gpu_lib, g, lam)
    mf = s.matched_filter(sc.y)
    ref = oracle.matched_filter(A, sc.y)
    assert np.abs(mf - ref).max() <= 1e-5 * np.abs(ref).max()
