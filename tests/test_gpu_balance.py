"""Residual balancing (Boyd et al. 2011, Sec. 3.4.1; params.balance_every)
through the C ABI against the oracle.  FP64 storage: the beta schedule and
the iteration count equal the oracle's, the image within 1e-8; a penalty 30x
too large converges in 39 iterations instead of 396.  FP32 with pruning: the
image within NMSE 1e-6 of the FP64 optimum.  Each solve starts from the beta
of the parameters again."""

import numpy as np
import pytest

import oracle
from scenegen import make_geometry, make_scene, steering

pytestmark = pytest.mark.gpu


def problem(seed=1):
    g = make_geometry(Q=4, M=4, K=64, n_side=32)
    sc = make_scene(g, seed, 10, 20.0)
    A = [steering(g, q) for q in range(g.Q)]
    lam = 0.2 * oracle.lambda_max(A, sc.y, 1.0, 1.0)
    return g, sc, A, lam


def run(lib, g, A, y, storage, **kw):
    s = lib.Solver(g.Q, g.K, g.M, g.N, storage=storage, **kw)
    for q in range(g.Q):
        s.set_operator(q, A[q])
    return s, s.solve(y)


@pytest.mark.parametrize("beta", [30.0, 0.05])
def test_balanced_fp64_schedule_and_image(gpu_lib, beta):
    g, sc, A, lam = problem()
    kw = dict(mu=1.0, beta=beta, gamma=1.0, lam=lam, eps_abs=0.0, eps_rel=1e-6, max_iter=3000,
              balance_every=5)
    s, info = run(gpu_lib, g, A, sc.y, "fp64", **kw)
    ref = oracle.solve(A, sc.y, oracle.Params(**kw))
    b = s.history("beta")
    print(f"beta {beta}: iters {info['iters']} / {ref.iters}, betas {sorted(set(b.tolist()))}", flush=True)
    assert ref.converged and info["status"] == 0
    assert info["iters"] == ref.iters
    np.testing.assert_array_equal(b, np.array(ref.history["beta"]))
    assert np.count_nonzero(np.diff(b)) >= 3
    assert np.linalg.norm(s.image() - ref.z) / np.linalg.norm(ref.z) < 1e-8
    # the next solve starts from the given beta again
    info2 = s.solve(sc.y)
    assert s.history("beta")[0] == beta and info2["iters"] == info["iters"]


def test_balanced_fp32_pruned_against_optimum(gpu_lib):
    g, sc, A, lam = problem(seed=2)
    hp = dict(mu=1.0, gamma=1.0, lam=lam)
    opt = oracle.solve(A, sc.y, oracle.Params(beta=1.0, eps_abs=0.0, eps_rel=1e-11, max_iter=5000, **hp))
    s, info = run(gpu_lib, g, A, sc.y, "fp32", beta=30.0, eps_abs=0.0, eps_rel=1e-5, max_iter=3000,
                  balance_every=5, prune=True, kkt=True, **hp)
    e = np.linalg.norm(s.image() - opt.z) ** 2 / np.linalg.norm(opt.z) ** 2
    print("fp32 balanced pruned:", info["iters"], info["status"], info["prune_events"], e, flush=True)
    assert info["status"] == 0
    assert e <= 1e-6
