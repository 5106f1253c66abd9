"""Batched solves (sadmm_solve_batch): several independent scenes with
different sensor counts, pixel counts, parameters and selectors iterated by
one launch per kernel.  Each scene must give exactly the result of solving it
alone (same arithmetic per scene), and match the oracle."""

import numpy as np
import pytest

import oracle
from scenegen import make_geometry, make_scene, steering

pytestmark = pytest.mark.gpu


def scene(Q, M, K, n_side, seed, n_targets):
    g = make_geometry(Q, M, K, n_side)
    sc = make_scene(g, seed, n_targets, 20.0)
    A = [steering(g, q) for q in range(Q)]
    lam = 0.2 * oracle.lambda_max(A, sc.y, 1.0, 1.0)
    return g, sc, A, lam


def solver(lib, g, A, lam, storage, **kw):
    s = lib.Solver(g.Q, g.K, g.M, g.N, storage=storage, lam=lam, **kw)
    for q in range(g.Q):
        s.set_operator(q, A[q])
    return s


SCENES = [dict(Q=4, M=4, K=64, n_side=32, seed=1, n_targets=10, prune=True, max_iter=60),
          dict(Q=3, M=4, K=32, n_side=20, seed=2, n_targets=5, prune=False, max_iter=40),
          dict(Q=6, M=2, K=64, n_side=24, seed=3, n_targets=6, prune=True, max_iter=50)]


@pytest.mark.parametrize("storage", ["fp64", "fp32"])
def test_batch_equals_individual_solves(gpu_lib, storage):
    probs = [scene(c["Q"], c["M"], c["K"], c["n_side"], c["seed"], c["n_targets"]) for c in SCENES]
    single = []
    for (g, sc, A, lam), c in zip(probs, SCENES):
        s = solver(gpu_lib, g, A, lam, storage, prune=c["prune"], max_iter=c["max_iter"],
                   stop=False, eps_rel=1e-4)
        s.solve(sc.y)
        single.append((s.image(), [s.active_mask(q) for q in range(g.Q)]))
    batch = [solver(gpu_lib, g, A, lam, storage, prune=c["prune"], max_iter=c["max_iter"],
                    stop=False, eps_rel=1e-4) for (g, sc, A, lam), c in zip(probs, SCENES)]
    infos = gpu_lib.solve_batch(batch, [sc.y for (g, sc, A, lam) in probs])
    for i, (s, (z1, m1)) in enumerate(zip(batch, single)):
        assert infos[i]["iters"] == SCENES[i]["max_iter"]
        assert np.array_equal(s.image(), z1), i
        for q in range(len(m1)):
            assert np.array_equal(s.active_mask(q), m1[q])


def test_batch_matches_oracle_with_early_stops(gpu_lib):
    """Scenes stop at different iterations (own tolerances); FP64 results match
    the oracle's per scene."""
    probs = [scene(c["Q"], c["M"], c["K"], c["n_side"], c["seed"], c["n_targets"]) for c in SCENES]
    tols = [1e-4, 1e-6, 1e-5]
    batch = []
    for (g, sc, A, lam), c, t in zip(probs, SCENES, tols):
        batch.append(solver(gpu_lib, g, A, lam, "fp64", prune=c["prune"], max_iter=500,
                            eps_rel=t))
    infos = gpu_lib.solve_batch(batch, [sc.y for (g, sc, A, lam) in probs])
    for (g, sc, A, lam), c, t, s, info in zip(probs, SCENES, tols, batch, infos):
        ref = oracle.solve(A, sc.y, oracle.Params(lam=lam, max_iter=500, eps_rel=t,
                                                  prune=c["prune"]))
        assert info["status"] == 0 and info["iters"] == ref.iters
        assert np.linalg.norm(s.image() - ref.z) <= 1e-8 * np.linalg.norm(ref.z)


def test_repeated_batch_solves_are_identical(gpu_lib):
    """The same batch solved twice on the same handles, and then each scene
    alone again: every iteration's end-of-iteration work (residuals, stop
    test, prune flag) runs in the last work-group of its kernel, picked by a
    completion count that each iteration leaves at zero; a count left over
    from a solve would shift the next solve's residuals or prune decisions."""
    probs = [scene(c["Q"], c["M"], c["K"], c["n_side"], c["seed"], c["n_targets"]) for c in SCENES]
    batch = [solver(gpu_lib, g, A, lam, "fp32", prune=c["prune"], max_iter=c["max_iter"],
                    stop=True, eps_rel=1e-4) for (g, sc, A, lam), c in zip(probs, SCENES)]
    ys = [sc.y for (g, sc, A, lam) in probs]
    first = gpu_lib.solve_batch(batch, ys)
    z1 = [s.image() for s in batch]
    second = gpu_lib.solve_batch(batch, ys)
    for i, s in enumerate(batch):
        assert second[i]["iters"] == first[i]["iters"], i
        assert second[i]["prune_events"] == first[i]["prune_events"], i
        assert np.array_equal(s.image(), z1[i]), i
    for i, s in enumerate(batch):
        info = s.solve(ys[i])
        assert info["iters"] == first[i]["iters"], i
        assert np.array_equal(s.image(), z1[i]), i
