"""Scenes that share one operator (sadmm_create_shared): their forward and
adjoint products run as multi-right-hand-side products on the FP32 matrix
instructions in sadmm_solve_batch.

Shapes: 17 scenes (a ragged second block of 16 right-hand sides), N = 900
pixels (not a multiple of the 64-pixel tile or the 1024-pixel chunk),
KM = 256.

Tolerances.  Against independent single-scene FP32 solves of the same
scenes (own operator copies, single-right-hand-side kernels) over a fixed 60
iterations: the two paths add the same FP32 products in different orders
(MFMA 4-wide k-steps and 1024-pixel chunks vs 256-pixel chunks and wave
reductions), about 1e-7 relative per product; the iteration is a contraction,
so the images stay within 1e-5 (relative L2).  Against the FP64 oracle run
to its own stop: the FP32 bar, image NMSE <= 1e-6.
"""

import numpy as np
import pytest

import oracle
from scenegen import make_geometry, make_scene, steering

pytestmark = pytest.mark.gpu

Q, M, K, SIDE, S = 4, 4, 64, 30, 17


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def nmse(a, b):
    return float(np.linalg.norm(a - b) ** 2 / max(np.linalg.norm(b) ** 2, 1e-300))


@pytest.fixture(scope="module")
def frames():
    g = make_geometry(Q, M, K, SIDE)
    A = [steering(g, q) for q in range(Q)]
    scenes = [make_scene(g, 40 + i, 6 + i % 5, 15.0 + i % 7) for i in range(S)]
    # one lambda for all frames (lambda is per handle; a common value keeps the
    # comparison simple): 0.2 lambda_max of the first frame
    lam = 0.2 * oracle.lambda_max(A, scenes[0].y, 1.0, 1.0)
    return g, A, scenes, lam


def shared_handles(lib, g, A, lam, **kw):
    src = lib.Solver(g.Q, g.K, g.M, g.N, storage="fp32", lam=lam, **kw)
    for q in range(g.Q):
        src.set_operator(q, A[q])
    hs = [src] + [lib.Solver(g.Q, g.K, g.M, g.N, storage="fp32", lam=lam, share=src, **kw)
                  for _ in range(S - 1)]
    return hs


def test_shared_batch_equals_single_scene_solves(gpu_lib, frames):
    g, A, scenes, lam = frames
    kw = dict(max_iter=60, stop=False)
    single = []
    for sc in scenes:
        s = gpu_lib.Solver(g.Q, g.K, g.M, g.N, storage="fp32", lam=lam, **kw)
        for q in range(g.Q):
            s.set_operator(q, A[q])
        s.solve(sc.y)
        single.append(s.image())
        s.close()
    hs = shared_handles(gpu_lib, g, A, lam, **kw)
    infos = gpu_lib.solve_batch(hs, [sc.y for sc in scenes])
    for i, (h, z1) in enumerate(zip(hs, single)):
        assert infos[i]["iters"] == 60
        err = rel(h.image(), z1)
        assert err <= 1e-5, (i, err)


def test_shared_batch_matches_oracle(gpu_lib, frames):
    g, A, scenes, lam = frames
    hs = shared_handles(gpu_lib, g, A, lam, max_iter=400, eps_rel=1e-4)
    infos = gpu_lib.solve_batch(hs, [sc.y for sc in scenes])
    iters = set()
    for i, (h, sc, info) in enumerate(zip(hs, scenes, infos)):
        ref = oracle.solve(A, sc.y, oracle.Params(lam=lam, max_iter=400, eps_rel=1e-4))
        assert info["status"] == 0
        iters.add(info["iters"])
        assert nmse(h.image(), ref.z) <= 1e-6, (i, nmse(h.image(), ref.z))
    assert len(iters) > 1   # scenes stopped at different iterations


def test_shared_batch_ragged_rows(gpu_lib):
    """KM = 96 (the last 64-row block of the products half empty), 5 scenes."""
    g = make_geometry(3, 2, 48, 20)
    A = [steering(g, q) for q in range(g.Q)]
    scenes = [make_scene(g, 70 + i, 5, 18.0) for i in range(5)]
    lam = 0.2 * oracle.lambda_max(A, scenes[0].y, 1.0, 1.0)
    src = gpu_lib.Solver(g.Q, g.K, g.M, g.N, storage="fp32", lam=lam, max_iter=300, eps_rel=1e-4)
    for q in range(g.Q):
        src.set_operator(q, A[q])
    hs = [src] + [gpu_lib.Solver(g.Q, g.K, g.M, g.N, storage="fp32", lam=lam, max_iter=300,
                                 eps_rel=1e-4, share=src) for _ in range(4)]
    gpu_lib.solve_batch(hs, [sc.y for sc in scenes])
    for h, sc in zip(hs, scenes):
        ref = oracle.solve(A, sc.y, oracle.Params(lam=lam, max_iter=300, eps_rel=1e-4))
        assert nmse(h.image(), ref.z) <= 1e-6


def test_create_shared_rejects_pruning_and_borrowed_setters(gpu_lib, frames):
    g, A, scenes, lam = frames
    src = gpu_lib.Solver(g.Q, g.K, g.M, g.N, storage="fp32", lam=lam)
    for q in range(g.Q):
        src.set_operator(q, A[q])
    with pytest.raises(gpu_lib.SadmmError):
        gpu_lib.Solver(g.Q, g.K, g.M, g.N, storage="fp32", lam=lam, prune=True, share=src)
    with pytest.raises(gpu_lib.SadmmError):
        gpu_lib.Solver(g.Q, g.K, g.M, g.N, storage="fp32", lam=lam, beta=2.0, share=src)
    h = gpu_lib.Solver(g.Q, g.K, g.M, g.N, storage="fp32", lam=lam, share=src)
    with pytest.raises(gpu_lib.SadmmError):
        h.set_operator(0, A[0])
    with pytest.raises(gpu_lib.SadmmError):
        h.set_active_mask(0, np.ones(g.N, np.uint8))
    with pytest.raises(gpu_lib.SadmmError):
        src.set_active_mask(0, np.ones(g.N, np.uint8))
    # a borrower alone builds its source's factor on demand
    info = h.solve(scenes[1].y)
    ref = oracle.solve(A, scenes[1].y, oracle.Params(lam=lam, max_iter=200, eps_rel=1e-4))
    assert info["iters"] > 0 and nmse(h.image(), ref.z) <= 1e-6
    h.close()
