"""The magnitude variant (Sec. II: x_q real, the image a non-negative
magnitude) through the C ABI against the oracle: the operator and
measurements stacked into their real form on the device (sadmm_stack_real),
the projected z-update (params.nonneg).  FP64 storage: images within 1e-8
(relative), selectors of the accelerated solve exact; FP32: NMSE 1e-6."""

import numpy as np
import pytest

import oracle
from scenegen import make_geometry, make_scene, steering

pytestmark = pytest.mark.gpu


def problem(seed=1, beta=1.0, gamma=1.0):
    g = make_geometry(Q=4, M=4, K=64, n_side=32)
    sc = make_scene(g, seed, 10, 20.0)
    A = [steering(g, q) for q in range(g.Q)]
    As, ys = oracle.stack_real(A, sc.y)
    lam = 0.2 * oracle.lambda_max(As, ys, 1.0, gamma)
    return g, A, sc.y, As, ys, dict(mu=1.0, beta=beta, gamma=gamma, lam=lam)


def gpu_real(lib, g, A, y, hp, storage, **kw):
    import torch
    s = lib.Solver(g.Q, 2 * g.K, g.M, g.N, storage=storage, **hp, **kw)
    for q in range(g.Q):
        At = torch.from_numpy(np.ascontiguousarray(A[q].T)).cuda()      # (N, KM): column-major A
        s.set_operator(q, lib.stack_real(At))
    yr = lib.stack_real(torch.from_numpy(np.ascontiguousarray(y)).cuda())
    info = s.solve(yr)
    return s, info


def test_stack_real_matches_oracle(gpu_lib):
    import torch
    g, A, y, As, ys, hp = problem()
    got = gpu_lib.stack_real(torch.from_numpy(np.ascontiguousarray(A[1].T)).cuda()).cpu().numpy()
    assert np.array_equal(got.T, As[1])
    gy = gpu_lib.stack_real(torch.from_numpy(np.ascontiguousarray(y).astype(np.complex64)).cuda())
    assert np.array_equal(gy.cpu().numpy(), ys.astype(np.complex64).astype(np.complex128))


@pytest.mark.parametrize("nonneg", [True, False])
def test_real_variant_fp64_fixed_iterations(gpu_lib, nonneg):
    g, A, y, As, ys, hp = problem()
    kw = dict(max_iter=80, stop=False, nonneg=nonneg)
    s, info = gpu_real(gpu_lib, g, A, y, hp, "fp64", **kw)
    ref = oracle.solve(As, ys, oracle.Params(**hp, **kw))
    z = s.image()
    assert np.abs(ref.z).max() > 0
    assert np.linalg.norm(z - ref.z) / np.linalg.norm(ref.z) < 1e-8
    assert not z.imag.any()
    if nonneg:
        assert (z.real >= 0).all()
    else:
        assert (ref.z.real < 0).any()           # without the projection the image goes negative
    for q in range(g.Q):
        xq = s.sensor_image(q)
        assert np.abs(xq.imag).max() <= 1e-12 * np.abs(xq).max()


def test_nonneg_pruned_fp64_selectors_exact(gpu_lib):
    """beta = 3 > gamma = 1: the primal residual meets its tolerance well before
    the dual one, so the SSC gate opens (4 elimination events)."""
    g, A, y, As, ys, hp = problem(seed=2, beta=3.0)
    kw = dict(max_iter=400, eps_abs=0.0, eps_rel=1e-4, prune=True, Kp=5, eps_p=1e-5, nonneg=True)
    s, info = gpu_real(gpu_lib, g, A, y, hp, "fp64", **kw)
    ref = oracle.solve(As, ys, oracle.Params(**hp, **kw))
    print("nonneg pruned:", info["iters"], ref.iters, info["prune_events"], ref.prune_events, flush=True)
    assert ref.prune_events > 0
    assert info["iters"] == ref.iters and info["prune_events"] == ref.prune_events
    for q in range(g.Q):
        assert np.array_equal(s.active_mask(q).astype(bool), ref.active[q])
    assert np.linalg.norm(s.image() - ref.z) / np.linalg.norm(ref.z) < 1e-8


def test_nonneg_pruned_fp32_image(gpu_lib):
    g, A, y, As, ys, hp = problem(seed=1, beta=3.0)
    kw = dict(max_iter=400, eps_abs=0.0, eps_rel=1e-5, prune=True, kkt=True, Kp=5, eps_p=1e-5, nonneg=True)
    s, info = gpu_real(gpu_lib, g, A, y, hp, "fp32", **kw)
    ref = oracle.solve(As, ys, oracle.Params(**hp, **{**kw, "eps_rel": 1e-10, "prune": False,
                                                      "kkt": False, "max_iter": 5000}))
    z = s.image()
    e = np.linalg.norm(z - ref.z) ** 2 / np.linalg.norm(ref.z) ** 2
    print("nonneg fp32 pruned:", info["iters"], info["status"], info["prune_events"], e, flush=True)
    assert info["status"] == 0 and info["prune_events"] > 0
    assert e <= 1e-6
    assert (z.real >= 0).all() and not z.imag.any()
