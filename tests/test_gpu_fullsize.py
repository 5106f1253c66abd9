"""Parity at the benchmark's shapes (KM = 2048 rows per sensor).

* c2 geometry with two of its sensors (N = 128^2: two 8192-column integer-Gram
  chunks, 528 Gram tiles, 16 outer Cholesky blocks): the factor against a CPU
  FP64 inverse of the stored complex64 values (1e-7, the integer-Gram bar),
  the 5-iteration image against the FP64 oracle (NMSE 1e-6, the FP32 bar;
  element-wise within 1e-3 of the image's peak).
* KM = 2048 on a 64^2 grid, FP64 storage, accelerated solve: selectors,
  compaction indices, prune events and iteration count equal the oracle's.
* c5 geometry (N = 512^2, matrix-free operator): the matched filter on a
  random 4096-pixel subset, and one full iteration whose selector keeps only
  that subset (generated forward, Woodbury and adjoint products at KM = 2048)
  against the oracle run on the subset's columns.
* the full c2 workload (8 sensors) run to eps_rel = 1e-4: FP32 accelerated
  solve, and FP16 / BF16 storage with the correction, against the stored FP64
  optimum x_ref (NMSE 1e-6).
"""

import json
import os

import numpy as np
import pytest

import oracle
from scenegen import config_scene, make_geometry, make_scene, steering

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def nmse(a, b):
    return float(np.linalg.norm(a - b) ** 2 / np.linalg.norm(b) ** 2)


def test_c2_geometry_two_sensors_factor_and_image(gpu_lib):
    g = make_geometry(Q=2, M=8, K=256, n_side=128)
    sc = make_scene(g, 11, 60, 15.0, extended=True)
    A = [np.asfortranarray(steering(g, q)) for q in range(g.Q)]
    lam = 0.2 * oracle.lambda_max(A, sc.y, 1.0, 1.0)
    hp = dict(mu=1.0, beta=1.0, gamma=1.0, lam=lam)
    print("c2 two sensors: building on the GPU", flush=True)
    s = gpu_lib.Solver(g.Q, g.K, g.M, g.N, storage="fp32", max_iter=5, stop=False, **hp)
    for q in range(g.Q):
        s.set_operator(q, A[q])
    s.solve(sc.y)
    z = s.image()
    W = s.factor(0)
    print("c2 two sensors: oracle", flush=True)
    ref = oracle.solve(A, sc.y, oracle.Params(max_iter=5, stop=False, **hp))
    assert np.abs(ref.z).max() > 0
    e = nmse(z, ref.z)
    emax = np.abs(z - ref.z).max() / np.abs(ref.z).max()
    print(f"c2 two sensors: NMSE {e:.3e}, max error / peak {emax:.3e}", flush=True)
    assert e <= 1e-6
    assert emax <= 1e-3
    # factor of sensor 0: (c/mu) I + A A^H of the complex64 values, inverted in FP64
    A32 = A[0].astype(np.complex64).astype(np.complex128)
    G = A32 @ A32.conj().T
    G[np.diag_indices_from(G)] += (hp["beta"] + hp["gamma"]) / hp["mu"]
    Wc = np.linalg.inv(G)
    KM = g.K * g.M
    ferr = np.linalg.norm(W[:KM, :KM] - Wc) / np.linalg.norm(Wc)
    print(f"c2 two sensors: factor error {ferr:.3e}", flush=True)
    assert ferr <= 1e-7


def test_km2048_fp64_pruned_masks_bit_exact(gpu_lib):
    g = make_geometry(Q=4, M=8, K=256, n_side=64)
    sc = make_scene(g, 12, 40, 15.0, extended=True)
    A = [np.asfortranarray(steering(g, q)) for q in range(g.Q)]
    lam = 0.2 * oracle.lambda_max(A, sc.y, 1.0, 1.0, dense_limit=0)
    kw = dict(mu=1.0, beta=1.0, gamma=1.0, lam=lam, max_iter=300, eps_abs=0.0, eps_rel=1e-4,
              prune=True, Kp=5, eps_p=1e-5)
    s = gpu_lib.Solver(g.Q, g.K, g.M, g.N, storage="fp64", **kw)
    for q in range(g.Q):
        s.set_operator(q, A[q])
    info = s.solve(sc.y)
    ref = oracle.solve(A, sc.y, oracle.Params(**kw))
    print(f"KM 2048 pruned: iters {info['iters']} / {ref.iters}, events {info['prune_events']} / "
          f"{ref.prune_events}, max active {info['max_active_frac']:.4f}", flush=True)
    assert ref.prune_events > 0
    assert info["iters"] == ref.iters and info["prune_events"] == ref.prune_events
    for q in range(g.Q):
        assert np.array_equal(s.active_mask(q).astype(bool), ref.active[q])
        assert np.array_equal(s.active_indices(q), np.flatnonzero(ref.active[q]))
    assert np.linalg.norm(s.image() - ref.z) / np.linalg.norm(ref.z) < 1e-8


def test_c5_geometry_subset_matched_filter_and_iteration(gpu_lib):
    g = make_geometry(Q=8, M=8, K=256, n_side=512)
    sc = make_scene(g, 13, 600, 15.0, extended=True)
    rng = np.random.default_rng(5)
    cols = np.sort(rng.choice(g.N, 4096, replace=False))
    A = [np.asfortranarray(steering(g, q, cols)) for q in range(g.Q)]
    s = gpu_lib.Solver(g.Q, g.K, g.M, g.N, storage="mf", max_iter=1, stop=False, lam=0.0)
    for q in range(g.Q):
        s.set_operator_geometry(q, g.tx[q], g.rx[q], g.pix, g.f0, g.bw)
    mf = s.matched_filter(sc.y)[:, cols]
    mref = oracle.matched_filter(A, sc.y)
    merr = np.abs(mf - mref).max() / mref.max()
    print(f"c5 subset: matched filter error / peak {merr:.3e}", flush=True)
    assert merr <= 1e-6
    s.close()
    lam = 0.2 * oracle.lambda_max(A, sc.y, 1.0, 1.0, dense_limit=0)
    hp = dict(mu=1.0, beta=1.0, gamma=1.0, lam=lam)
    s = gpu_lib.Solver(g.Q, g.K, g.M, g.N, storage="mf", max_iter=1, stop=False, **hp)
    mask = np.zeros(g.N, np.uint8)
    mask[cols] = 1
    for q in range(g.Q):
        s.set_operator_geometry(q, g.tx[q], g.rx[q], g.pix, g.f0, g.bw)
        s.set_active_mask(q, mask)
    s.solve(sc.y)
    ref = oracle.solve(A, sc.y, oracle.Params(max_iter=1, stop=False, **hp))
    z = s.image()
    assert not z[mask == 0].any()
    for q in (0, 5):
        xq = s.sensor_image(q)[cols]
        e = nmse(xq, ref.X[q])
        print(f"c5 subset: sensor {q} x NMSE {e:.3e}", flush=True)
        assert e <= 1e-6
    if np.abs(ref.z).max() > 0:
        assert nmse(z[cols], ref.z) <= 1e-6


def _c2_workload():
    info = json.load(open(os.path.join(GOLD, "c2_seed100.json")))
    x_ref = np.load(os.path.join(GOLD, "c2_seed100_xref.npy"))
    sc = config_scene("c2", info["seed"])
    hp = dict(mu=info["mu"], beta=info["beta"], gamma=info["gamma"], lam=info["lam"])
    return sc, sc.geom, hp, x_ref


@pytest.mark.parametrize("storage,refine", [("fp32", 0), ("fp16", 10), ("bf16", 10)])
def test_c2_workload_to_tolerance_against_optimum(gpu_lib, storage, refine):
    sc, g, hp, x_ref = _c2_workload()
    s = gpu_lib.Solver(g.Q, g.K, g.M, g.N, storage=storage, prune=True, kkt=True, max_iter=400,
                       eps_abs=0.0, eps_rel=1e-4, Kp=5, eps_p=1e-5, refine_every=refine, **hp)
    for q in range(g.Q):
        s.set_operator_geometry(q, g.tx[q], g.rx[q], g.pix, g.f0, g.bw)
    info = s.solve(sc.y)
    z = s.image()
    e = nmse(z, x_ref)
    emax = np.abs(z - x_ref).max() / np.abs(x_ref).max()
    dx = s.history("retake_change")
    print(f"c2 {storage}: iters {info['iters']} status {info['status']} events {info['prune_events']} "
          f"direct sensors {info['direct_sensors']} NMSE {e:.3e} max err / peak {emax:.3e} "
          f"retakes {[(int(k) + 1, float(dx[k])) for k in np.flatnonzero(dx)[:6]]}", flush=True)
    assert info["status"] == 0
    assert e <= 1e-6
    assert emax <= 2e-3
