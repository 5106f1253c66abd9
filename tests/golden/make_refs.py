"""Writes the stored reference values of the benchmark workload using only the
FP64 oracle (never the GPU path).

    python tests/golden/make_refs.py

Workload c2 (Q=8 sensors, M=8 Rx, K=256 samples, 128x128 pixels, 60
point/extended targets, 15 dB), scene seed 100:
  c2_seed100.json        lambda_max, lambda (= 0.2 lambda_max), oracle run info
  c2_seed100_xref.npy    the optimum image x_ref (complex128, N): plain SADMM
                         iterated until the primal residual reaches the FP64
                         round-off floor (eps_rel = 1e-10 is below that floor,
                         so the run ends at max_iter)

Batched uneven frames c4 (M=8, K=128, per-frame Q and grid drawn by
scenegen.configs.c4_frames), batch seed 7, 16 frames:
  c4_batch_seed7.json    per-frame lambda_max and lambda (= 0.2 lambda_max)

    python tests/golden/make_refs.py c4

The full batched workload (256 frames, same seed, so its first 16 frames are
those above), lambda_max by the Woodbury / conjugate-gradient path:
  c4_batch256_seed7.json

    python tests/golden/make_refs.py c4 256

Workload c1 (Q=4, M=4, K=64, 32x32 pixels, 10 targets, 20 dB), scene seed 0:
  c1_seed0.json          lambda_max and lambda (= 0.2 lambda_max)

    python tests/golden/make_refs.py c1
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from scenegen import CONFIGS, config_scene, steering  # noqa: E402
from scenegen.configs import c4_frames, c4_scene  # noqa: E402


def main(seed: int = 100, max_iter: int = 300):
    cfg = CONFIGS["c2"]
    sc = config_scene("c2", seed)
    g = sc.geom
    A = [steering(g, q) for q in range(g.Q)]
    t0 = time.time()
    lmax = oracle.lambda_max(A, sc.y, cfg["mu"], cfg["gamma"])
    lam = cfg["lambda_frac"] * lmax
    p = oracle.Params(mu=cfg["mu"], beta=cfg["beta"], gamma=cfg["gamma"], lam=lam,
                      eps_abs=0.0, eps_rel=1e-10, max_iter=max_iter, stop=True)
    R = oracle.solve(A, sc.y, p)
    x_ref = R.z
    # iterations the oracle needs to bring NMSE vs x_ref to 1e-3 (plain and pruned)
    ks = {}
    for name, prune in (("plain", False), ("pruned", True)):
        q = oracle.Params(mu=cfg["mu"], beta=cfg["beta"], gamma=cfg["gamma"], lam=lam,
                          eps_abs=0.0, eps_rel=cfg["eps_rel"], max_iter=200, stop=True,
                          prune=prune, Kp=cfg["Kp"], eps_p=cfg["eps_p"])
        Rq = oracle.solve(A, sc.y, q, x_ref=x_ref)
        nm = Rq.history["nmse"]
        ks[name] = dict(iters_to_eps_rel=Rq.iters,
                        iters_to_nmse_1e3=next((i + 1 for i, v in enumerate(nm) if v <= 1e-3), None),
                        final_nmse=nm[-1],
                        final_max_active_frac=Rq.history["max_active_frac"][-1])
    info = dict(workload="c2", seed=seed, lambda_max=lmax, lambda_frac=cfg["lambda_frac"],
                lam=lam, mu=cfg["mu"], beta=cfg["beta"], gamma=cfg["gamma"],
                x_ref_iters=R.iters, x_ref_final_r=R.history["r"][-1],
                x_ref_final_eps_pri=R.history["eps_pri"][-1],
                x_ref_nnz=int(np.count_nonzero(np.abs(x_ref) > 0)),
                runs=ks, seconds=time.time() - t0)
    np.save(os.path.join(HERE, f"c2_seed{seed}_xref.npy"), x_ref)
    with open(os.path.join(HERE, f"c2_seed{seed}.json"), "w") as f:
        json.dump(info, f, indent=1)
    print(json.dumps(info, indent=1))


def main_c4(seed: int = 7, n_frames: int = 16, lambda_frac: float = 0.2):
    frames = c4_frames(n_frames, seed)
    for i, fr in enumerate(frames):
        sc = c4_scene(fr)
        A = [steering(sc.geom, q) for q in range(sc.geom.Q)]
        # the Woodbury / conjugate-gradient path (exact to its tolerance)
        fr["lambda_max"] = oracle.lambda_max(A, sc.y, 1.0, 1.0, dense_limit=0 if n_frames > 16 else 4096)
        fr["lam"] = lambda_frac * fr["lambda_max"]
        if n_frames > 16 and i % 16 == 0:
            print(f"frame {i}", flush=True)
    info = dict(workload="c4", seed=seed, n_frames=n_frames, lambda_frac=lambda_frac,
                mu=1.0, beta=1.0, gamma=1.0, frames=frames)
    name = f"c4_batch_seed{seed}.json" if n_frames == 16 else f"c4_batch{n_frames}_seed{seed}.json"
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(info, f, indent=1)
    print(json.dumps(info, indent=1))


def main_c1(seed: int = 0, lambda_frac: float = 0.2):
    cfg = CONFIGS["c1"]
    sc = config_scene("c1", seed)
    A = [steering(sc.geom, q) for q in range(sc.geom.Q)]
    lmax = oracle.lambda_max(A, sc.y, cfg["mu"], cfg["gamma"])
    info = dict(workload="c1", seed=seed, lambda_max=lmax, lambda_frac=lambda_frac,
                lam=lambda_frac * lmax, mu=cfg["mu"], beta=cfg["beta"], gamma=cfg["gamma"])
    with open(os.path.join(HERE, f"c1_seed{seed}.json"), "w") as f:
        json.dump(info, f, indent=1)
    print(json.dumps(info, indent=1))


if __name__ == "__main__":
    if sys.argv[1:2] == ["c1"]:
        main_c1()
    elif sys.argv[1:2] == ["c4"]:
        main_c4(n_frames=int(sys.argv[2]) if len(sys.argv) > 2 else 16)
    else:
        main()
