"""Named synthetic workloads (geometry + scene recipe + solver hyperparameters).

The paper's own scene (Sec. IV) is not published; these seeded workloads stand
in for it.  Hyperparameters: mu, beta, gamma are the data weight, the
augmented-Lagrangian penalty and the per-sensor ridge; the l1 weight is
`lambda_frac` times the problem's lambda_max (the smallest l1 weight whose
optimum image is identically zero), or the absolute `lambda_abs` where given.

* c1     -- Q=4 sensors, M=4 Rx, K=64 (KM=256), 32x32 pixels, 77 GHz / 1 GHz,
            10 point targets, 20 dB, 200 iterations.
* c2     -- Q=8, M=8, K=256 (KM=2048), 128x128 pixels, 60 point/extended
            targets (~1% support), 15 dB, run to relative residual 1e-4.
* c4     -- batched uneven frames: M=8, K=128 (KM=1024), per-frame N in
            {32^2, 48^2, 64^2, 96^2}, Q in {4, 6, 8}, support 0.5-3%,
            SNR U(10, 25) dB.
* c5     -- Q=8, M=8, K=256, 512x512 pixels (matrix-free operator).
* paper  -- the hyperparameters printed in Sec. IV (mu=3, beta=100,
            lambda=20, eps_abs=1e-4, eps_rel=1e-2, K_p=5, eps_p=1e-5) on a
            64x64 grid of 0.05 m cells, Q=4, M=8, 58-62 GHz chirp (4 GHz
            around 60 GHz), SNR 3 dB.  The paper does not state K; K=64 here.
"""

from __future__ import annotations

import numpy as np

from .geometry import make_geometry
from .scene import make_scene

CONFIGS = {
    "c1": dict(Q=4, M=4, K=64, n_side=32, side=4.0, radius=10.0, f0=77e9, bw=1e9,
               n_targets=10, snr_db=20.0, extended=False,
               mu=1.0, beta=1.0, gamma=1.0, lambda_frac=0.2,
               eps_abs=0.0, eps_rel=1e-4, max_iter=200, Kp=5, eps_p=1e-5),
    "c2": dict(Q=8, M=8, K=256, n_side=128, side=4.0, radius=10.0, f0=77e9, bw=1e9,
               n_targets=60, snr_db=15.0, extended=True,
               mu=1.0, beta=1.0, gamma=1.0, lambda_frac=0.2,
               eps_abs=0.0, eps_rel=1e-4, max_iter=2000, Kp=5, eps_p=1e-5),
    "c5": dict(Q=8, M=8, K=256, n_side=512, side=4.0, radius=10.0, f0=77e9, bw=1e9,
               n_targets=600, snr_db=15.0, extended=True,
               mu=1.0, beta=1.0, gamma=1.0, lambda_frac=0.2,
               eps_abs=0.0, eps_rel=1e-4, max_iter=2000, Kp=5, eps_p=1e-5),
    "paper": dict(Q=4, M=8, K=64, n_side=64, side=3.2, radius=10.0, f0=58e9, bw=4e9,
                  n_targets=20, snr_db=3.0, extended=True,
                  mu=3.0, beta=100.0, gamma=100.0, lambda_abs=20.0,
                  eps_abs=1e-4, eps_rel=1e-2, max_iter=2000, Kp=5, eps_p=1e-5),
}

# Batched uneven frames: per-frame parameters drawn from these sets.
C4_SIDES = (32, 48, 64, 96)
C4_QS = (4, 6, 8)


def config_geometry(name: str, **over):
    c = dict(CONFIGS[name])
    c.update(over)
    return make_geometry(c["Q"], c["M"], c["K"], c["n_side"], c["side"],
                         c["radius"], c["f0"], c["bw"])


def config_scene(name: str, seed: int, **over):
    c = dict(CONFIGS[name])
    c.update(over)
    g = config_geometry(name, **over)
    return make_scene(g, seed, c["n_targets"], c["snr_db"], c["extended"])


def c4_frames(n_frames: int, seed: int):
    """Per-frame (Q, n_side, support_fraction, snr_db, scene_seed) for a batch."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_frames):
        side = int(C4_SIDES[int(rng.integers(0, len(C4_SIDES)))])
        Q = int(C4_QS[int(rng.integers(0, len(C4_QS)))])
        frac = float(rng.uniform(0.005, 0.03))
        snr = float(rng.uniform(10.0, 25.0))
        out.append(dict(Q=Q, n_side=side, support=frac, snr_db=snr,
                        seed=int(seed * 100003 + i)))
    return out


def c4_scene(frame: dict):
    """Scene for one batched frame (M=8, K=128, extended targets)."""
    g = make_geometry(frame["Q"], 8, 128, frame["n_side"], 4.0, 10.0, 77e9, 1e9)
    # extended targets average ~2.5 pixels each
    n_t = max(1, int(round(frame["support"] * g.N / 2.5)))
    return make_scene(g, frame["seed"], n_t, frame["snr_db"], extended=True)
