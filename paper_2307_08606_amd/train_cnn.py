"""Train the pixel-pruning CNN on the GPU with labels from the engine's own
pruned solves.

    python -m paper_2307_08606_amd.train_cnn --workload c2 --scenes 48 --epochs 6 \\
        --out paper_2307_08606_amd/weights/cnn_c2.npz

For each seeded training scene (scenegen, seeds 10000 + i; held-out seeds
30000 + i are never used here): the matched-filter images |A_q^H y_q| are the
input, and the label of pixel n is 1 when the converged accelerated solve
(freeze elimination, 60 iterations, so every pixel whose value has settled is
eliminated) has z_n = 0 and has eliminated n from every sensor.  The network (sadmm_cnn_*) is trained with its own forward/backward
kernels and Adam.  Prints per-epoch loss and held-out precision/recall at the
elimination threshold.

Each scene also reports the fraction of pixels that could be eliminated at
x = 0 from every sensor without the optimality re-check reinstating them:
max_q |x_q[n]| / max_m |x_q[m]| <= 10 eps_rel (the re-check's default
tolerance; frozen at 0, a pixel's coordinate step is about |x_q[n]|).  With
--measure-only only that is measured (any workload, c5 included) and printed
as JSON.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from paper_2307_08606_amd import sadmm_lib as lib  # noqa: E402
from scenegen import CONFIGS, config_geometry, config_scene  # noqa: E402


def make_solver(g, cfg, lam, stream, max_iter=60, storage="fp32"):
    s = lib.Solver(g.Q, g.K, g.M, g.N, storage=storage, prune=True, kkt=False, reuse_factor=True,
                   max_iter=max_iter, stop=False, check_every=8, Kp=cfg["Kp"], eps_p=cfg["eps_p"],
                   eps_abs=0.0, eps_rel=cfg["eps_rel"], mu=cfg["mu"], beta=cfg["beta"],
                   gamma=cfg["gamma"], lam=lam, stream=stream)
    for q in range(g.Q):
        s.set_operator_geometry(q, g.tx[q], g.rx[q], g.pix, g.f0, g.bw)
    return s


def scene_sample(s, g, seed, workload):
    sc = config_scene(workload, seed)
    mf = s.matched_filter(sc.y)                       # (Q, N)
    x = (mf / mf.max()).reshape(g.Q, g.n_side, g.n_side).astype(np.float32)
    s.set_reference(None)
    s.solve(sc.y)
    z = s.image()
    masks = np.stack([s.active_mask(q).astype(bool) for q in range(g.Q)])
    t = ((np.abs(z) == 0) & (~masks).all(axis=0)).astype(np.float32)
    return x, t.reshape(g.n_side, g.n_side), zero_eliminable(s, g)


def zero_eliminable(s, g, tol=None):
    """Fraction of pixels whose every sensor value is within the re-check's
    tolerance of 0 (relative to that sensor's largest), and of (q, n) pairs."""
    tol = 10.0 * s.params.eps_rel if tol is None else tol
    ax = np.abs(np.stack([s.sensor_image(q) for q in range(g.Q)]))
    small = ax <= tol * ax.max(axis=1, keepdims=True)
    return float(small.all(axis=0).mean()), float(small.mean())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--lam", type=float, default=None, help="absolute lambda (default: stored c2 value)")
    ap.add_argument("--scenes", type=int, default=48)
    ap.add_argument("--heldout", type=int, default=8)
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--channels", type=int, default=32)
    ap.add_argument("--pos-weight", type=float, default=1.0)
    ap.add_argument("--threshold", type=float, default=0.9)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=os.path.join(HERE, "weights", "cnn_c2.npz"))
    ap.add_argument("--measure-only", action="store_true",
                    help="only measure the zero-eliminable fractions of --scenes scenes")
    a = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    cfg = CONFIGS[a.workload]
    lam = a.lam
    if lam is None:
        ref = json.load(open(os.path.join(os.path.dirname(HERE), "tests", "golden", "c2_seed100.json")))
        lam = ref["lam"]
    g = config_geometry(a.workload)
    s = make_solver(g, cfg, lam, stream, storage="mf" if g.N > 128 * 128 else "fp32")
    t0 = time.time()
    if a.measure_only:
        fr = []
        for i in range(a.scenes):
            sc = config_scene(a.workload, 10000 + i)
            s.solve(sc.y)
            fr.append(zero_eliminable(s, g))
        print(json.dumps(dict(workload=a.workload, scenes=a.scenes, lam=lam, iterations=60,
                              tol=10.0 * s.params.eps_rel,
                              pixel_fraction=[f[0] for f in fr], pair_fraction=[f[1] for f in fr],
                              seconds=round(time.time() - t0, 1))), flush=True)
        return
    train = [scene_sample(s, g, 10000 + i, a.workload)[:2] for i in range(a.scenes)]
    held_full = [scene_sample(s, g, 30000 + i, a.workload) for i in range(a.heldout)]
    held = [h[:2] for h in held_full]
    pos = float(np.mean([t.mean() for _, t in train]))
    zel = [h[2] for h in held_full]
    print(f"labels: {a.scenes} training scenes, positive fraction {pos:.3f}, "
          f"{time.time() - t0:.1f} s; zero-eliminable pixels {np.mean([z[0] for z in zel]):.2e}, "
          f"(q, n) pairs {np.mean([z[1] for z in zel]):.2e} (held-out scenes)", flush=True)
    net = lib.Cnn(g.Q, a.channels, g.n_side, g.n_side, stream=stream)
    rng = np.random.default_rng(a.seed)
    init = {}
    for k, shp in net.shapes().items():
        if k.startswith("W"):
            fan = shp[1] * 9
            init[k] = rng.standard_normal(shp) * np.sqrt(2.0 / fan)
        else:
            init[k] = np.zeros(shp)
    net.set_params(init)
    for ep in range(a.epochs):
        order = rng.permutation(len(train))
        losses = [net.train_step(train[i][0], train[i][1], a.pos_weight, a.lr) for i in order]
        tp = fp = fn = 0
        for x, t in held:
            pr = net.forward(x) >= a.threshold
            tp += int((pr & (t > 0.5)).sum())
            fp += int((pr & (t < 0.5)).sum())
            fn += int((~pr & (t > 0.5)).sum())
        prec = tp / max(tp + fp, 1)
        rec = tp / max(tp + fn, 1)
        print(f"epoch {ep}: loss {np.mean(losses):.4f}  held-out precision {prec:.4f} "
              f"recall {rec:.4f} at p >= {a.threshold}", flush=True)
    params = net.get_params()
    os.makedirs(os.path.dirname(a.out), exist_ok=True)
    np.savez(a.out, **{k: v.astype(np.float32) for k, v in params.items()},
             meta=json.dumps(dict(workload=a.workload, Q=g.Q, C=a.channels, H=g.n_side,
                                  W=g.n_side, lam=lam, scenes=a.scenes, epochs=a.epochs,
                                  lr=a.lr, pos_weight=a.pos_weight, threshold=a.threshold,
                                  heldout_precision=prec, heldout_recall=rec,
                                  positive_fraction=pos)))
    print(f"saved {a.out}")
    # held-out effect on the solve: time-to-NMSE<=1e-3 with and without the CNN
    import json as _j
    for thr in (0.5, 0.9, 0.99):
        ev = evaluate(g, cfg, lam, stream, net, thr, a.workload, a.heldout)
        print("heldout " + _j.dumps(ev), flush=True)


def evaluate(g, cfg, lam, stream, net, thr, workload, n):
    """Held-out scenes: plain solve to the FP32 optimum (reference), then
    time-to-NMSE<=1e-3 (factor build included) without and with the CNN."""
    out = dict(threshold=thr, plain_ms=[], cnn_ms=[], cnn_pruned=[], cnn_nmse_final=[],
               cnn_iters=[], plain_iters=[])
    for i in range(n):
        sc = config_scene(workload, 30000 + i)
        ref = lib.Solver(g.Q, g.K, g.M, g.N, storage="fp32", prune=False, reuse_factor=True,
                         max_iter=60, stop=False, mu=cfg["mu"], beta=cfg["beta"],
                         gamma=cfg["gamma"], lam=lam, stream=stream)
        for q in range(g.Q):
            ref.set_operator_geometry(q, g.tx[q], g.rx[q], g.pix, g.f0, g.bw)
        ref.solve(sc.y)
        xr = ref.image()
        ref.close()
        for name, use in (("plain", False), ("cnn", True)):
            s = lib.Solver(g.Q, g.K, g.M, g.N, storage="fp32", prune=True, kkt=True,
                           reuse_factor=False, max_iter=200, stop=True, Kp=cfg["Kp"],
                           eps_p=cfg["eps_p"], eps_rel=cfg["eps_rel"], mu=cfg["mu"],
                           beta=cfg["beta"], gamma=cfg["gamma"], lam=lam, stream=stream)
            for q in range(g.Q):
                s.set_operator_geometry(q, g.tx[q], g.rx[q], g.pix, g.f0, g.bw)
            if use:
                s.set_pruning_cnn(net, thr)
            s.set_reference(xr, 1e-3)
            info = s.solve(sc.y)
            out[f"{name}_ms"].append(round(s.timing()["total_ms"], 2))
            out[f"{name}_iters"].append(info["iters"])
            if use:
                out["cnn_pruned"].append(int(g.N - s.active_indices(0).size))
                s.set_reference(None)
                s.solve(sc.y)
                z = s.image()
                out["cnn_nmse_final"].append(float(np.linalg.norm(z - xr) ** 2 / np.linalg.norm(xr) ** 2))
            s.close()
    return out


if __name__ == "__main__":
    main()
