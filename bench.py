"""Benchmark: time-to-NMSE <= 1e-3 of the sharing-ADMM radar imager on one MI355X.

Workload c2: Q=8 sensors on a 10 m circle, M=8 Rx + 1 Tx each, K=256 LFM
samples (KM = 2048 rows per sensor), 128x128 = 16384 pixels, 60 point /
extended targets (~1% support), 15 dB SNR, scene seed 100 (synthetic; the
paper's scene is not published).  mu = beta = gamma = 1, lambda = 0.2
lambda_max, eps_rel = 1e-4.  The FP64 oracle's optimum image x_ref and lambda
are stored in tests/golden (written by tests/golden/make_refs.py).

One step = one complete solve from the measurements (resident in HBM) to the
first iteration whose image has NMSE <= 1e-3 against x_ref, including the FP64
factor build (Gram + Cholesky + inverse) and every pixel elimination.  The
headline `value` is the pruned (accelerated, Alg. 1) FP32 solve; the plain
FP32 solve is timed beside it.

    python bench.py [--steps K] [--warmup W] [--no-cpu] [--gpus 1]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("time-to-NMSE≤1e-3 vs FP64 oracle: learned+pruned vs plain SADMM; "
          "iters/s; HBM GB/s")
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
INT8_PEAK_TOPS = 5000.0        # dense int8 matrix peak, tera-ops/s
# int8 operations per complex multiply-add of the integer Gram: 13 digit pairs
# x 4 real products x 2 (multiply + add)
INT8_OPS_PER_CMAC = 13 * 4 * 2
PMC_SUMMARY = os.path.join(ROOT, "profiles", "gram_i8_c2_pmc.json")
GRAM_SOURCES = ("paper_2307_08606_amd/csrc/gram_i8.hip", "paper_2307_08606_amd/csrc/gram.h")


def gram_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in GRAM_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the integer Gram kernel from the committed
    rocprofv3 counter summary, or None when the kernel source changed since."""
    try:
        pm = json.load(open(PMC_SUMMARY))
    except (OSError, ValueError):
        return None
    if pm.get("source_sha256") != gram_source_hash():
        return None
    return pm.get("traffic_bytes_per_launch")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--storage", default="fp32", choices=["fp32", "fp16", "bf16", "fp64"])
    ap.add_argument("--only", default="", choices=["", "pruned", "plain", "iter", "c4", "c4batch"],
                    help="'pruned' or 'plain' to time one variant; 'iter' runs only steady "
                         "iterations (c2 FP32, 40; c5 matrix-free, 10) for counter runs; "
                         "'c4' runs only the batched-frames leg and prints its figures; 'c4batch' "
                         "only its batched solves (one warm-up, one timed), for kernel traces")
    ap.add_argument("--copy-calib", action="store_true",
                    help="run a plain 1 GiB device copy (counter calibration) and exit")
    return ap.parse_args()


def load_refs():
    gdir = os.path.join(ROOT, "tests", "golden")
    info = json.load(open(os.path.join(gdir, "c2_seed100.json")))
    x_ref = np.load(os.path.join(gdir, "c2_seed100_xref.npy"))
    return info, x_ref


def make_solver(lib, g, hp, prune, storage, stream):
    s = lib.Solver(g.Q, g.K, g.M, g.N, storage=storage, prune=prune, kkt=False,
                   reuse_factor=False, max_iter=200, stop=True, check_every=4,
                   Kp=5, eps_p=1e-5, eps_abs=0.0, eps_rel=1e-4, stream=stream, **hp)
    for q in range(g.Q):
        s.set_operator_geometry(q, g.tx[q], g.rx[q], g.pix, g.f0, g.bw)
    return s


def time_variant(torch, s, y_dev, steps, warmup):
    for _ in range(warmup):
        s.solve(y_dev)
    s.set_profiling(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    lib_ms = []
    for _ in range(steps):
        infos.append(s.solve(y_dev))
        lib_ms.append(s.timing()["total_ms"])
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    stats = s.kernel_stats()
    s.set_profiling(0)
    return wall, infos, lib_ms, stats


def cpu_baseline(sc, info, k_star):
    """The FP64 oracle on the whole workload: oracle.solve of the plain method
    with all 8 sensors for k* iterations (k* = the iterations the oracle needs
    for NMSE <= 1e-3, stored by tests/golden/make_refs.py), factor build
    included, operator generation excluded."""
    import oracle
    from scenegen import steering
    g = sc.geom
    A = [steering(g, q) for q in range(g.Q)]
    p = oracle.Params(mu=info["mu"], beta=info["beta"], gamma=info["gamma"], lam=info["lam"],
                      eps_abs=0.0, eps_rel=1e-4, max_iter=k_star, stop=False)
    t0 = time.perf_counter()
    R = oracle.solve(A, sc.y, p)
    ms = (time.perf_counter() - t0) * 1e3
    del A
    try:
        from threadpoolctl import threadpool_info
        cores = max(int(p.get("num_threads", 1)) for p in threadpool_info()) or os.cpu_count()
    except Exception:
        cores = os.cpu_count()
    return dict(value=round(ms, 1), unit="ms", cores=int(cores), kind="oracle",
                sample=f"whole workload: oracle.solve (FP64, plain SADMM) with all {g.Q} sensors for "
                       f"k*={R.iters} iterations, factor build included, operator generation excluded")


def probes(torch, lib):
    """Roofline denominators measured on this device: 1 GiB non-temporal copy
    and read, register-only int8 (16x16x64 and 32x32x32) and FP64 matrix
    loops; the published figures beside them."""
    return dict(hbm_copy_GBps=round(lib.probe_bandwidth_gbps("copy"), 1),
                hbm_read_GBps=round(lib.probe_bandwidth_gbps("read"), 1),
                int8_mfma_16x16x64_TOPs=round(lib.probe_mfma_tops("i8"), 1),
                int8_mfma_32x32x32_TOPs=round(lib.probe_mfma_tops("i8_32"), 1),
                fp64_mfma_TFLOPs=round(lib.probe_mfma_tops("f64"), 2),
                published=dict(hbm_GBps=HBM_PEAK_GBS, int8_TOPs=INT8_PEAK_TOPS,
                               fp64_TFLOPs=FP64_PEAK_TFLOPS))


def asadmm_leg(torch, lib, stream, g, hp, y_dev, xref_dev, eps_list=(1e-4, 1e-5), reps=2):
    """The paper's comparison (Sec. IV): accelerated (SSC pruning, Alg. 1) vs
    plain SADMM, both FP32, run to the relative residual tolerance.  Solve
    time (factor build and every prune event included), iterations,
    max_q N_q / N per iteration and the final NMSE against the FP64 optimum."""
    out = {}
    for eps in eps_list:
        r = {}
        for name, prune in (("plain", False), ("pruned", True)):
            s = lib.Solver(g.Q, g.K, g.M, g.N, storage="fp32", prune=prune,
                           reuse_factor=False, max_iter=400, stop=True, check_every=4, Kp=5,
                           eps_p=1e-5, eps_abs=0.0, eps_rel=eps, stream=stream, **hp)
            for q in range(g.Q):
                s.set_operator_geometry(q, g.tx[q], g.rx[q], g.pix, g.f0, g.bw)
            s.set_reference(xref_dev, nmse_target=0.0)
            s.solve(y_dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                i = s.solve(y_dev)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / reps
            fr = s.history("max_active_frac")
            nm = s.history("nmse")
            tm = s.timing()
            r[name] = dict(ms=round(ms, 2), iters=i["iters"], status=i["status"],
                           factor_ms=round(tm["factor_ms"], 2), iter_ms=round(tm["iter_ms"], 2),
                           final_nmse=float(nm[-1]) if len(nm) else None,
                           prune_events=i["prune_events"], reinstated=i["reinstated"],
                           final_active_frac=round(float(fr[-1]), 4) if len(fr) else 1.0,
                           mean_active_frac=round(float(np.mean(fr)), 4) if len(fr) else 1.0,
                           active_frac_curve=[round(float(v), 4) for v in fr[::max(1, len(fr) // 16)]])
            s.close()
        r["pruned"]["time_saving"] = round(1.0 - r["pruned"]["ms"] / r["plain"]["ms"], 4)
        r["pruned"]["iteration_time_saving"] = round(1.0 - r["pruned"]["iter_ms"] / max(r["plain"]["iter_ms"], 1e-9), 4)
        out[f"{eps:g}"] = r
    return out


def c5_asadmm_leg(torch, lib, stream, hp, max_iter=60):
    """Matrix-free 512 x 512 scene: plain vs pruned (Alg. 1) run to
    eps_rel = 1e-4 or max_iter; no FP64 optimum exists at this size, so the
    pruned image is compared with the plain one (same support expected)."""
    from scenegen import config_geometry, make_scene
    g5 = config_geometry("c5")
    sc5 = make_scene(g5, 100, 600, 15.0, extended=True)
    y5 = torch.from_numpy(np.ascontiguousarray(sc5.y)).to("cuda")
    r, img = {}, {}
    for name, prune in (("plain", False), ("pruned", True)):
        s = lib.Solver(g5.Q, g5.K, g5.M, g5.N, storage="mf", prune=prune,
                       reuse_factor=False, max_iter=max_iter, stop=True, check_every=4, Kp=5,
                       eps_p=1e-5, eps_abs=0.0, eps_rel=1e-4, stream=stream, **hp)
        for q in range(g5.Q):
            s.set_operator_geometry(q, g5.tx[q], g5.rx[q], g5.pix, g5.f0, g5.bw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        i = s.solve(y5)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        fr = s.history("max_active_frac")
        tm = s.timing()
        img[name] = s.image()
        r[name] = dict(ms=round(ms, 1), iters=i["iters"], status=i["status"],
                       factor_ms=round(tm["factor_ms"], 1), iter_ms=round(tm["iter_ms"], 1),
                       prune_events=i["prune_events"], reinstated=i["reinstated"],
                       final_active_frac=round(float(fr[-1]), 4) if len(fr) else 1.0,
                       mean_active_frac=round(float(np.mean(fr)), 4) if len(fr) else 1.0)
        s.close()
    d = img["pruned"] - img["plain"]
    r["pruned_vs_plain_nmse"] = float(np.vdot(d, d).real / max(np.vdot(img["plain"], img["plain"]).real, 1e-300))
    r["time_saving"] = round(1.0 - r["pruned"]["ms"] / r["plain"]["ms"], 4)
    return r


def batch_leg(torch, lib, stream, reps=2, n_check=8,
              legs=("fp32_plain_sequential", "fp32_plain_batched", "sequential", "batched",
                    "shared_batched", "ttn_fp32_plain_sequential", "ttn_fp32_plain_batched",
                    "ttn_sequential", "ttn_batched", "ttn_shared_batched")):
    """c4: 256 independent frames of uneven sensor count (4, 6, 8) and grid
    (32^2 .. 96^2 pixels), M = 8, K = 128, operators generated on the device,
    a fresh factor per solve.  Two configurations: plain SADMM with the
    operator stored in FP32 (fp32_plain_*), and the accelerated one (SSC
    pruning, operator stored as planar BF16 with FP32 arithmetic, FP64 factor
    and FP32 corrections at iterations 2, 4, 8, then every 10).  Each is timed
    solving the frames one by one (*sequential) and as one batch (*batched:
    one launch per kernel for all frames), after one tile autotune per
    pixel-count bucket and storage.  The frames of one (Q, N) class share the
    array geometry, hence the operator: *shared_batched solves each class as
    one batch of handles borrowing one FP32 operator and its factor (plain
    SADMM; one factor build per class and call; the products of all frames
    of a class as multi-right-hand-side products).  Two stopping modes: every
    frame run to
    eps_rel = 1e-4, and (ttn_*) every frame stopped at the first iteration
    with NMSE <= 1e-3 against the FP64 solve of the same frame (eps_rel =
    1e-7, computed first, outside the timing).  NMSE of a sample of the
    converged frames against those FP64 solves."""
    from scenegen.configs import c4_scene
    info = json.load(open(os.path.join(ROOT, "tests", "golden", "c4_batch256_seed7.json")))
    frames = info["frames"]
    scenes = [c4_scene(fr) for fr in frames]
    base = dict(prune=True, kkt=False, reuse_factor=False, max_iter=300, stop=True, check_every=8,
                Kp=5, eps_p=1e-5, eps_abs=0.0, eps_rel=1e-4, stream=stream, mu=info["mu"],
                beta=info["beta"], gamma=info["gamma"])
    configs = {"fp32_plain": dict(storage="fp32", prune=False),
               "bf16": dict(storage="bf16", refine_every=10)}

    def handle(i, **kw):
        g = scenes[i].geom
        s = lib.Solver(g.Q, g.K, g.M, g.N, lam=frames[i]["lam"], **{**base, **kw})
        for q in range(g.Q):
            s.set_operator_geometry(q, g.tx[q], g.rx[q], g.pix, g.f0, g.bw)
        return s

    mark = torch.zeros(1, device="cuda")

    def timed(fn):
        fn()
        mark.add_(1.0)                  # a one-element kernel: bounds the timed solves in traces
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            infos = fn()
        torch.cuda.synchronize()
        mark.add_(1.0)
        return dict(ms=(time.perf_counter() - t0) * 1e3 / reps, iters=[i["iters"] for i in infos],
                    status=[i["status"] for i in infos])

    ys = [torch.from_numpy(np.ascontiguousarray(sc.y)).to("cuda") for sc in scenes]
    order = sorted(range(len(frames)), key=lambda i: (scenes[i].geom.N * scenes[i].geom.Q, i))
    pick = [order[int(round(j * (len(order) - 1) / max(n_check - 1, 1)))] for j in range(n_check)]
    # FP64 solves of every frame needed (the time-to-NMSE references and the
    # sampled accuracy check), 64 frames per batch
    need = sorted(set(pick) | (set(range(len(frames))) if any(l.startswith("ttn_") for l in legs) else set()))
    xref, ref_status = {}, {}
    for c0 in range(0, len(need), 64):
        part = need[c0:c0 + 64]
        rs = [handle(i, storage="fp64", prune=False, eps_rel=1e-7, max_iter=3000, check_every=16)
              for i in part]
        infos = lib.solve_batch(rs, [ys[i] for i in part])
        for i, r, inf in zip(part, rs, infos):
            xref[i] = torch.from_numpy(r.image()).to("cuda")
            ref_status[i] = inf["status"]
        for r in rs:
            r.close()
    out, widths, images = {}, {}, {}
    for cname, ckw in configs.items():
        prefix = "fp32_plain_" if cname == "fp32_plain" else ""
        mine = [l for l in legs if l.replace("ttn_", "") in (prefix + "sequential", prefix + "batched")]
        if not mine:
            continue
        for i, fr in enumerate(frames):              # one tune per pixel-count bucket
            if (cname, fr["n_side"]) not in widths:
                s = handle(i, **ckw)
                widths[(cname, fr["n_side"])] = s.autotune(ys[i], 8)
                s.close()
        solvers = [handle(i, **ckw) for i in range(len(frames))]
        for ttn in (False, True):
            if not any(l.startswith("ttn_") == ttn for l in mine):
                continue
            for i, s in enumerate(solvers):
                s.set_reference(xref[i] if ttn else None, 1e-3 if ttn else 0.0)
            for leg in mine:
                if leg.startswith("ttn_") != ttn:
                    continue
                if leg.endswith("sequential"):
                    out[leg] = timed(lambda: [s.solve(y) for s, y in zip(solvers, ys)])
                else:
                    out[leg] = timed(lambda: lib.solve_batch(solvers, ys))
                if not ttn:
                    for i in pick:
                        images[(cname, i)] = solvers[i].image()
        free, total = torch.cuda.mem_get_info()
        out[f"{cname}_device_mem_in_use_GB"] = round((total - free) / 1e9, 1)
        for s in solvers:
            s.close()
    if any(l.replace("ttn_", "") == "shared_batched" for l in legs):
        classes = {}
        for i, fr in enumerate(frames):
            classes.setdefault((fr["Q"], fr["n_side"]), []).append(i)
        groups = []
        for key in sorted(classes):
            idx = classes[key]
            for c0 in range(0, len(idx), 64):          # at most 64 scenes per shared batch
                part = idx[c0:c0 + 64]
                g = scenes[part[0]].geom
                src = handle(part[0], storage="fp32", prune=False)
                kw = {**base, "prune": False}
                hs = [src] + [lib.Solver(g.Q, g.K, g.M, g.N, storage="fp32", lam=frames[i]["lam"],
                                         share=src, **kw) for i in part[1:]]
                groups.append((part, hs))

        def run_shared():
            infos = [None] * len(frames)
            for part, hs in groups:
                for i, inf in zip(part, lib.solve_batch(hs, [ys[i] for i in part])):
                    infos[i] = inf
            return infos

        for ttn in (False, True):
            leg = ("ttn_" if ttn else "") + "shared_batched"
            if leg not in legs:
                continue
            for part, hs in groups:
                for i, h in zip(part, hs):
                    h.set_reference(xref[i] if ttn else None, 1e-3 if ttn else 0.0)
            out[leg] = timed(run_shared)
            if not ttn:
                for part, hs in groups:
                    for i, h in zip(part, hs):
                        if i in pick:
                            images[("fp32_shared", i)] = h.image()
        out["shared_classes"] = len(classes)
        for part, hs in groups:
            for h in reversed(hs):
                h.close()
    nm = []
    for i in pick:
        z64 = xref[i].cpu().numpy()
        d = dict(frame=i, Q=scenes[i].geom.Q, N=scenes[i].geom.N, ref_status=ref_status[i])
        for cname in list(configs) + ["fp32_shared"]:
            if (cname, i) in images:
                z = images[(cname, i)]
                d[f"{cname}_nmse"] = float(np.linalg.norm(z - z64) ** 2 / np.linalg.norm(z64) ** 2)
        nm.append(d)
    out["frames"] = len(frames)
    out["widths"] = {f"{c}_{k}": v for (c, k), v in sorted(widths.items())}
    out["nmse_vs_fp64"] = nm
    out["refs_converged"] = all(v == 0 for v in ref_status.values())
    out["sum_QN"] = int(sum(sc.geom.Q * sc.geom.N for sc in scenes))
    it_b = out["batched" if "batched" in out else legs[-1]]["iters"]
    out["sum_iters_QN"] = int(sum(it * sc.geom.Q * sc.geom.N for it, sc in zip(it_b, scenes)))
    return out


def c1_leg(torch, lib, stream, iters=200, reps=5):
    """c1 workload (Q=4, M=4, K=64, N=32^2, seed 0, lambda = 0.2 lambda_max
    from the stored reference): a solve of exactly `iters` iterations (stop
    test off) with its factor already built, FP32 storage, replayed from the
    iteration graph; the shape is latency-bound (8 MiB of operator)."""
    from scenegen import config_scene
    ref = json.load(open(os.path.join(ROOT, "tests", "golden", "c1_seed0.json")))
    sc = config_scene("c1", 0)
    g = sc.geom
    s = lib.Solver(g.Q, g.K, g.M, g.N, storage="fp32", prune=False, reuse_factor=True, max_iter=iters,
                   stop=False, check_every=iters, stream=stream, mu=ref["mu"], beta=ref["beta"],
                   gamma=ref["gamma"], lam=ref["lam"])
    for q in range(g.Q):
        s.set_operator_geometry(q, g.tx[q], g.rx[q], g.pix, g.f0, g.bw)
    y = torch.from_numpy(np.ascontiguousarray(sc.y)).to("cuda")
    s.solve(y)                                     # factor and graph
    ms = []
    for _ in range(reps):
        s.solve(y)
        ms.append(s.timing()["iter_ms"])
    s.close()
    it_ms = float(np.median(ms)) / iters
    return dict(iter_us=it_ms * 1e3, iters_per_s=1e3 / it_ms)


def shared_leg(torch, lib, stream, info, S=32, iters=31):
    """S frames of the c2 geometry (scene seeds 100..100+S-1) sharing one FP32
    operator: one solve_batch iterates all of them with multi-right-hand-side
    products.  Per-iteration time of the whole batch = (time of `iters`
    iterations - time of 1 iteration) / (iters - 1), factor built beforehand."""
    from scenegen import config_geometry, make_scene
    g = config_geometry("c2")
    hp = dict(mu=info["mu"], beta=info["beta"], gamma=info["gamma"], lam=info["lam"])
    ys = [torch.from_numpy(np.ascontiguousarray(make_scene(g, 100 + i, 60, 15.0, extended=True).y)).to("cuda")
          for i in range(S)]

    def handles(max_iter):
        src = lib.Solver(g.Q, g.K, g.M, g.N, storage="fp32", prune=False, reuse_factor=True,
                         max_iter=max_iter, stop=False, check_every=max_iter, stream=stream, **hp)
        for q in range(g.Q):
            src.set_operator_geometry(q, g.tx[q], g.rx[q], g.pix, g.f0, g.bw)
        return [src] + [lib.Solver(g.Q, g.K, g.M, g.N, storage="fp32", prune=False, max_iter=max_iter,
                                   stop=False, check_every=max_iter, stream=stream, share=src, **hp)
                        for _ in range(S - 1)]

    ms = {}
    for n in (1, iters):
        hs = handles(n)
        lib.solve_batch(hs, ys)              # builds the shared factor
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lib.solve_batch(hs, ys)
        torch.cuda.synchronize()
        ms[n] = (time.perf_counter() - t0) * 1e3
        for h in reversed(hs):
            h.close()
    it_ms = (ms[iters] - ms[1]) / (iters - 1)
    flops = 2 * 8.0 * g.Q * g.K * g.M * g.N * S       # forward + adjoint complex MACs
    return dict(S=S, iter_ms=it_ms, frame_iters_per_s=S / (it_ms * 1e-3),
                product_tflops=flops / (it_ms * 1e-3) / 1e12)


def c3_leg(torch, lib, stream, g, hp, y_dev, xref_dev, reps=3):
    """c2 shapes with the operator stored as planar FP16 / BF16 (FP32
    arithmetic, FP64 factor) and corrected toward the operator regenerated in
    FP32 from the geometry: pruned time-to-NMSE <= 1e-3 with a correction every
    3 iterations (status read every iteration), the image NMSE once the solve
    meets eps_rel = 1e-4 with a correction every 10 iterations and without any,
    and the steady iteration time with and without it (40 iterations, status
    read every 8, so corrections at 16 and 32)."""
    def solver(st, every, **kw):
        base = dict(storage=st, prune=True, kkt=False, reuse_factor=False, max_iter=200, stop=True,
                    check_every=4, Kp=5, eps_p=1e-5, eps_abs=0.0, eps_rel=1e-4, refine_every=every,
                    stream=stream)
        base.update(kw)
        s = lib.Solver(g.Q, g.K, g.M, g.N, **base, **hp)
        for q in range(g.Q):
            s.set_operator_geometry(q, g.tx[q], g.rx[q], g.pix, g.f0, g.bw)
        return s

    out = {}
    for st in ("fp16", "bf16"):
        r = {}
        s = solver(st, 3, check_every=1)
        s.set_reference(xref_dev, nmse_target=1e-3)
        s.solve(y_dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            i = s.solve(y_dev)
        torch.cuda.synchronize()
        r["ttn_ms"] = (time.perf_counter() - t0) * 1e3 / reps
        r["ttn_iters"] = i["iters"]
        r["ttn_nmse"] = i["nmse"]
        s.close()
        for every in (0, 10):
            s = solver(st, every)
            s.set_reference(xref_dev, nmse_target=0.0)
            i = s.solve(y_dev)
            r[f"conv_nmse_{every}"] = i["nmse"]
            r[f"conv_iters_{every}"] = i["iters"]
            s.close()
            s = solver(st, every, prune=False, reuse_factor=True, max_iter=40, stop=False, check_every=8)
            s.solve(y_dev)
            s.set_profiling(1)
            s.solve(y_dev)
            r[f"iter_ms_{every}"] = s.timing()["iter_ms"] / 40
            s.close()
        out[st] = r
    return out


def iter_only(torch, lib, stream, g, hp, y_dev, storage):
    """Steady iterations only (factor built beforehand, outside any counter
    window that filters on the iteration kernels): 40 c2 iterations in the
    given storage and 10 c5 matrix-free iterations."""
    from scenegen import config_geometry, make_scene
    out = {}
    s = lib.Solver(g.Q, g.K, g.M, g.N, storage=storage, prune=False, reuse_factor=True, max_iter=40,
                   stop=False, check_every=8, stream=stream, **hp)
    for q in range(g.Q):
        s.set_operator_geometry(q, g.tx[q], g.rx[q], g.pix, g.f0, g.bw)
    s.solve(y_dev)
    s.solve(y_dev)
    out["c2_iter_ms"] = s.timing()["iter_ms"] / 40
    s.close()
    g5 = config_geometry("c5")
    sc5 = make_scene(g5, 100, 600, 15.0, extended=True)
    y5 = torch.from_numpy(np.ascontiguousarray(sc5.y)).to("cuda")
    s5 = lib.Solver(g5.Q, g5.K, g5.M, g5.N, storage="mf", prune=False, reuse_factor=True, max_iter=10,
                    stop=False, check_every=10, stream=stream, **hp)
    for q in range(g5.Q):
        s5.set_operator_geometry(q, g5.tx[q], g5.rx[q], g5.pix, g5.f0, g5.bw)
    s5.solve(y5)
    s5.solve(y5)
    out["c5_mf_iter_ms"] = s5.timing()["iter_ms"] / 10
    s5.close()
    torch.cuda.synchronize()
    print(json.dumps(out))


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the engine is single-GPU "
              "(sharding over several GPUs is not built).", file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_calib:
        n = 1 << 30
        a = torch.empty(n, dtype=torch.uint8, device="cuda")
        b = torch.empty(n, dtype=torch.uint8, device="cuda")
        a.fill_(1)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n}))
        return
    from paper_2307_08606_amd import sadmm_lib as lib
    from scenegen import config_scene

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream().cuda_stream
    info, x_ref = load_refs()
    sc = config_scene("c2", info["seed"])
    g = sc.geom
    hp = dict(mu=info["mu"], beta=info["beta"], gamma=info["gamma"], lam=info["lam"])
    y_dev = torch.from_numpy(np.ascontiguousarray(sc.y)).to("cuda")
    xref_dev = torch.from_numpy(x_ref).to("cuda")

    if args.only == "iter":
        iter_only(torch, lib, stream, g, hp, y_dev, args.storage)
        return
    if args.only == "c4":
        print(json.dumps(batch_leg(torch, lib, stream)), flush=True)
        return
    if args.only == "c4batch":
        r = batch_leg(torch, lib, stream, reps=1, n_check=0, legs=("batched",))
        print(json.dumps(dict(frames=r["frames"], batched_ms=round(r["batched"]["ms"], 1),
                              iters=int(sum(r["batched"]["iters"])), sum_iters_QN=r["sum_iters_QN"])),
              flush=True)
        return

    results = {}
    variants = [("pruned", True), ("plain", False)]
    if args.only:
        variants = [v for v in variants if v[0] == args.only]
    for name, prune in variants:
        s = make_solver(lib, g, hp, prune, args.storage, stream)
        s.set_reference(xref_dev, nmse_target=1e-3)
        wall, infos, lib_ms, stats = time_variant(torch, s, y_dev, args.steps, args.warmup)
        results[name] = dict(ms_per_step=wall, lib_ms=lib_ms, infos=infos, stats=stats,
                             timing=s.timing())
        # steady-state iteration rate on a warm factor (no time-to-NMSE stop)
        if name == "plain":
            sw = lib.Solver(g.Q, g.K, g.M, g.N, storage=args.storage, prune=False,
                            reuse_factor=True, max_iter=40, stop=False, check_every=8,
                            stream=stream, **hp)
            for q in range(g.Q):
                sw.set_operator_geometry(q, g.tx[q], g.rx[q], g.pix, g.f0, g.bw)
            sw.solve(y_dev)                      # builds the factor
            sw.set_profiling(1)                  # iterations replayed from the graph
            sw.solve(y_dev)
            t = sw.timing()
            sw.set_profiling(2)                  # per-stage events (direct launches)
            sw.solve(y_dev)
            results["steady"] = dict(iter_ms=t["iter_ms"], iters=40, stats=sw.kernel_stats(),
                                     staged_iter_ms=sw.timing()["iter_ms"])
            sw.close()
        s.close()

    head = results[variants[0][0]]
    st = head["stats"]
    # Roofline of the dominant kernel of the headline solve: the Gram of the
    # factor build (the integer int8 kernel for non-FP64 storage).  achieved =
    # the method's flops (8 per complex multiply-add over the Hermitian
    # triangle) per second; for the integer kernel the peak is the dense int8
    # matrix rate, and the 13 digit-pair products per multiply-add it issues
    # are reported separately (int8_issue_frac).
    n, ms, work = st["gram"]
    integer = args.storage != "fp64"
    achieved = work / (ms * 1e-3) / 1e12
    dens = probes(torch, lib) if not args.only else None
    if integer:
        roof = dict(bound="mfma", achieved=round(achieved, 1), peak=INT8_PEAK_TOPS, unit="TFLOP/s",
                    frac=round(achieved / INT8_PEAK_TOPS, 4), traffic=measured_traffic(),
                    kernel="gram_i8_kernel (exact integer Gram Ahat Ahat^H, int8 16x16x64 MFMA)",
                    peak_kind="dense int8 matrix rate, published (TOP/s)",
                    int8_ops_per_method_flop=INT8_OPS_PER_CMAC / 8,
                    int8_issue_frac=round(achieved * INT8_OPS_PER_CMAC / 8 / INT8_PEAK_TOPS, 4))
        if dens:
            roof["frac_of_measured_peak"] = round(
                achieved / max(dens["int8_mfma_16x16x64_TOPs"], dens["int8_mfma_32x32x32_TOPs"]), 4)
    else:
        roof = dict(bound="mfma", achieved=round(achieved, 2), peak=FP64_PEAK_TFLOPS, unit="TFLOP/s",
                    frac=round(achieved / FP64_PEAK_TFLOPS, 4), traffic=None,
                    kernel="herk_mfma_kernel (FP64 Gram Ahat Ahat^H on 16x16x4 FP64 MFMA)")
        if dens:
            roof["frac_of_measured_peak"] = round(achieved / dens["fp64_mfma_TFLOPs"], 4)
    per_launch = work / max(n, 1)
    roof["launches"] = n
    roof["avg_launch_ms"] = round(ms / max(n, 1), 4)
    roof["flops_per_launch"] = per_launch
    roof["class_ms_per_solve"] = {k: round(v[1] / args.steps, 3) for k, v in st.items() if v[0]}

    # matrix-free operator at 512 x 512 pixels (c5 geometry): steady-state rate
    if not args.only:
        from scenegen import config_geometry, make_scene
        g5 = config_geometry("c5")
        sc5 = make_scene(g5, 100, 600, 15.0, extended=True)
        s5 = lib.Solver(g5.Q, g5.K, g5.M, g5.N, storage="mf", prune=False, reuse_factor=True,
                        max_iter=10, stop=False, check_every=10, stream=stream, **hp)
        for q in range(g5.Q):
            s5.set_operator_geometry(q, g5.tx[q], g5.rx[q], g5.pix, g5.f0, g5.bw)
        y5 = torch.from_numpy(np.ascontiguousarray(sc5.y)).to("cuda")
        s5.solve(y5)                                 # factor build (one-time)
        t5 = s5.timing()
        s5.set_profiling(1)
        s5.solve(y5)
        t5b = s5.timing()
        s5.set_profiling(2)
        s5.solve(y5)
        st5 = s5.kernel_stats()
        s5.close()
        el = 2.0 * g5.Q * g5.KM * g5.N               # generated entries per iteration
        results["c5_mf"] = dict(factor_ms=t5["factor_ms"], iter_ms=t5b["iter_ms"] / 10,
                                stats=st5, elems_per_iter=el)

    # c1 (Q=4, KM=256, N=32^2): latency-bound steady iterations, 200 fixed
    # iterations replayed from the iteration graph, FP32, lambda = 0.2 lambda_max
    if not args.only:
        results["c1"] = c1_leg(torch, lib, stream)
    # batched uneven frames (c4): 256 frames of different Q and grid size
    # solved one by one and as one batch (one launch per kernel for all frames)
    if not args.only:
        results["c4"] = batch_leg(torch, lib, stream)
    # frames of one geometry sharing the c2 operator (multi-RHS products)
    if not args.only and args.storage == "fp32":
        results["shared"] = shared_leg(torch, lib, stream, info)

    # 16-bit operator storage with the correction (c3)
    if not args.only and args.storage == "fp32":
        results["c3"] = c3_leg(torch, lib, stream, g, hp, y_dev, xref_dev)
    # accelerated vs plain SADMM run to the residual tolerance (Sec. IV)
    if not args.only and args.storage == "fp32":
        results["asadmm"] = asadmm_leg(torch, lib, stream, g, hp, y_dev, xref_dev)
        results["c5_asadmm"] = c5_asadmm_leg(torch, lib, stream, hp)

    steady = results.get("steady")
    extra = {}
    if steady:
        sst = steady["stats"]
        extra["iters_per_s"] = round(steady["iters"] / (steady["iter_ms"] * 1e-3), 1)
        for k in ("fwd", "xupd", "wprod"):
            nn, mm, ww = sst[k]
            if nn:
                extra[f"{k}_GBps"] = round(ww / (mm * 1e-3) / 1e9, 1)
                extra[f"{k}_hbm_frac"] = round(ww / (mm * 1e-3) / 1e9 / HBM_PEAK_GBS, 3)
                extra[f"{k}_avg_us"] = round(mm / nn * 1e3, 1)
                if dens:
                    extra[f"{k}_read_probe_frac"] = round(ww / (mm * 1e-3) / 1e9 / dens["hbm_read_GBps"], 3)
    if "c5_mf" in results:
        r5 = results["c5_mf"]
        extra["c5_matrix_free_factor_ms"] = round(r5["factor_ms"], 1)
        extra["c5_matrix_free_iter_ms"] = round(r5["iter_ms"], 3)
        extra["c5_matrix_free_Gelem_per_s"] = round(r5["elems_per_iter"] / (r5["iter_ms"] * 1e-3) / 1e9, 1)
        extra["c5_matrix_free_stage_ms"] = {k: round(v[1] / max(v[0], 1), 3)
                                            for k, v in r5["stats"].items() if v[0]}
    if "shared" in results:
        r = results["shared"]
        extra["c2_shared_frames"] = r["S"]
        extra["c2_shared_batch_iter_ms"] = round(r["iter_ms"], 3)
        extra["c2_shared_frame_iters_per_s"] = round(r["frame_iters_per_s"], 1)
        extra["c2_shared_product_tflops"] = round(r["product_tflops"], 1)
    if "c3" in results:
        for st, r in results["c3"].items():
            extra[f"c3_{st}_refined_ttn_ms"] = round(r["ttn_ms"], 2)
            extra[f"c3_{st}_refined_ttn_iters"] = r["ttn_iters"]
            extra[f"c3_{st}_converged_nmse"] = {"refined": r["conv_nmse_10"], "uncorrected": r["conv_nmse_0"]}
            extra[f"c3_{st}_iter_ms"] = {"refined": round(r["iter_ms_10"], 4),
                                         "uncorrected": round(r["iter_ms_0"], 4)}
    if "asadmm" in results:
        extra["c2_asadmm_vs_sadmm"] = results["asadmm"]
    if "c5_asadmm" in results:
        extra["c5_asadmm_vs_sadmm"] = results["c5_asadmm"]
    if dens:
        extra["measured_denominators"] = dens
    if "c1" in results:
        extra["c1_iters_per_s"] = round(results["c1"]["iters_per_s"], 1)
        extra["c1_iter_us"] = round(results["c1"]["iter_us"], 2)
    if "c4" in results:
        r4 = results["c4"]
        extra["c4_frames"] = r4["frames"]
        extra["c4_storage"] = {"fp32_plain": "FP32 operator, plain SADMM",
                               "accelerated": "BF16 planes (FP32 arithmetic, FP64 factor, correction "
                                              "every 10 iterations), SSC pruning"}
        for k in ("fp32_plain_sequential", "fp32_plain_batched", "sequential", "batched", "shared_batched",
                  "ttn_fp32_plain_sequential", "ttn_fp32_plain_batched", "ttn_sequential", "ttn_batched",
                  "ttn_shared_batched"):
            if k in r4:
                extra[f"c4_{k}_frames_per_s"] = round(r4["frames"] / (r4[k]["ms"] * 1e-3), 1)
                extra[f"c4_{k}_ms"] = round(r4[k]["ms"], 1)
                it = np.array(r4[k]["iters"])
                extra[f"c4_{k}_iters"] = dict(min=int(it.min()), median=float(np.median(it)),
                                              max=int(it.max()), total=int(it.sum()))
                # status 0: converged; 2: NMSE target reached (time-to-NMSE legs)
                extra[f"c4_{k}_all_stopped_as_asked"] = all(
                    st == (2 if k.startswith("ttn_") else 0) for st in r4[k]["status"])
        for pre in ("", "ttn_"):
            for leg in ("batched", "shared_batched"):
                if pre + leg in r4 and pre + "fp32_plain_sequential" in r4:
                    name = "accelerated_batched" if leg == "batched" else "shared_batched"
                    extra[f"c4_{pre}{name}_vs_plain_fp32_sequential"] = round(
                        r4[pre + "fp32_plain_sequential"]["ms"] / r4[pre + leg]["ms"], 2)
        extra["c4_fp64_references_converged"] = r4["refs_converged"]
        extra["c4_tile_widths"] = r4["widths"]
        for c in ("fp32_plain", "bf16", "fp32_shared"):
            vals = [d[f"{c}_nmse"] for d in r4["nmse_vs_fp64"] if f"{c}_nmse" in d]
            if vals:
                extra[f"c4_{c}_max_nmse_vs_fp64"] = max(vals)
            if f"{c}_device_mem_in_use_GB" in r4:
                extra[f"c4_{c}_device_mem_in_use_GB"] = r4[f"{c}_device_mem_in_use_GB"]
        extra["c4_nmse_vs_fp64"] = r4["nmse_vs_fp64"]
    for name in ("pruned", "plain"):
        if name in results:
            r = results[name]
            i0 = r["infos"][-1]
            extra[f"{name}_ms"] = round(r["ms_per_step"], 2)
            extra[f"{name}_iters"] = i0["iters"]
            extra[f"{name}_nmse"] = i0["nmse"]
            extra[f"{name}_factor_ms"] = round(r["timing"]["factor_ms"], 2)
            extra[f"{name}_max_active_frac"] = round(i0["max_active_frac"], 4)
    cpu = None
    if not args.no_cpu:
        k_star = info["runs"]["plain"]["iters_to_nmse_1e3"] or 5
        cpu = cpu_baseline(sc, info, k_star)

    line = {
        "metric": METRIC,
        "value": round(head["ms_per_step"], 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "fp32", "fp64": "f64", "fp16": "fp16-storage/fp32",
                  "bf16": "bf16-storage/fp32"}[args.storage],
        "data": "synthetic",
        "config": {"workload": f"c2 {variants[0][0]} SADMM: Q=8, M=8, K=256 (KM=2048), "
                               "N=128x128, 60 targets, 15 dB, seed 100, NMSE<=1e-3 vs FP64 "
                               "oracle optimum, factor build included",
                   "storage": args.storage},
        "roofline": roof,
        "cpu_baseline": cpu,
        **extra,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
