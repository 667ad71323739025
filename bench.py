#!/usr/bin/env python3
"""Throughput of one ADMM bundle-adjustment iteration on one MI355X.

A step is one full ADMM iteration over every observation of the workload:
local robust-LM solves with the deferred scaled-dual update (Eqs. 9, 12,
13), point and camera consensus (Eqs. 10, 11), residual norms and rho
balancing.  Inputs are generated, validated and uploaded before the timed
region; the timed region runs exactly --steps iterations.

Prints one JSON line: obs-updates/s (observations x iterations / second),
the local-solve kernel on the HBM roofline (the iteration's algorithmic
state bytes over its launch time, HIP events on the library's stream; its
vector-ALU figures beside it), the FP64 oracle pinned to one host core on iterations 2-3 of the
same workload (its first iteration is the reference for the GPU-vs-oracle
check printed with the result), and, for the 2M-observation trajectory
workload, the time to the oracle's final inlier RMSE for the plain and the
learned start.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "obs-updates/s per ADMM iter (2M obs); time-to-RMSE, warm-start vs plain LM"
FP32_VECTOR_PEAK_TFLOPS = 78.6   # 256 CU x 64 lanes x 2 (FMA) x 2.4 GHz, non-packed FP32
FP32_PACKED_PEAK_TFLOPS = 157.3  # the same with packed FP32 (two FMAs per lane and cycle)
HBM_PEAK_GBS = 8000.0
BF16_MFMA_PEAK_TFLOPS = 2500.0   # dense
MLP_FLOPS_PER_OBS = 2 * (32 * 128 + 128 * 128 + 128 * 16)   # padded 32 -> 128 -> 128 -> 16

WORKLOADS = {
    # name: (scene maker kwargs, solver options, description)
    "trajectory": dict(scene="config2", opts=dict(precision="fp32", loss="huber", loss_param=2.0, rho=1e5,
                                                   rho_balancing=True, rho_min=1e5, rho_max=1e7),
                       desc="1000 cameras on a random-walk trajectory, 200000 points, Zipf tracks 2..60, "
                            "5% outliers; Huber 2 px, rho 1e5 with residual balancing in [1e5, 1e7]; "
                            "FP32 local / FP64 consensus"),
    "trajectory_blocks": dict(scene="config2", opts=dict(precision="fp32", loss="huber", loss_param=2.0, rho=1e5,
                                                         rho_balancing=True, rho_min=1e5, rho_max=1e7,
                                                         camera_blocks=True),
                              desc="as trajectory, with block local updates: the observations of a camera form "
                                   "blocks of up to 64 that share one camera copy (Sec. 3.1.4); 5 LM steps"),
    "trajectory_blocks2": dict(scene="config2", opts=dict(precision="fp32", loss="huber", loss_param=2.0, rho=1e5,
                                                          rho_balancing=True, rho_min=1e5, rho_max=1e7,
                                                          camera_blocks=True, block_cameras=2),
                               desc="as trajectory, with two-camera blocks (Sec. 3.1.4, kappa = 2): cameras in "
                                    "pairs, each pair's points in runs of 64 with one copy per block point and "
                                    "camera; 5 LM steps"),
    "trajectory_euler": dict(scene="config2_euler", opts=dict(precision="fp32", loss="huber", loss_param=2.0,
                                                              rho=1e5, rho_balancing=True, rho_min=1e5, rho_max=1e7,
                                                              camera="euler"),
                             desc="the trajectory workload (seed 7) with the paper's camera of Eq. (1): Euler "
                                  "angles and translation, known focal length, no distortion; FP32 local / FP64 "
                                  "consensus"),
    "trajectory_shard8": dict(scene="config2_shard8", opts=dict(precision="fp32", loss="huber", loss_param=2.0,
                                                                rho=1e5, rho_balancing=True, rho_min=1e5, rho_max=1e7),
                              desc="one rank's share of the trajectory workload when 8 GPUs partition the "
                                   "observations by point: every 8th point's whole track and the cameras that see "
                                   "them; FP32 local / FP64 consensus"),
    "sphere": dict(scene="config1", opts=dict(precision="fp32", loss="student_t", loss_param=4.0, rho=1e3),
                   desc="100 cameras on a sphere cap, 20000 points, 8..15 cameras per point; Student-t nu 4, "
                        "rho 1e3; FP32 local / FP64 consensus"),
    "sphere_fp64": dict(scene="config1", opts=dict(precision="fp64", loss="student_t", loss_param=4.0, rho=1e3),
                        desc="as sphere, FP64 throughout"),
    "ring": dict(scene="config0", opts=dict(precision="fp64", loss="huber", loss_param=2.0, rho=1e4),
                 desc="10 cameras on a circle, 200 points, all 2000 observations; Huber 2 px, rho 1e4; FP64"),
    "batched": dict(scene="config3", opts=dict(precision="fp32", loss="student_t", loss_param=4.0, rho=1e3),
                    desc="64 independent sphere-cap problems (seeds 1000..1063), cameras log-uniform 5..300, "
                         "2k..300k observations each, in the same launches; Student-t nu 4, rho 1e3; "
                         "FP32 local / FP64 consensus"),
}


def make_scenes(kind):
    """List of the workload's problems."""
    from scenes import make_config0, make_config1, make_config2, make_config3
    if kind == "config3":
        return make_config3()
    if kind == "config2_shard8":
        from scenes import point_shard
        return [point_shard(make_config2(), 0, 8)]
    if kind == "config2_euler":
        # seed 7: its perturbed Euler start keeps every point in front of its cameras
        return [make_config2(seed=7, camera="euler")]
    return [{"config0": make_config0, "config1": make_config1, "config2": make_config2}[kind]()]


# iterations of the tuning handle: every local-solve schedule candidate (8)
# and every consensus segment schedule (3) once, with room to spare
TUNING_ITERATIONS = 16


# every source of device code: the HIP files and the headers they include
KERNEL_SOURCES = ("dba_kernels.hip", "dba_block_kernels.hip", "mlp_kernels.hip", "dba_device.h", "dba_internal.h",
                  "dba_layout.h", "block_device.h", "mlp_device.h")


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1708_07954_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:12]


# committed counter summary of each workload's local-solve kernel
COUNTER_SUMMARIES = {"trajectory": "local_solve_trajectory_counters.md",
                     "trajectory_blocks": "block_local_trajectory.md",
                     "trajectory_euler": "kernels_trajectory_euler_2M.md",
                     "sphere": "kernels_sphere_230k.md",
                     "sphere_fp64": "kernels_sphere_230k.md",
                     "ring": "kernels_ring_2k.md",
                     "batched": "kernels_batched_3M.md",
                     "trajectory_blocks2": "block2_local_trajectory.md",
                     "trajectory_shard8": "kernels_trajectory_shard8.md"}


def recorded_traffic(workload):
    """HBM bytes per local-solve launch from the committed counter summary,
    if it was taken on the current kernel source."""
    if workload not in COUNTER_SUMMARIES:
        return None, None
    path = os.path.join(ROOT, "profiles", COUNTER_SUMMARIES[workload])
    if not os.path.exists(path):
        return None, None
    text = open(path).read()
    src = re.search(r"kernel_source_hash:\s*(\w+)", text)
    # a summary covering several workloads keys each figure by workload name
    tb = (re.search(r"traffic_bytes_per_launch\[" + re.escape(workload) + r"\]:\s*([0-9.eE+]+)", text)
          or re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text))
    if not src or not tb or src.group(1) != kernel_source_hash():
        return None, None
    return float(tb.group(1)), path


def measure_copy_bandwidth(torch):
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    return 5 * 2 * src.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9


def oracle_target(workload):
    """Final inlier RMSE of the stored FP64 oracle run of the workload
    (written by tests/golden/make_golden.py), or None."""
    path = os.path.join(ROOT, "tests", "golden", f"{workload}.npz")
    if not os.path.exists(path):
        return None, None
    import numpy as np
    z = np.load(path, allow_pickle=False)
    return float(z["stats"][1]), int(z["iterations"])


def _time_to_target(binding, scene, kw, goal, max_iters, net=None):
    """Iterations and wall time of one configuration to an inlier RMSE goal:
    per-kernel times over the first 20 iterations of a fresh run; the
    crossing iteration from per-iteration RMSE checks; then a fresh run of
    exactly that many iterations, timed (graph instantiation included), and
    the steady per-iteration time of the 50 iterations after it."""
    import numpy as np
    import torch
    inl = ~scene.outlier

    def make():
        s = binding.Solver(**kw)
        if net is not None:
            binding.dba_set_mlp(s.h, net[0], net[1])
        s.set_scene(scene)
        s.set_eval_mask(inl)
        return s
    s = make()
    binding.dba_set_kernel_timing(s.h, True)
    s.iterate(20)
    torch.cuda.synchronize()
    kt = binding.dba_kernel_times(s.h)
    s.close()
    kernels = {k: v[0] / v[1] for k, v in kt.items() if v[1]}
    s = make()
    hit, last = None, None
    for k in range(1, max_iters + 1):
        s.iterate(1)
        last = s.residuals(want_rmse=True)["rmse_masked"]
        if not np.isfinite(last) or last > 1e6:
            break
        if last <= goal:
            hit = k
            break
    s.close()
    out = {"iterations": hit, "inlier_rmse_at_stop": last, "kernel_ms": kernels}
    if hit is None:
        out["seconds"] = None
        return out
    s = make()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.iterate(hit)
    torch.cuda.synchronize()
    out["seconds"] = time.perf_counter() - t0
    s.iterate(20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.iterate(50)
    torch.cuda.synchronize()
    out["ms_per_iter_steady"] = (time.perf_counter() - t0) * 20.0
    s.close()
    return out


def tuned_schedule(binding, scenes, kw):
    """Launch and segment schedules the autotuner picks for a configuration,
    on a handle of its own (the tuning iterations are real iterations, which
    the measured runs then do not repeat)."""
    tuner = binding.Solver(**kw).set_scenes(scenes)
    tuner.iterate(TUNING_ITERATIONS)
    sched = binding.dba_schedule(tuner.h)
    seg = binding.dba_segment_schedule(tuner.h)
    tuner.close()
    assert seg["tuned"] > 0, "the consensus schedule was not tuned within the tuning iterations"
    return dict(block_waves=sched["block_waves"], persistent=sched["persistent"],
                segment_schedule=seg["segment_schedule"])


def time_to_rmse(binding, scene, opts, sched, target, max_iters=400, learned_steps=(1, 2, 3, 4, 5)):
    """Wall time of plain 5-step LM, of the paper's L-BFGS local solver for
    the Huber misfit (5 and 10 iterations), of block local updates (one camera
    copy per 64 observations, Sec. 3.1.4) and of the learned start (+ k LM
    steps) to reach the oracle's final inlier RMSE (within 0.5 %)."""
    from paper_1708_07954_amd import warmstart
    goal = target * 1.005

    def run(kw, net=None):
        return _time_to_target(binding, scene, kw, goal, max_iters, net)

    res = {"target_inlier_rmse": target, "reached_when_within": 0.005, "max_iterations": max_iters}
    res["plain_lm5"] = run(dict(opts, lm_steps=5, block_waves=sched["block_waves"], persistent=sched["persistent"],
                                segment_schedule=sched.get("segment_schedule", 0)))
    print(f"[bench] time-to-RMSE plain: {res['plain_lm5']}", file=sys.stderr, flush=True)
    if opts.get("loss") == "huber":
        for k in (5, 10):
            res[f"lbfgs{k}"] = run(dict(opts, solver="lbfgs", lm_steps=k, block_waves=sched["block_waves"],
                                        persistent=sched["persistent"],
                                        segment_schedule=sched.get("segment_schedule", 0)))
            print(f"[bench] time-to-RMSE L-BFGS, {k} iterations: {res[f'lbfgs{k}']}", file=sys.stderr, flush=True)
    # block local updates run other kernels: each configuration with the
    # schedule the autotuner picks for it
    for k in (1, 2, 5):
        kw = dict(opts, lm_steps=k, camera_blocks=True)
        res[f"blocks_lm{k}"] = run(dict(kw, **tuned_schedule(binding, [scene], kw)))
        print(f"[bench] time-to-RMSE blocks, {k} LM steps: {res[f'blocks_lm{k}']}", file=sys.stderr, flush=True)
    for k in (1, 2, 5):
        kw = dict(opts, lm_steps=k, camera_blocks=True, block_cameras=2)
        res[f"blocks2_lm{k}"] = run(dict(kw, **tuned_schedule(binding, [scene], kw)))
        print(f"[bench] time-to-RMSE two-camera blocks, {k} LM steps: {res[f'blocks2_lm{k}']}", file=sys.stderr,
              flush=True)
    best = lambda key: min((res[f"{key}_lm{k}"]["seconds"] for k in (1, 2, 5)
                            if res[f"{key}_lm{k}"]["seconds"] is not None), default=None)
    b1, b2 = best("blocks"), best("blocks2")
    res["blocks2_over_blocks_time"] = (b2 / b1) if (b1 and b2) else None
    if not learned_steps:
        t_plain = res["plain_lm5"]["seconds"]
        tb = min((res[f"blocks_lm{k}"]["seconds"] for k in (1, 2, 5) if res[f"blocks_lm{k}"]["seconds"] is not None),
                 default=None)
        res["blocks_over_plain_time"] = (tb / t_plain) if (tb is not None and t_plain) else None
        return res
    params, norm, rep = warmstart.train_default()
    res["training"] = {"pairs": rep["pairs"], "collect_seconds": rep["collect_seconds"],
                       "train_seconds": rep["train_seconds"], "final_epoch_loss": rep["epoch_loss"][-1],
                       "scenes": "10 trajectory-family scenes, 100 cameras, 20000 points, seeds 2000-2009"}
    for k in learned_steps:
        res[f"learned_lm{k}"] = run(dict(opts, start="learned", learned_lm_steps=k, block_waves=sched["block_waves"],
                                         persistent=sched["persistent"], segment_schedule=sched.get("segment_schedule", 0)),
                                    net=(params, norm))
        print(f"[bench] time-to-RMSE learned+{k}: {res[f'learned_lm{k}']}", file=sys.stderr, flush=True)
    # the fused learned-start kernel on the BF16 MFMA roofline: network
    # FLOPs per observation x observations / kernel time (a lower bound on the
    # network's own rate, the kernel also runs the guard and the LM steps)
    L = scene.n_obs
    for k in learned_steps:
        t = res[f"learned_lm{k}"]["kernel_ms"].get("learned")
        if t:
            res[f"learned_lm{k}"]["mlp_tflops_lower_bound"] = MLP_FLOPS_PER_OBS * L / (t * 1e-3) / 1e12
    res["mlp_flops_per_obs"] = MLP_FLOPS_PER_OBS
    res["bf16_mfma_peak_tflops"] = BF16_MFMA_PEAK_TFLOPS
    t_plain = res["plain_lm5"]["seconds"]
    tb = min((res[f"blocks_lm{k}"]["seconds"] for k in (1, 2, 5) if res[f"blocks_lm{k}"]["seconds"] is not None),
             default=None)
    res["blocks_over_plain_time"] = (tb / t_plain) if (tb is not None and t_plain) else None
    best = min((res[f"learned_lm{k}"]["seconds"] for k in learned_steps
                if res[f"learned_lm{k}"]["seconds"] is not None), default=None)
    res["learned_over_plain_time"] = (best / t_plain) if (best is not None and t_plain) else None
    return res


def block_size_sweep(binding, scene, opts, target, sizes=(64, 48, 32, 16, 8, 4, 2, 1), steps=(1, 2, 5),
                     max_iters=300):
    """Block local updates (Sec. 3.1.4) with pi observations per block, one
    camera per block: iterations and wall time to the oracle's final inlier
    RMSE (within 0.5 %) for every pi and LM step count.  One block is one
    wavefront, so the cost of an iteration follows the number of blocks."""
    goal = target * 1.005
    res = {"target_inlier_rmse": target, "reached_when_within": 0.005, "max_iterations": max_iters,
           "schedule": {"block_waves": 1, "persistent": 0}}
    for pi in sizes:
        for k in steps:
            kw = dict(opts, camera_blocks=True, block_points=pi, lm_steps=k, block_waves=1, persistent=0)
            r = _time_to_target(binding, scene, kw, goal, max_iters)
            res[f"pi{pi}_lm{k}"] = {q: r.get(q) for q in ("iterations", "seconds", "ms_per_iter_steady",
                                                       "inlier_rmse_at_stop")}
            res[f"pi{pi}_lm{k}"]["local_ms"] = r["kernel_ms"].get("local")
            print(f"[bench] block size {pi}, {k} LM steps: {res[f'pi{pi}_lm{k}']}", file=sys.stderr, flush=True)
    return res


def size_sweep(binding, opts, factors=(0.0625, 0.125, 0.25, 0.5, 1.0, 2.0, 4.0, 8.0), iters=50):
    """Time of one iteration against the number of observations L (the
    paper's cost model: the local solves and the dual update are O(L), the
    consensus O(L + m + n)).  Up to L = 2M: one trajectory scene of 1000 f
    cameras and 200000 f points (seed 2; f = 1 is the 2M workload).  Above:
    f copies of the 2M problem as independent problems in the same launches
    (a longer or denser trajectory's perturbed start puts points behind
    cameras, which the library rejects).  Each size with its own autotuned
    schedule; iterations replayed from the captured graph.  A least-squares
    line t = a + b L summarises the points."""
    import numpy as np
    import torch
    from scenes import make_config2

    base = make_config2()
    rows = []
    for f in factors:
        if f <= 1.0:
            scenes = [make_config2(n_cams=int(round(1000 * f)), n_points=int(round(200000 * f)))]
        else:
            scenes = [base] * int(f)
        L = sum(sc.n_obs for sc in scenes)
        tuner = binding.Solver(**opts).set_scenes(scenes)
        tuner.iterate(TUNING_ITERATIONS)
        sched = binding.dba_schedule(tuner.h)
        seg = binding.dba_segment_schedule(tuner.h)["segment_schedule"]
        tuner.close()
        s = binding.Solver(block_waves=sched["block_waves"], persistent=sched["persistent"], segment_schedule=seg, **opts)
        s.set_scenes(scenes)
        s.iterate(20)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.iterate(iters)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / iters
        binding.dba_set_kernel_timing(s.h, True)
        s.iterate(10)
        torch.cuda.synchronize()
        kt = binding.dba_kernel_times(s.h)
        s.close()
        row = {"factor": f, "n_problems": len(scenes), "n_obs": L,
               "n_cams": sum(sc.n_cams for sc in scenes), "n_points": sum(sc.n_points for sc in scenes),
               "ms_per_iter": ms, "obs_updates_per_s": L / (ms * 1e-3), "schedule": sched,
               "kernel_ms": {k: v[0] / v[1] for k, v in kt.items() if v[1]}}
        rows.append(row)
        print(f"[bench] size {L} ({len(scenes)} problem(s)): {ms:.4f} ms/iteration, "
              f"{row['obs_updates_per_s']:.3e} obs-updates/s", file=sys.stderr, flush=True)
    L = np.array([r["n_obs"] for r in rows], dtype=float)
    t = np.array([r["ms_per_iter"] for r in rows])
    A = np.stack([np.ones_like(L), L], 1)
    (a, b), *_ = np.linalg.lstsq(A, t, rcond=None)
    fit = A @ np.array([a, b])
    r2 = 1.0 - ((t - fit) ** 2).sum() / ((t - t.mean()) ** 2).sum()
    return {"rows": rows, "fit_intercept_ms": float(a), "fit_ns_per_obs": float(b * 1e6), "fit_r2": float(r2),
            "max_rel_deviation_from_fit": float(np.max(np.abs(t - fit) / t))}


def convergence_study(binding, rho=100.0, iters=200, seeds=32, checkpoints=(0, 10, 25, 50, 100, 200)):
    """The paper's convergence study (Sec. 4.2, Fig. 3) with its camera
    (Eq. 1): 5 cameras, 10 points, all 50 observations, pixel noise 1;
    camera angles and positions started with noise 0.1, points with noise
    sigma = 0.2 .. 1.7; squared-l2 against Huber (delta 2) misfit, rho as
    given.  Every (sigma, seed) problem of one loss runs in the same
    batched launches (FP64); the medians over the seeds of the reprojection
    RMSE at the checkpoints and of the final point MSE against the ground
    truth are reported per sigma."""
    import numpy as np
    from scenes import make_sphere_scene
    sigmas = [round(0.2 + 0.15 * k, 2) for k in range(11)]
    scenes = [make_sphere_scene(seed=1000 + q, n_cams=5, n_points=10, k_lo=5, k_hi=5, radius=10.0, box=2.0,
                                rot_sigma=0.1, trans_sigma=0.1, point_sigma=sig, camera="euler")
              for sig in sigmas for q in range(seeds)]
    res = {"rho": rho, "iterations": iters, "seeds": seeds, "sigmas": sigmas, "checkpoints": list(checkpoints),
           "scene": "5 cameras on a sphere cap (radius 10) looking at the origin, 10 points in [-2, 2]^3, "
                    "all 50 observations, pixel noise 1, Euler camera (Eq. 1)"}
    for loss, lp in (("l2", 1.0), ("huber", 2.0)):
        s = binding.Solver(precision="fp64", camera="euler", loss=loss, loss_param=lp, rho=rho).set_scenes(scenes)
        curves = np.zeros((len(scenes), len(checkpoints)))
        done = 0
        for c, it in enumerate(checkpoints):
            s.iterate(it - done)
            done = it
            for q in range(len(scenes)):
                curves[q, c] = s.residuals(q, want_rmse=True)["rmse"]
        mse = np.array([np.mean(np.sum((s.params(q)[1] - sc.points_gt) ** 2, axis=1))
                        for q, sc in enumerate(scenes)])
        s.close()
        curves = curves.reshape(len(sigmas), seeds, len(checkpoints))
        mse = mse.reshape(len(sigmas), seeds)
        res[loss] = {"rmse_median": [[float(np.nanmedian(curves[k, :, c])) for c in range(len(checkpoints))]
                                     for k in range(len(sigmas))],
                     "final_point_mse_median": [float(np.nanmedian(mse[k])) for k in range(len(sigmas))]}
        print(f"[bench] convergence study {loss}: final RMSE medians "
              f"{[round(r[-1], 3) for r in res[loss]['rmse_median']]}", file=sys.stderr, flush=True)
    return res


def profile_learned(binding, wl):
    """Short learned-start run for counter collection: collects pairs on two
    training scenes, trains two epochs, then 20 learned-start iterations (3 LM
    steps) of the workload with kernel timing."""
    import torch
    from paper_1708_07954_amd import warmstart
    feats, deltas = warmstart.collect(warmstart.training_scenes()[:2], iters=20, per_iter=5000, seed=1)
    params, norm, rep = warmstart.train(feats, deltas, epochs=2)
    sc = make_scenes(wl["scene"])[0]
    s = binding.Solver(**dict(wl["opts"], start="learned", learned_lm_steps=3))
    binding.dba_set_mlp(s.h, params, norm)
    s.set_scene(sc)
    binding.dba_set_kernel_timing(s.h, True)
    s.iterate(20)
    torch.cuda.synchronize()
    kt = {k: v[0] / v[1] for k, v in binding.dba_kernel_times(s.h).items() if v[1]}
    s.close()
    print(json.dumps({"profile_learned": True, "n_obs": sc.n_obs, "pairs": rep["pairs"],
                      "train_seconds": rep["train_seconds"], "kernel_ms": kt,
                      "mlp_tflops_lower_bound": MLP_FLOPS_PER_OBS * sc.n_obs / (kt["learned"] * 1e-3) / 1e12}),
          flush=True)


def block_baseline_and_parity(binding, sc, opts):
    """Block local updates: the oracle's dense block solver timed on one core
    over the first blocks of the workload (a bounded sample, about 15 s), and
    the GPU after 3 iterations against the stored oracle run
    (tests/golden/trajectory_blocks.npz) when it exists."""
    import numpy as np
    import oracle
    o = dict(opts)
    b = oracle.BlockADMM(oracle.Problem.from_scene(sc), sc.cams_init, sc.points_init, block=64, loss=o["loss"],
                         loss_param=o["loss_param"], rho=o["rho"], lm_steps=o.get("lm_steps", 5))
    allowed = os.sched_getaffinity(0)
    core = min(allowed)
    os.sched_setaffinity(0, {core})
    n_obs, nb = 0, 0
    try:
        c0 = time.perf_counter()
        while time.perf_counter() - c0 < 15.0 and nb < b.n_blocks:
            ks = b.blk_obs[b.blk_off[nb]:b.blk_off[nb + 1]]
            j = int(b.blk_cam[nb])
            theta = np.concatenate([b.ycopy[nb], b.xcopy[ks].ravel()])
            oracle.block_local_solve(b.opts, sc.obs_uv[ks], b.cons_y[j], b.cons_x[sc.obs_point[ks]], theta,
                                     o["rho"], o["rho"], o.get("lm_steps", 5))
            n_obs += ks.shape[0]
            nb += 1
        dt = time.perf_counter() - c0
    finally:
        os.sched_setaffinity(0, allowed)
    base = {"value": n_obs / dt, "unit": "obs-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"block local solves of the first {nb} of {b.n_blocks} blocks ({n_obs} observations) of "
                      f"the first iteration, dense (9 + 3 x 64)-unknown LM, single-threaded FP64 C oracle pinned "
                      f"to core {core}, {dt:.1f} s on {cpu_model()}; consensus and duals (O(L), negligible) "
                      f"not included"}
    parity = None
    path = os.path.join(ROOT, "tests", "golden", "trajectory_blocks.npz")
    if os.path.exists(path):
        g = np.load(path, allow_pickle=False)
        if str(g["checksum"]) == sc.checksum():
            sys.path.insert(0, os.path.join(ROOT, "tests"))
            from _util import golden_points, param_rel_err
            chk = binding.Solver(**opts).set_scene(sc)
            chk.iterate(int(g["iterations"]))
            cams, pts = chk.params()
            rmse = chk.residuals(want_rmse=True)["rmse"]
            chk.close()
            parity = {"iterations": int(g["iterations"]),
                      "max_param_rel_err": param_rel_err(cams, pts[golden_points(g)], g["cams"], g["points"]),
                      "tolerance": 1e-3 if opts["precision"] == "fp32" else 1e-9,
                      "rmse_rel_diff": abs(rmse - float(g["stats"][0])) / float(g["stats"][0]),
                      "reference": "stored FP64 oracle run with block local updates"}
    return base, parity


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="trajectory", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-time-to-rmse", action="store_true",
                    help="skip the time-to-RMSE comparison (learned start vs plain LM)")
    ap.add_argument("--profile-learned", action="store_true",
                    help="only train the network briefly and run 20 learned-start iterations (for profilers)")
    ap.add_argument("--block-sweep", action="store_true",
                    help="trajectory workloads: also sweep the block size pi of the block local updates "
                         "(1..64 observations per block, 1 / 2 / 5 LM steps) to the oracle's final RMSE")
    ap.add_argument("--size-sweep", action="store_true",
                    help="also time one iteration at 0.125M..16M observations of trajectory problems "
                         "(the workload's options)")
    ap.add_argument("--convergence-study", action="store_true",
                    help="also run the paper's l2-vs-Huber convergence study (5 cameras, 10 points, Euler camera)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run a plain device copy of this size (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus_requested": args.gpus}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1708_07954_amd import binding, cost

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}), flush=True)
        sys.exit(1)
    wl = WORKLOADS[args.workload]
    if args.profile_learned:
        profile_learned(binding, wl)
        return
    t_gen = time.perf_counter()
    scenes = make_scenes(wl["scene"])
    L = sum(sc.n_obs for sc in scenes)
    t_gen = time.perf_counter() - t_gen
    opts = dict(wl["opts"])
    fp32 = opts["precision"] == "fp32"
    print(f"[bench] workload {args.workload}: {len(scenes)} problem(s), L={L}, generated in {t_gen:.1f}s",
          file=sys.stderr, flush=True)

    # launch schedule: autotuned once on a separate handle (tuning runs real,
    # bitwise-equivalent iterations), then fixed for the measured handle
    tuner = binding.Solver(**opts).set_scenes(scenes)
    tuner.iterate(TUNING_ITERATIONS)
    sched = binding.dba_schedule(tuner.h)
    seg = binding.dba_segment_schedule(tuner.h)
    assert seg["tuned"] > 0, "the consensus schedule was not tuned within the tuning iterations"
    sched["segment_schedule"] = seg["segment_schedule"]
    torch.cuda.synchronize()
    tuner.close()
    print(f"[bench] schedule {sched}", file=sys.stderr, flush=True)

    s = binding.Solver(block_waves=sched["block_waves"], persistent=sched["persistent"],
                       segment_schedule=sched["segment_schedule"], **opts).set_scenes(scenes)
    s.iterate(args.warmup)
    torch.cuda.synchronize()

    # timed region: K iterations in batches of 16, the local-solve kernel
    # (the roofline's kernel) of each batch's first iteration between two HIP
    # events on the library's stream and the rest of the batch replayed from
    # a graph (a sample of its launches: events around every launch would
    # slow the region they measure); the graphs are captured by a call
    # before the region
    binding.dba_set_kernel_timing(s.h, True, sampled=True)
    s.iterate(17)
    torch.cuda.synchronize()
    binding.dba_set_kernel_timing(s.h, True, sampled=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.iterate(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ktimes = binding.dba_kernel_times(s.h)
    ms_per_step = (t1 - t0) * 1e3 / max(args.steps, 1)
    value = L * args.steps / (t1 - t0)

    # the other kernels' durations, from a separate pass with every kernel
    # between events (after the timed region)
    binding.dba_set_kernel_timing(s.h, True)
    s.iterate(17)
    torch.cuda.synchronize()
    binding.dba_set_kernel_timing(s.h, True)
    s.iterate(min(args.steps, 64))
    torch.cuda.synchronize()
    for k, v in binding.dba_kernel_times(s.h).items():
        if k not in ("local", "learned"):
            ktimes[k] = v
    binding.dba_set_kernel_timing(s.h, False)

    # the same iterations replayed from the captured hipGraph (production path)
    s.iterate(16)
    torch.cuda.synchronize()
    g0 = time.perf_counter()
    s.iterate(args.steps)
    torch.cuda.synchronize()
    ms_graph = (time.perf_counter() - g0) * 1e3 / max(args.steps, 1)
    rep = s.residuals(want_rmse=True)
    print(f"[bench] {ms_per_step:.3f} ms/step (graph {ms_graph:.3f}) residuals {rep}", file=sys.stderr, flush=True)

    kt = {k: dict(avg_ms=(v[0] / v[1] if v[1] else None), launches=v[1]) for k, v in ktimes.items() if v[1]}
    local_ms = kt["local"]["avg_ms"]
    blocks = bool(opts.get("camera_blocks"))
    blocks2 = blocks and opts.get("block_cameras", 1) == 2
    if blocks2:
        import numpy as np
        copies = sum(len(np.unique((sc.obs_cam // 2).astype(np.int64) * sc.n_points + sc.obs_point)) for sc in scenes)
        flops_per_obs = cost.block2_flops_per_obs(opts.get("lm_steps", 5), L / copies)
    elif blocks:
        flops_per_obs = cost.block_flops_per_obs(opts.get("lm_steps", 5))
    else:
        flops_per_obs = cost.local_flops_per_obs(opts.get("lm_steps", 5), opts.get("camera", "angle_axis"))
    flops = flops_per_obs * L
    alu_achieved = flops / (local_ms * 1e-3) / 1e12
    traffic, traffic_src = recorded_traffic(args.workload)
    byt = cost.bytes_per_obs(fp32)
    if blocks2:
        bytes_obs = cost.block2_bytes_per_obs(fp32, L / copies)
    elif blocks:
        bytes_obs = cost.block_bytes_per_obs(fp32, cost.obs_per_block([sc.obs_cam for sc in scenes],
                                                                     opts.get("block_points", 64)))
    else:
        bytes_obs = byt["minimal"]
    # the local kernel on the HBM roofline: the iteration's algorithmic state
    # traffic (each observation's pixel, indexes, copies and scaled duals read
    # and written once) over the kernel's average launch time, against 8 TB/s
    hbm_achieved = bytes_obs * L / (local_ms * 1e-3) / 1e9
    roofline = {"kernel": "local (k_local_block2)" if blocks2 else "local (k_local_block)" if blocks else "local (k_local)",
                "bound": "hbm", "achieved": round(hbm_achieved, 3), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(hbm_achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "bytes_per_obs": bytes_obs, "obs_per_launch": L, "avg_launch_ms": local_ms,
                # the whole iteration (every kernel and gap) against the same bytes
                "step_frac": round(bytes_obs * L / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                # the same kernel on the vector-ALU roofline: this library's
                # count of its arithmetic against the non-packed peak it can
                # issue, and the published figure (which counts packed FP32)
                # with the flop counts of a local solve by a dense Cholesky
                # (8 500 per observation) and by Woodbury (3 300)
                "alu": {"flops_per_obs": flops_per_obs, "achieved_tflops": round(alu_achieved, 3),
                        "nonpacked_peak_tflops": FP32_VECTOR_PEAK_TFLOPS if fp32 else 78.6,
                        "frac_nonpacked": round(alu_achieved / (FP32_VECTOR_PEAK_TFLOPS if fp32 else 78.6), 4)}}
    if fp32 and not blocks:
        for name, per_obs in (("cholesky_8500", 8500), ("woodbury_3300", 3300)):
            roofline["alu"][f"frac_published_{name}"] = round(per_obs * L / (local_ms * 1e-3) / 1e12
                                                              / FP32_PACKED_PEAK_TFLOPS, 4)
        roofline["alu"]["published_fp32_vector_peak_tflops"] = FP32_PACKED_PEAK_TFLOPS
    cons_ms = kt["consensus"]["avg_ms"]
    consensus_line = {"avg_launch_ms": cons_ms,
                      "hbm_algorithmic_GBps": round(byt["consensus"] * L / (cons_ms * 1e-3) / 1e9, 1)}

    # measured device-copy bandwidth (1 GiB read + 1 GiB written), context for
    # the 8 TB/s HBM peak; skipped in counter-calibration runs, whose only
    # plain copy must be the calibration probe
    copy_gbps = None
    if not args.copy_probe_mib:
        copy_gbps = measure_copy_bandwidth(torch)
        roofline["measured_copy_GBps"] = round(copy_gbps, 1)
        consensus_line["frac_of_measured_copy"] = round(consensus_line["hbm_algorithmic_GBps"] / copy_gbps, 4)
    consensus_line["hbm_peak_GBps"] = HBM_PEAK_GBS

    # optional plain copy, for scaling the FETCH_SIZE / WRITE_SIZE counters
    if args.copy_probe_mib:
        n = args.copy_probe_mib * (1 << 20) // 4
        a = torch.empty(n, dtype=torch.float32, device="cuda")
        b = torch.ones(n, dtype=torch.float32, device="cuda")
        for _ in range(3):
            a.copy_(b)
        torch.cuda.synchronize()

    out = {"metric": METRIC, "value": value, "unit": "obs-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32" if fp32 else "f64", "data": "synthetic",
           "config": {"workload": f"{args.workload}: {wl['desc']}", "n_obs": L, "n_problems": len(scenes),
                      "n_cams": sum(sc.n_cams for sc in scenes), "n_points": sum(sc.n_points for sc in scenes),
                      "scene_checksum": ",".join(sc.checksum() for sc in scenes[:4]) + ("..." if len(scenes) > 4 else ""),
                      "local_precision": "f32" if fp32 else "f64", "consensus_precision": "f64",
                      "lm_steps": opts.get("lm_steps", 5), "schedule": sched, "parallelism": "single GPU"},
           "ms_per_step_graph": ms_graph, "kernels": kt,
           "kernel_timing": "local: HIP events recorded on the library's stream around the first local launch "
                            "of each 16-iteration batch of the timed region, the rest of the batch replayed from "
                            "a graph; consensus, norms: a separate pass with every kernel between events",
           "roofline": roofline, "consensus": consensus_line,
           "residuals_after": {k: rep[k] for k in ("primal", "dual", "rho_x", "rmse", "iteration")}}
    if traffic_src:
        out["roofline"]["traffic_source"] = os.path.relpath(traffic_src, ROOT)

    if args.workload in ("trajectory", "trajectory_euler") and not args.no_time_to_rmse:
        target, its = oracle_target(args.workload)
        if target is not None:
            # the learned start belongs to the 9-parameter camera
            ttr = time_to_rmse(binding, scenes[0], opts, sched, target,
                               learned_steps=(1, 2, 3, 4, 5) if args.workload == "trajectory" else ())
            ttr["target_source"] = f"FP64 oracle, {its} iterations (tests/golden/{args.workload}.npz)"
            out["time_to_rmse"] = ttr

    if args.size_sweep and args.workload.startswith("trajectory"):
        out["size_sweep"] = size_sweep(binding, opts)

    if args.convergence_study:
        out["convergence_study"] = convergence_study(binding)

    if args.block_sweep and args.workload.startswith("trajectory"):
        target, its = oracle_target("trajectory")
        if target is not None:
            sw = block_size_sweep(binding, scenes[0], wl["opts"], target)
            sw["target_source"] = f"FP64 oracle, {its} iterations (tests/golden/trajectory.npz)"
            out["block_size_sweep"] = sw

    if not args.no_cpu_baseline and opts.get("camera_blocks"):
        out["cpu_baseline"], out["parity_vs_oracle"] = block_baseline_and_parity(binding, scenes[0], opts)
    elif not args.no_cpu_baseline:
        import oracle
        import numpy as np
        o = wl["opts"]
        # the oracle on one host core: iteration 1 is the parity reference,
        # iterations 2 and 3 are timed (median), as the CPU baseline
        allowed = os.sched_getaffinity(0)
        core = min(allowed)
        os.sched_setaffinity(0, {core})
        runs, first, times = [], [], []
        try:
            for sc in scenes:
                a = oracle.ADMM(oracle.Problem.from_scene(sc), sc.cams_init, sc.points_init, loss=o["loss"],
                                loss_param=o["loss_param"], rho=o["rho"], rho_balancing=o.get("rho_balancing", False),
                                camera=o.get("camera", "angle_axis"))
                a.opts.rho_min, a.opts.rho_max = o.get("rho_min", 1e-6), o.get("rho_max", 1e6)
                a.iterate(1)
                first.append((a.cons_y.copy(), a.cons_x.copy(), a.stats()[0]))
                runs.append(a)
            for _ in range(2):
                c0 = time.perf_counter()
                for a in runs:
                    a.iterate(1)
                times.append(time.perf_counter() - c0)
        finally:
            os.sched_setaffinity(0, allowed)
        dt = float(np.median(times))
        out["cpu_baseline"] = {"value": L / dt, "unit": "obs-updates/s", "cores": 1, "kind": "oracle",
                               "sample": f"ADMM iterations 2 and 3 (median) over all {L} observations "
                                         f"({len(scenes)} problem(s)), single-threaded FP64 C oracle pinned to "
                                         f"core {core}, {dt:.1f} s per iteration on {cpu_model()} "
                                         f"({os.cpu_count()} logical CPUs visible)"}
        # the same first iteration on the GPU, compared with the oracle
        chk = binding.Solver(**opts).set_scenes(scenes)
        chk.iterate(1)
        sys.path.insert(0, os.path.join(ROOT, "tests"))
        from _util import param_rel_err
        worst, rdiff = 0.0, 0.0
        for q, (cy, cx, rmse) in enumerate(first):
            cams, pts = chk.params(q)
            worst = max(worst, param_rel_err(cams, pts, cy, cx))
            rdiff = max(rdiff, abs(chk.residuals(q, want_rmse=True)["rmse"] - rmse) / rmse)
        out["parity_vs_oracle_1iter"] = {"max_param_rel_err": worst, "tolerance": 1e-3 if fp32 else 1e-9,
                                         "rmse_rel_diff": rdiff, "rmse_tolerance": 5e-3 if fp32 else 1e-9}
        chk.close()
    s.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
