"""Training pipeline of the learned warm start, driven through the C ABI:
plain FP32 runs on seeded scenes collect (features, converged update) pairs
on the GPU (dba_collect_pairs), then the network is trained on the GPU
(dba_mlp_train).  Returns the FP32 parameter block and normalisation."""
from __future__ import annotations

import time

import numpy as np

from . import binding

# solver of the collection runs: the trajectory workload's loss and rho rule
TRAIN_SOLVER = dict(precision="fp32", loss="huber", loss_param=2.0, rho=1e5, rho_balancing=True,
                    rho_min=1e5, rho_max=1e7)
TRAIN_SEEDS = tuple(range(2000, 2010))
VALIDATION_SEED = 2010


def training_scenes(seeds=TRAIN_SEEDS, n_cams=100, n_points=20000):
    """Trajectory-family scenes (nadir cameras on a random walk, Zipf tracks,
    5 % outliers) of 100 cameras and 20 000 points each."""
    from scenes import make_trajectory_scene
    return [make_trajectory_scene(seed=q, n_cams=n_cams, n_points=n_points) for q in seeds]


def train_default(seed=0, iters=100, per_iter=5000, epochs=10):
    """Collects 10 x iters x per_iter pairs (5M by default) and trains; returns
    params, norm and a report with the collection and training times."""
    t0 = time.perf_counter()
    feats, deltas = collect(training_scenes(), iters=iters, per_iter=per_iter, seed=seed + 1)
    t_collect = time.perf_counter() - t0
    params, norm, rep = train(feats, deltas, epochs=epochs, batch=4096, lr=1e-3, seed=seed)
    rep["collect_seconds"] = t_collect
    return params, norm, rep


def collect(scenes, iters, per_iter, seed=0, conv_steps=30, solver=None):
    feats, deltas = [], []
    for q, sc in enumerate(scenes):
        s = binding.Solver(**(solver or TRAIN_SOLVER)).set_scene(sc)
        f, d = binding.dba_collect_pairs(s.h, iters, per_iter, seed=seed + q, conv_steps=conv_steps)
        s.close()
        feats.append(f)
        deltas.append(d)
    return np.concatenate(feats), np.concatenate(deltas)


def train(feats, deltas, epochs=10, batch=4096, lr=1e-3, seed=0):
    h = binding.dba_create(binding.make_options(precision="fp32"))
    try:
        t0 = time.perf_counter()
        losses = binding.dba_mlp_train(h, feats, deltas, epochs=epochs, batch=batch, lr=lr, seed=seed)
        t_train = time.perf_counter() - t0
        params, norm = binding.dba_get_mlp(h)
    finally:
        binding.dba_destroy(h)
    return params, norm, dict(epoch_loss=losses.tolist(), train_seconds=t_train, pairs=int(feats.shape[0]))


def validation_error(params, norm, feats, deltas):
    """Mean squared error of the network's standardized prediction on
    held-out pairs, and that of predicting zero (the plain start)."""
    h = binding.dba_create(binding.make_options(precision="fp32"))
    try:
        binding.dba_set_mlp(h, params, norm)
        pred = binding.dba_mlp_forward(h, feats)
    finally:
        binding.dba_destroy(h)
    sd, mu = norm[64:76], norm[52:64]
    e_net = np.mean(((pred - deltas) / sd) ** 2)
    e_zero = np.mean(((0.0 - deltas) / sd) ** 2)
    return float(e_net), float(e_zero)
