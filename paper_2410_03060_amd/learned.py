"""Training and use of the learned parts (host orchestration only): the initial
guess and the learned neighbourhood-inverse preconditioner.

Every step runs in libchaff: the training currents come from the library's
own solver, the features and targets from its feature and target kernels,
and each optimisation step is one chaff_mlp_train_step (BF16 forward and
backward on matrix cores, FP32 Adam).  This module only decides which clouds
to solve, in which order to visit the rows (a seeded permutation drawn on
the host), and the learning-rate schedule.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import binding as B
from . import workloads as W


@dataclass
class SampleSet:
    feat: torch.Tensor            # [rows, 192] int16 (BF16 bit patterns)
    target: torch.Tensor          # [rows, 14] float32
    clouds: int = 0
    solve_seconds: float = 0.0
    iterations: list = field(default_factory=list)


def solve_opts_for_training(tol: float = 1e-6):
    return B.solve_opts(tol=tol, inner_tol=1e-5, restart=5000, max_cycles=60, prec=B.C64, method=B.COCG)


def solved_samples(workloads, opts=None, device="cuda") -> SampleSet:
    """Solve every workload with the library and collect (features, targets)."""
    opts = opts or solve_opts_for_training()
    feats, targs, iters = [], [], []
    t0 = time.perf_counter()
    for wl in workloads:
        cl = B.build_cloud(wl.cloud, device)
        Z, Pinv = B.fill_Z(cl, B.C64)
        X, info = B.solve(cl, Z, Pinv, wl.inc.k_hat, wl.inc.e_hat, opts)
        feats.append(B.mlp_features(cl, wl.inc.k_hat, wl.inc.e_hat))
        targs.append(B.mlp_targets(cl, Pinv, wl.inc.k_hat, wl.inc.e_hat, X))
        iters.append(info["iterations"])
        del Z, Pinv, X
        B.destroy(cl)
    torch.cuda.synchronize()
    return SampleSet(torch.cat(feats), torch.cat(targs), len(workloads), time.perf_counter() - t0, iters)


def nbhd_samples(workloads, size: int, device="cuda") -> SampleSet:
    """Samples of the learned neighbourhood inverse: for every workload the library
    computes the raw neighbourhood rows (chaff_nbhd_raw_rows), their features and
    targets; rows of empty slots are left out."""
    feats, targs = [], []
    t0 = time.perf_counter()
    for wl in workloads:
        cl = B.build_cloud(wl.cloud, device)
        Z, P = B.fill_Z(cl, B.C64)
        Mr = B.nbhd_raw_rows(cl, Z, size)
        valid = (B.nbhd_table(cl, Mr, size) >= 0)[:, :, None].expand(cl.n, size, 7).reshape(-1)
        feats.append(B.nbhd_mlp_features(cl, Mr, size)[valid])
        targs.append(B.nbhd_mlp_targets(cl, Mr, P, size)[valid])
        del Z, P, Mr
        B.destroy(cl)
    torch.cuda.synchronize()
    return SampleSet(torch.cat(feats), torch.cat(targs), len(workloads), time.perf_counter() - t0, [])


@dataclass
class TrainResult:
    theta: torch.Tensor
    losses: list
    steps: int
    seconds: float


def train(samples: SampleSet, theta0: np.ndarray, epochs: int = 4, batch: int = 4096, lr: float = 2e-3,
          lr_min: float = 2e-5, seed: int = 0, device="cuda", log_every: int = 0) -> TrainResult:
    """Adam with a cosine learning-rate decay over seeded row permutations."""
    n = samples.feat.shape[0]
    tr = B.MlpTrainer(theta0, batch, device)
    steps_per_epoch = (n + batch - 1) // batch
    total = epochs * steps_per_epoch
    losses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step = 0
    for ep in range(epochs):
        order = torch.as_tensor(W.shuffle_order(seed + ep, n), device=device)
        ep_loss = torch.zeros(1, dtype=torch.float64, device=device)
        for b0 in range(0, n, batch):
            idx = order[b0:b0 + batch]
            rate = lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * step / max(total - 1, 1)))
            loss = tr.step(samples.feat, samples.target, idx, rate)
            ep_loss += loss.double() * idx.shape[0]
            step += 1
            if log_every and step % log_every == 0:
                print(f"[mlp] step {step}/{total} loss {loss.item():.4e}", flush=True)
        losses.append(float(ep_loss.item() / n))
    torch.cuda.synchronize()
    return TrainResult(tr.theta, losses, step, time.perf_counter() - t0)


def relative_target_error(theta, samples: SampleSet) -> float:
    """||y - t||_2 / ||t||_2 over a sample set (the loss as a relative L2 error)."""
    num = 0.0
    den = 0.0
    for r0 in range(0, samples.feat.shape[0], 1 << 20):
        f = samples.feat[r0:r0 + (1 << 20)]
        t = samples.target[r0:r0 + (1 << 20)]
        y = B.mlp_forward(theta, f)
        num += float(((y - t).double() ** 2).sum())
        den += float((t.double() ** 2).sum())
    return math.sqrt(num / den)
