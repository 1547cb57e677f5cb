"""Learned importance map for weight windows: generation, training and use.

This module sequences library calls; every step runs in the library's
kernels (transport, forward importance sums, sample building, BF16
matrix-core training, windows from the network).  The sequence:

1. Pilot (analog): a short analog run estimates the detector response R0 (the
   weight leaking through the far face); the bootstrap map is linear in depth,
   ln I = a x / L with a = -ln(max(R0, 1 / pilot histories)) -- the importance
   of the far face relative to the source, or a floor from the pilot size
   when no pilot history scored.
2. Bootstrap: a run with those windows and the forward importance estimate on
   an x by ln E grid.
3. Training: samples (cell centre, ln(num / den)) weighted by their inverse
   relative variance, full-batch Adam on the network.
4. Optionally refine: rerun with windows from the network, rebuild the sums,
   train again from the current parameters.

The production windows then come from the network, its ln I clamped to the
span of the training targets (outside the cells it was fitted on the network
extrapolates, and an unbounded map could split without limit); analog
transport remains the unbiased reference for its estimate.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import mc


@dataclass
class LearnedImportance:
    params: np.ndarray            # [MC_MLP_NPAR] float32
    slope: float                  # bootstrap ln I slope a (ln I = a x / L)
    ln_range: tuple               # smallest and largest training target (the windows' clamp)
    pilot_response: float         # analog pilot detector estimate
    loss_curves: list             # per training round, loss before each step
    n_samples: list               # per training round
    seconds: dict = field(default_factory=dict)  # wall time of pilot, bootstrap, training


def slab_extent(prob):
    e = prob.geometry.x_edges
    return float(e[0]), float(e[-1])


def learn(t, seed: int, pilot: int = 1_000_000, boot: int = 1_000_000, nx: int = 100, ne: int = 32,
          refine: int = 0, steps: int = 2000, lr: float = 1e-2, replicas: int = 4, min_credits: float = 10.0,
          rel_floor: float = 0.1, first_pid: int = 0, kappa: float = 3.0, ratio: float = 5.0) -> LearnedImportance:
    """Run the generation / training sequence on the Transport ``t`` (a slab
    problem); leaves the context analog with the trained network loaded."""
    x0, x1 = slab_extent(t.prob)
    L = x1 - x0
    ctx = t.ctx
    sec = {}
    # 1. analog pilot
    tic = time.perf_counter()
    mc.mc_set_weight_windows(ctx)
    t.reset()
    t.run_batch(seed, first_pid, pilot)
    r0 = float(t.tallies(mc.MC_T_GLOBAL)[0][mc.MC_G_LEAK_XHI])
    slope = mc.mc_ww_bootstrap_slope(ctx)
    sec["pilot"] = time.perf_counter() - tic
    # 2. bootstrap windows with the importance grid
    tic = time.perf_counter()
    grid = dict(imp_nx=nx, imp_ne=ne, imp_x0=x0, imp_x1=x1)
    mc.mc_set_weight_windows(ctx, kind=mc.MC_WW_LINEAR, lin=(0.0, slope, 0.0), length=L, kappa=kappa,
                             ratio=ratio, **grid)
    t.reset()
    t.run_batch(seed, first_pid + pilot, boot)
    sec["bootstrap"] = time.perf_counter() - tic
    # 3. training
    tic = time.perf_counter()
    opts = mc.train_opts(steps=steps, replicas=replicas, lr=lr, min_credits=min_credits, rel_floor=rel_floor,
                         length=L, seed=seed)
    mc.mc_mlp_init(ctx, seed)
    curves, counts = [], []
    curve, n, span = mc.mc_importance_train(ctx, opts)
    curves.append(curve)
    counts.append(n)
    sec["train"] = time.perf_counter() - tic
    # 4. refinement rounds
    for k in range(refine):
        tic = time.perf_counter()
        mc.mc_set_weight_windows(ctx, kind=mc.MC_WW_MLP, length=L, kappa=kappa, ratio=ratio, ln_lo=span[0],
                                 ln_hi=span[1], **grid)
        t.reset()
        t.run_batch(seed, first_pid + pilot + (k + 1) * boot, boot)
        curve, n, span = mc.mc_importance_train(ctx, opts)
        curves.append(curve)
        counts.append(n)
        sec[f"refine{k + 1}"] = time.perf_counter() - tic
    params = mc.mc_mlp_get(ctx)
    mc.mc_set_weight_windows(ctx)
    t.reset()
    return LearnedImportance(params=params, slope=slope, ln_range=span, pilot_response=r0, loss_curves=curves,
                             n_samples=counts, seconds=sec)


@dataclass
class Production:
    mean: float          # detector estimate per source particle
    stderr: float
    rel: float           # stderr / mean
    seconds: float       # wall time of the batches
    gpu_ms: float        # summed batch time on the GPU
    fom: float           # 1 / (rel^2 seconds)
    histories: int
    splits: float        # split copies per source particle
    roulette: float


def production(t, seed: int, histories: int, batches: int, windows: str = "analog", lin=None,
               first_pid: int = 0, kappa: float = 3.0, ratio: float = 5.0, ln_range=(0.0, 0.0)) -> Production:
    """Detector estimate of ``histories`` in ``batches`` batches with analog
    transport ("analog"), linear windows ("linear", ln I = lin) or windows
    from the context's network ("mlp"), ln I clamped to ln_range; figure of
    merit 1 / (R^2 T)."""
    x0, x1 = slab_extent(t.prob)
    L = x1 - x0
    if windows == "analog":
        mc.mc_set_weight_windows(t.ctx)
    elif windows == "linear":
        mc.mc_set_weight_windows(t.ctx, kind=mc.MC_WW_LINEAR, lin=lin, length=L, kappa=kappa, ratio=ratio,
                                 ln_lo=ln_range[0], ln_hi=ln_range[1])
    elif windows == "mlp":
        mc.mc_set_weight_windows(t.ctx, kind=mc.MC_WW_MLP, length=L, kappa=kappa, ratio=ratio, ln_lo=ln_range[0],
                                 ln_hi=ln_range[1])
    else:
        raise ValueError(windows)
    t.reset()
    per = histories // batches
    gpu_ms = 0.0
    tic = time.perf_counter()
    for b in range(batches):
        t.run_batch(seed, first_pid + b * per, per)
        gpu_ms += t.stats()["batch_ms"]
    sec = time.perf_counter() - tic
    g, s, _ = t.tallies(mc.MC_T_GLOBAL)
    mean, se = float(g[mc.MC_G_LEAK_XHI]), float(s[mc.MC_G_LEAK_XHI])
    rel = se / mean if mean > 0 else math.inf
    fom = 1.0 / (rel * rel * sec) if mean > 0 and se > 0 else 0.0
    mc.mc_set_weight_windows(t.ctx)
    return Production(mean=mean, stderr=se, rel=rel, seconds=sec, gpu_ms=gpu_ms, fom=fom, histories=per * batches,
                      splits=float(g[mc.MC_G_SPLIT]), roulette=float(g[mc.MC_G_ROULETTE]))
