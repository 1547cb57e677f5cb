"""Transport at the benchmark's sizes and launch shapes, checked on histories
the oracle can afford one by one and on properties that hold at any size.

* 17x17 lattice: one batch of 1e6 histories through the batched entry point
  (mc_run_batches) with the autotuner's shapes from the committed cache
  (several event loops running consecutive batches, the one-launch tail).
* 300-nuclide 255x255 lattice: one batch of 2e7 histories with its tuned
  shapes (millions in flight, sorted lookup queues), mesh flux tally.
* Sampled pids at the start, middle and end of each batch against the
  oracle's histories of the same pids: fate, draws and final energy equal for
  at least 90 % (with geometry the device and host logarithms may differ in
  the last ulp, which can move a crossing).
* Every history ends (fate set); the history log sums to the global tallies
  (path length to rounding, collisions exactly); absorption plus cutoff is
  one per source particle (reflective boundaries, no leakage); the mesh
  path-length tally sums to the total path length.
"""
import os
import shutil
import sys

import numpy as np
import pytest

import mcsynth
import oracle
from paper_2403_12345_amd import mc
from paper_2403_12345_amd.transport import Transport

pytestmark = pytest.mark.gpu

CACHE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2403_12345_amd",
                     "tuning_cache.txt")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    return torch


def _tuned(t, prob, n, tmp_path):
    # a copy: a cache miss tunes into the copy, never into the committed file
    cache = tmp_path / "tuning_cache.txt"
    shutil.copy(CACHE, cache)
    return mc.mc_autotune(t.ctx, prob.seed, 1 << 40, n, str(cache))


def _check_samples(prob, g, seed, n, k=300):
    op = oracle.OracleProblem(prob)
    same = []
    for first in (0, n // 2 - k // 2, n - k):
        o = oracle.run(op, seed, first, k, history=True).history
        h = g[first:first + k]
        same.append((h["n_draws"] == o["n_draws"]) & (h["E_final"] == o["E_final"]) & (h["fate"] == o["fate"]))
    frac = float(np.concatenate(same).mean())
    _say(f"identical sampled histories: {frac:.4f}")
    assert frac > 0.9


def _check_log_sums(g, glob, n):
    assert np.all(g["fate"] > 0)
    assert glob[mc.MC_G_NCOLL] * n == pytest.approx(float(g["n_coll"].astype(np.int64).sum()), rel=1e-12)
    assert glob[mc.MC_G_TRACK] * n == pytest.approx(float(g["track"].sum()), rel=1e-9)
    assert glob[mc.MC_G_LEAK] == 0.0
    assert glob[mc.MC_G_ABSORB] + glob[mc.MC_G_CUTOFF] == pytest.approx(1.0, abs=1e-12)


@pytest.mark.timeout(600)
def test_lattice_benchmark_batch(torch_cuda, tmp_path):
    torch = torch_cuda
    prob = mcsynth.c2_problem()
    n, seed = prob.histories, prob.seed
    with Transport(prob) as t:
        tuning = _tuned(t, prob, n, tmp_path)
        _say(f"17x17 lattice, 1e6 histories, tuning {tuning}")
        log = torch.zeros(n * mc.HISTORY_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
        t.run_batches(seed, 0, n, 1, history_log=log)
        torch.cuda.synchronize()
        g = log.cpu().numpy().view(mc.HISTORY_DTYPE)
        glob, _, meta = t.tallies(mc.MC_T_GLOBAL)
        pins, _, _ = t.tallies(mc.MC_T_FLUX_TRACK)
    assert meta.histories == n
    _check_log_sums(g, glob, n)
    # the pins' cylinders hold part of the path, the moderator the rest
    assert 0.0 < pins.sum() < glob[mc.MC_G_TRACK]
    _check_samples(prob, g, seed, n)


@pytest.mark.timeout(600)
def test_300_nuclide_lattice_benchmark_batch(torch_cuda, tmp_path):
    torch = torch_cuda
    prob = mcsynth.c3_problem()
    n, seed = prob.histories, prob.seed
    with Transport(prob) as t:
        tuning = _tuned(t, prob, n, tmp_path)
        _say(f"300-nuclide lattice, 2e7 histories, tuning {tuning}")
        log = torch.zeros(n * mc.HISTORY_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
        t.run_batch(seed, 0, n, history_log=log)
        torch.cuda.synchronize()
        g = log.cpu().numpy().view(mc.HISTORY_DTYPE)
        del log
        glob, _, meta = t.tallies(mc.MC_T_GLOBAL)
        mesh, _, _ = t.tallies(mc.MC_T_FLUX_TRACK)
        st = t.stats()
    assert meta.histories == n
    assert st["sorted_lookups"] > 0
    _check_log_sums(g, glob, n)
    assert mesh.sum() == pytest.approx(glob[mc.MC_G_TRACK], rel=1e-9)
    _check_samples(prob, g, seed, n, k=100)
