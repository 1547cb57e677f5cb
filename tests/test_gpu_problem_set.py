"""GPU tests of the batching layer: 64 uneven independent problems in one
persistent kernel (optionally replayed from a captured hipGraph), and the
autotuners.

A problem's histories depend only on its Philox key and pids, so in the set
they must be the ones a stand-alone run gives (and, for infinite media, the
oracle's); tallies agree to summation order.
"""
import os
import sys
import tempfile

import numpy as np
import pytest

import mcsynth
import oracle
from paper_2403_12345_amd import mc
from paper_2403_12345_amd.transport import ProblemSet, Transport

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    return torch


@pytest.fixture(scope="module")
def c4():
    return mcsynth.c4_problem_set()


def _set_histories(torch, ps, probs, **kw):
    total = sum(p.histories for p in probs)
    log = torch.zeros(total * mc.HISTORY_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    ps.run_batch(history_log=log, **kw)
    torch.cuda.synchronize()
    h = log.cpu().numpy().view(mc.HISTORY_DTYPE)
    offs = np.concatenate([[0], np.cumsum([p.histories for p in probs])])
    return [h[offs[i]:offs[i + 1]] for i in range(len(probs))]


FIELDS = ("fate", "n_coll", "n_cross", "n_draws", "E_final")


def test_problem_set_histories_match_standalone_runs(torch_cuda, c4):
    torch = torch_cuda
    _say(f"problem set: {len(c4)} problems, {sum(p.histories for p in c4)} histories")
    with ProblemSet(c4) as ps:
        hs = _set_histories(torch, ps, c4)
        assert ps.stats()["lost"] == 0
    for i in (0, 1, 2, 3, 10, 31, 62, 63):
        p = c4[i]
        with Transport(p) as t:
            log = torch.zeros(p.histories * mc.HISTORY_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
            t.run_batch(p.seed, 0, p.histories, history_log=log)
            torch.cuda.synchronize()
            g = log.cpu().numpy().view(mc.HISTORY_DTYPE)
        for f in FIELDS:
            assert np.array_equal(hs[i][f], g[f]), (i, f)
        np.testing.assert_allclose(hs[i]["track"], g["track"], rtol=1e-12)


def test_infinite_problems_match_the_oracle(torch_cuda, c4):
    torch = torch_cuda
    with ProblemSet(c4) as ps:
        hs = _set_histories(torch, ps, c4)
    for i in (0, 2, 4):
        p = c4[i]
        o = oracle.run(oracle.OracleProblem(p), p.seed, 0, p.histories, history=True).history
        for f in FIELDS:
            assert np.array_equal(hs[i][f], o[f]), (i, f)


def test_problem_set_tallies_match_standalone(torch_cuda, c4):
    """Three batches: each problem's batch statistics equal its stand-alone
    statistics up to summation order."""
    with ProblemSet(c4) as ps:
        for _ in range(3):
            ps.run_batch()
        for i in (1, 6, 33):
            p = c4[i]
            m, s, meta = ps.tallies(i, mc.MC_T_FLUX_TRACK)
            g, _, _ = ps.tallies(i, mc.MC_T_GLOBAL)
            assert meta.n_batches == 3 and meta.histories == 3 * p.histories
            with Transport(p) as t:
                for b in range(3):
                    t.run_batch(p.seed, b * p.histories, p.histories)
                m2, s2, _ = t.tallies(mc.MC_T_FLUX_TRACK)
                g2, _, _ = t.tallies(mc.MC_T_GLOBAL)
            np.testing.assert_allclose(m, m2, rtol=1e-9, atol=1e-300)
            np.testing.assert_allclose(g, g2, rtol=1e-9, atol=1e-300)


def test_graph_replays_equal_eager_batches(torch_cuda, c4):
    """Batches replayed from the captured graph, with eager work and
    synchronizations in between, give the eager batches' tallies bit for bit."""
    torch = torch_cuda
    sub = c4[:16]
    res = {}
    for use_graph in (False, True):
        with ProblemSet(sub) as ps:
            per_batch = []
            for b in range(3):
                ps.run_batch(use_graph=use_graph)
                # unrelated eager work on the same stream between replays
                x = torch.ones(1 << 20, device="cuda", dtype=torch.float64)
                assert float((x * 2).sum()) == 2.0 * (1 << 20)
                torch.cuda.synchronize()
                per_batch.append([ps.tallies(i, mc.MC_T_FLUX_TRACK)[0].copy() for i in range(len(sub))] +
                                 [ps.tallies(i, mc.MC_T_GLOBAL)[0].copy() for i in range(len(sub))])
            res[use_graph] = per_batch
    for b in range(3):
        for a, g in zip(res[False][b], res[True][b]):
            assert np.array_equal(a, g), b


def test_launch_shapes_do_not_change_histories(torch_cuda, c4):
    torch = torch_cuda
    sub = c4[:12]
    base = None
    for tile, per_cu in ((256, 2), (1024, 1), (2048, 8)):
        with ProblemSet(sub) as ps:
            mc.mc_set_tuning(ps.ctx, set_tile_histories=tile, set_grid=per_cu * 256)
            hs = _set_histories(torch, ps, sub)
        if base is None:
            base = hs
        else:
            for a, b in zip(base, hs):
                for f in FIELDS:
                    assert np.array_equal(a[f], b[f])


def test_autotuners_pick_valid_shapes_and_cache(torch_cuda, c4):
    torch = torch_cuda
    with tempfile.TemporaryDirectory() as d:
        cache = os.path.join(d, "tune.txt")
        with ProblemSet(c4[:16]) as ps:
            best = mc.mc_autotune_problem_set(ps.ctx, cache)
            assert best["set_tile_histories"] in (256, 512, 1024, 2048)
            assert best["set_grid"] in (256, 512, 1024, 2048)
            assert mc.mc_get_problem_tallies(ps.ctx, 0, mc.MC_T_GLOBAL, mc.MC_N_GLOBAL)[2].n_batches == 0
            again = mc.mc_autotune_problem_set(ps.ctx, cache)
            assert again == best
        prob = mcsynth.c1_problem()
        with Transport(prob) as t:
            tb = mc.mc_autotune(t.ctx, 77, 10**9, prob.histories, cache)
            assert tb["lookup_ilp"] in (1, 2, 4)
            assert t.tallies(mc.MC_T_GLOBAL)[2].n_batches == 0
            log = torch.zeros(2000 * mc.HISTORY_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
            t.run_batch(1, 0, 2000, history_log=log)
            torch.cuda.synchronize()
            g = log.cpu().numpy().view(mc.HISTORY_DTYPE)
        o = oracle.run(oracle.OracleProblem(prob), 1, 0, 2000, history=True).history
        for f in FIELDS:
            assert np.array_equal(g[f], o[f])
        lines = open(cache).read().strip().splitlines()
        assert len(lines) == 2
