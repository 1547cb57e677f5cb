"""The C ABI's context and tally contract on the GPU.

* Device memory from a caller's allocator (PyTorch's caching allocator through
  the binding) gives the same results as hipMalloc, and is handed back on
  destroy.
* Checkpoint and resume between batches: raw batch sums read from one
  context and restored into a fresh one, then more batches, give the same
  tallies bit for bit as one uninterrupted run (section 2, "Tallying": the
  active batches' sums are the whole state of the estimate).
* The fixed-point mesh tally refuses a batch whose weighted track total could
  wrap a bin (MC_ERANGE) and accepts one just below the bound.
* The bootstrap slope of the learned-importance sequence comes from the
  library: -ln(max(R0, 1/N)).
"""
import math

import numpy as np
import pytest

import mcsynth
from paper_2403_12345_amd import mc
from paper_2403_12345_amd.transport import Transport
from tests.test_oracle_mesh import mesh_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    return torch


def _all(t):
    return [t.tallies(k)[:2] for k in (mc.MC_T_FLUX_TRACK, mc.MC_T_FLUX_COLLISION, mc.MC_T_GLOBAL)]


def test_caller_allocator_matches_hipmalloc(torch_cuda):
    torch = torch_cuda
    print("allocator: torch caching allocator against hipMalloc", flush=True)
    prob = mcsynth.c1_problem()
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated(0)
    out = []
    for alloc in ("torch", None):
        with Transport(prob, allocator=alloc) as t:
            t.run_batch(1, 0, 5000)
            t.run_batch(1, 5000, 5000)
            if alloc == "torch":
                assert torch.cuda.memory_allocated(0) > base + (1 << 20)
            out.append(_all(t))
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated(0) == base
    for (m1, s1), (m2, s2) in zip(out[0], out[1]):
        assert np.array_equal(m1, m2) and np.array_equal(s1, s2)


@pytest.mark.parametrize("case", ["c1", "mesh"])
def test_resume_between_batches_is_bitwise(torch_cuda, case):
    print(f"resume: {case}", flush=True)
    prob = mcsynth.c1_problem() if case == "c1" else mesh_problem()
    per = 4000
    with Transport(prob) as t:
        for b in range(6):
            t.run_batch(9, b * per, per)
        whole = _all(t)
        whole_meta = t.tallies(mc.MC_T_GLOBAL)[2]
    with Transport(prob) as t:
        for b in range(3):
            t.run_batch(9, b * per, per)
        state = t.checkpoint()
    assert state["n_batches"] == 3 and state["histories"] == 3 * per
    with Transport(prob) as t:
        t.restore(state)
        for b in range(3, 6):
            t.run_batch(9, b * per, per)
        resumed = _all(t)
        meta = t.tallies(mc.MC_T_GLOBAL)[2]
    assert meta.n_batches == whole_meta.n_batches == 6 and meta.histories == 6 * per
    for (m1, s1), (m2, s2) in zip(whole, resumed):
        assert np.array_equal(m1, m2) and np.array_equal(s1, s2)


def test_set_tallies_rejects_bad_state(torch_cuda):
    with Transport(mcsynth.c1_problem()) as t:
        with pytest.raises(mc.MCError, match="MC_EINVAL"):
            mc.mc_set_tallies(t.ctx, mc.MC_T_GLOBAL, np.zeros(3), np.zeros(3), 1, 10)
        with pytest.raises(mc.MCError, match="MC_EINVAL"):
            mc.mc_set_tallies(t.ctx, mc.MC_T_GLOBAL, np.full(12, np.nan), np.zeros(12), 1, 10)
        with pytest.raises(mc.MCError, match="MC_EINVAL"):
            mc.mc_set_tallies(t.ctx, mc.MC_T_GLOBAL, np.zeros(12), np.zeros(12), 5, 2)
        with pytest.raises(mc.MCError, match="MC_ESTATE"):
            mc.mc_set_tallies(t.ctx, mc.MC_T_REACTION, np.zeros(1), np.zeros(1), 1, 10)


def _absorber_mesh(sigma_a):
    """Infinite pure absorber (one flight per history, mean length 1/Sigma_a)
    with a mesh tally around the point source."""
    nuc = mcsynth.constant_nuclide(sigma_a / 0.01, 0.0, 56.0)
    mat = mcsynth.Material(nuclides=np.array([0], np.int32), densities=np.array([0.01]))
    return mcsynth.Problem(name="absorber_mesh", nuclides=[nuc], materials=[mat],
                           geometry=mcsynth.Geometry(kind=mcsynth.GEOM_INFINITE, material=0),
                           source=mcsynth.Source(kind=mcsynth.SRC_POINT),
                           tally=mcsynth.Tally(mcsynth.TALLY_MESH, mesh_dims=(4, 4, 4),
                                               mesh_box=(-500.0, 500.0, -500.0, 500.0, -500.0, 500.0)),
                           histories=1, batches=1, seed=3)


def test_mesh_range_guard(torch_cuda):
    """With Sigma_a = 1e-3 /cm a history's track is 1000 cm on average: 2.5e6
    histories put a batch's weighted track near 2.5e9 > 2^31 (MC_ERANGE);
    1.5e6 histories (1.5e9) pass."""
    print("mesh range guard", flush=True)
    with Transport(_absorber_mesh(1e-3)) as t:
        t.run_batch(5, 0, 1_500_000)
        g, _, _ = t.tallies(mc.MC_T_GLOBAL)
        assert 1.4e9 < g[mc.MC_G_TRACK] * 1.5e6 < 1.6e9
        with pytest.raises(mc.MCError, match="MC_ERANGE"):
            t.run_batch(5, 1_500_000, 2_500_000)


def test_bootstrap_slope_from_the_library(torch_cuda):
    prob = mcsynth.slab_problem(sigma_t=(0.5, 0.5, 0.5), thickness=(4.0, 4.0, 4.0))
    with Transport(prob) as t:
        with pytest.raises(mc.MCError, match="MC_ESTATE"):
            mc.mc_ww_bootstrap_slope(t.ctx)
        t.run_batch(7, 0, 20_000)
        r0 = t.tallies(mc.MC_T_GLOBAL)[0][mc.MC_G_LEAK_XHI]
        a = mc.mc_ww_bootstrap_slope(t.ctx)
    assert r0 > 0 and a == -math.log(max(r0, 1.0 / 20_000))
    assert abs(r0 - math.exp(-6.0)) < 5 * math.sqrt(math.exp(-6.0) / 20_000)
