"""The allocation-free lookup entry point (mc_lookup_macro_noalloc) against
mc_lookup_macro: the same kernels with the sort's scratch in the library's
static device array, so the same bits, on two calls in a row (the second with
fewer pairs, so it runs on what the first left in the array) sorted and
unsorted; no device memory requested from the context's allocator during the
calls; sizes above the maximum rejected."""
import ctypes as C
import sys

import numpy as np
import pytest

import mcsynth
from paper_2403_12345_amd import mc
from paper_2403_12345_amd.transport import Transport

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    return torch


class CountingAlloc:
    """An mc_alloc whose callbacks count requests and take the memory from
    PyTorch's caching allocator."""

    def __init__(self, torch):
        self.calls = 0
        self.torch = torch

        def _alloc(user, nbytes, device, stream):
            self.calls += 1
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), int(device), int(stream or 0))
            except Exception:
                return None

        def _release(user, ptr, device, stream):
            torch.cuda.caching_allocator_delete(int(ptr))

        self._a = mc._ALLOC_FN(_alloc)
        self._r = mc._RELEASE_FN(_release)
        self.desc = mc.mc_alloc(self._a, self._r, None)


def _inputs(torch, prob, n, seed):
    rng = np.random.default_rng(seed)
    E = torch.from_numpy(mcsynth.lookup_energies(rng, n)).cuda()
    mat = torch.from_numpy(rng.integers(0, len(prob.materials), n).astype(np.int32)).cuda()
    return E, mat


@pytest.mark.parametrize("sorted_", [True, False])
def test_noalloc_equals_lookup_macro_twice(torch_cuda, sorted_):
    torch = torch_cuda
    print(f"noalloc lookups, 17x17 lattice materials, sorted={sorted_}, n = 1e6 then 300001", flush=True)
    sys.stdout.flush()
    prob = mcsynth.c2_problem()
    counter = CountingAlloc(torch)
    with Transport(prob, allocator=counter.desc) as t:
        for n, seed in ((mc.MC_NOALLOC_MAX_LOOKUPS, 11), (300_001, 12)):
            E, mat = _inputs(torch, prob, n, seed)
            ref_a = torch.empty(n, dtype=torch.float64, device="cuda")
            ref_s = torch.empty_like(ref_a)
            mc.mc_lookup_macro(t.ctx, E, mat, ref_a, ref_s, sorted_)
            got_a = torch.full_like(ref_a, float("nan"))
            got_s = torch.full_like(ref_a, float("nan"))
            torch.cuda.synchronize()
            before = counter.calls
            mc.mc_lookup_macro_noalloc(t.ctx, E, mat, got_a, got_s, sorted_)
            torch.cuda.synchronize()
            assert counter.calls == before, "the no-allocation entry point requested device memory"
            assert torch.equal(got_a, ref_a) and torch.equal(got_s, ref_s), (n, sorted_)


def test_noalloc_rejects_sizes_above_the_maximum(torch_cuda):
    torch = torch_cuda
    prob = mcsynth.c1_problem()
    n = mc.MC_NOALLOC_MAX_LOOKUPS + 1
    with Transport(prob) as t:
        E = torch.full((n,), 1.0e3, dtype=torch.float64, device="cuda")
        mat = torch.zeros(n, dtype=torch.int32, device="cuda")
        out = torch.empty(n, dtype=torch.float64, device="cuda")
        with pytest.raises(mc.MCError) as ei:
            mc.mc_lookup_macro_noalloc(t.ctx, E, mat, out, out.clone(), True)
        assert ei.value.code == mc.MC_EINVAL and "maximum" in str(ei.value)
        # a call at the limit still works afterwards
        k = 1000
        a = torch.empty(k, dtype=torch.float64, device="cuda")
        s = torch.empty_like(a)
        ra, rs = torch.empty_like(a), torch.empty_like(a)
        mc.mc_lookup_macro_noalloc(t.ctx, E[:k], mat[:k], a, s, True)
        mc.mc_lookup_macro(t.ctx, E[:k], mat[:k], ra, rs, True)
        torch.cuda.synchronize()
        assert torch.equal(a, ra) and torch.equal(s, rs)
