"""GPU parity of the lookup and sort steps against the oracle (through the C ABI).

Bar: grid indices bit-exact; interpolated and macroscopic fp64 cross sections
within 1e-12 relative (both sides sum in material order with contraction
off, so they are expected to agree bit for bit, which is checked too).
"""
import sys

import numpy as np
import pytest

import mcsynth
import oracle
from paper_2403_12345_amd import mc
from paper_2403_12345_amd.transport import Transport

pytestmark = pytest.mark.gpu

REL = 1e-12


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    return torch


@pytest.fixture(scope="module")
def c2(torch_cuda):
    prob = mcsynth.c2_problem()
    t = Transport(prob)
    yield prob, t, oracle.OracleProblem(prob)
    t.close()


def _edge_energies(prob, mat, rng, n_random):
    """Grid points of the material's nuclides and their ulp neighbours, the hash
    bin edges and their ulp neighbours, both ends, and random energies."""
    pts = [mcsynth.lookup_energies(rng, n_random), [mcsynth.EMIN, mcsynth.EMAX]]
    for k in prob.materials[mat].nuclides[:4]:
        E = prob.nuclides[k].E
        sel = E[rng.integers(0, E.size, 3000)]
        pts += [sel, np.nextafter(sel, 0), np.nextafter(sel, np.inf)]
    M = prob.n_hash_bins
    edges = mcsynth.EMIN * np.exp(np.arange(M + 1) * (np.log(mcsynth.EMAX / mcsynth.EMIN) / M))
    sel = edges[rng.integers(0, M + 1, 4000)]
    pts += [sel, np.nextafter(sel, 0), np.nextafter(sel, np.inf)]
    e = np.concatenate(pts)
    return e[(e >= mcsynth.EMIN) & (e <= mcsynth.EMAX)]


@pytest.mark.parametrize("mat", [0, 1, 2])
def test_nuclide_indices_bit_exact_and_xs(c2, torch_cuda, mat):
    torch = torch_cuda
    prob, t, op = c2
    rng = np.random.default_rng(100 + mat)
    e = _edge_energies(prob, mat, rng, 20000)
    nk = prob.materials[mat].nuclides.size
    _say(f"nuclide lookup mat={mat} n={e.size} nk={nk}")
    E = torch.from_numpy(e).cuda()
    idx = torch.empty(e.size * nk, dtype=torch.int32, device="cuda")
    sc = torch.empty(e.size * nk, dtype=torch.float64, device="cuda")
    ss = torch.empty(e.size * nk, dtype=torch.float64, device="cuda")
    mc.mc_lookup_nuclides(t.ctx, mat, E, idx, sc, ss)
    torch.cuda.synchronize()
    idx = idx.cpu().numpy().reshape(e.size, nk)
    sc = sc.cpu().numpy().reshape(e.size, nk)
    ss = ss.cpu().numpy().reshape(e.size, nk)
    for q, k in enumerate(prob.materials[mat].nuclides):
        ri, rc, rs = oracle.micro_xs(op, int(k), e)
        assert np.array_equal(idx[:, q], ri), f"nuclide {k}: index mismatch"
        for got, ref in ((sc[:, q], rc), (ss[:, q], rs)):
            rel = np.abs(got - ref) / np.maximum(np.abs(ref), 1e-300)
            assert rel.max() <= REL
            assert np.array_equal(got, ref)


@pytest.mark.parametrize("sorted_,ilp", [(False, 4), (True, 4), (False, 1), (True, 2)])
def test_macro_lookup_matches_oracle(c2, torch_cuda, sorted_, ilp):
    """Every launch shape of the lookup kernel gives the oracle's values."""
    torch = torch_cuda
    prob, t, op = c2
    mc.mc_set_tuning(t.ctx, lookup_ilp=ilp)
    rng = np.random.default_rng(7)
    n = 200_003  # several tiles and a ragged tail
    e = mcsynth.lookup_energies(rng, n)
    m = rng.integers(0, 3, n).astype(np.int32)
    _say(f"macro lookup sorted={sorted_} n={n}")
    E = torch.from_numpy(e).cuda()
    Mt = torch.from_numpy(m).cuda()
    Sa = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
    Ss = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
    mc.mc_lookup_macro(t.ctx, E, Mt, Sa, Ss, sorted_)
    torch.cuda.synchronize()
    mc.mc_set_tuning(t.ctx)
    ra, rs = oracle.macro_xs(op, m, e)
    for got, ref in ((Sa.cpu().numpy(), ra), (Ss.cpu().numpy(), rs)):
        rel = np.abs(got - ref) / np.maximum(np.abs(ref), 1e-300)
        assert rel.max() <= REL
        assert np.array_equal(got, ref)


@pytest.mark.parametrize("n", [1, 4095, 4097, 100_000, 300_001])
def test_sort_queue_is_a_sorted_permutation(c2, torch_cuda, n):
    torch = torch_cuda
    prob, t, op = c2
    rng = np.random.default_rng(8)
    e = mcsynth.lookup_energies(rng, n)
    m = rng.integers(0, 3, n).astype(np.int32)
    _say(f"sort n={n}")
    if n > 1000:
        e[: n // 3] = 0.0253  # a third of the queue in one key: many equal keys
    perm = torch.empty(n, dtype=torch.int32, device="cuda")
    keys = torch.empty(n, dtype=torch.int32, device="cuda")
    mc.mc_sort_queue(t.ctx, torch.from_numpy(e).cuda(), torch.from_numpy(m).cuda(), perm, keys)
    torch.cuda.synchronize()
    perm = perm.cpu().numpy().view(np.uint32).astype(np.int64)
    keys = keys.cpu().numpy().view(np.uint32).astype(np.int64)
    assert np.array_equal(np.sort(perm), np.arange(n))
    assert np.all(np.diff(keys) >= 0)
    # stable: equal keys keep their input order
    same_key = np.diff(keys) == 0
    assert np.all(np.diff(perm)[same_key] > 0)
    M = prob.n_hash_bins
    assert np.array_equal(keys // M, m[perm])
    # the bin part is the hash bin of E up to the last-ulp rounding of ln E at an edge
    b_host = np.clip(np.floor((np.log(e) - np.log(mcsynth.EMIN)) * (M / np.log(mcsynth.EMAX / mcsynth.EMIN))),
                     0, M - 1).astype(np.int64)
    assert np.all(np.abs(keys % M - b_host[perm]) <= 1)
    # energies within one material are ordered up to the bin width
    same = (keys[1:] // M) == (keys[:-1] // M)
    ep = e[perm]
    assert np.all(ep[1:][same & ((keys[1:] % M) > (keys[:-1] % M) + 1)] >
                  ep[:-1][same & ((keys[1:] % M) > (keys[:-1] % M) + 1)])


def test_lookup_edge_cases(c2, torch_cuda):
    """n = 1, n = 255/257 (around one workgroup), energies at both grid ends."""
    torch = torch_cuda
    prob, t, op = c2
    for n in (1, 255, 257):
        e = np.full(n, mcsynth.EMAX) if n == 1 else np.linspace(mcsynth.EMIN, mcsynth.EMAX, n)
        m = (np.arange(n) % 3).astype(np.int32)
        Sa = torch.empty(n, dtype=torch.float64, device="cuda")
        Ss = torch.empty(n, dtype=torch.float64, device="cuda")
        mc.mc_lookup_macro(t.ctx, torch.from_numpy(e).cuda(), torch.from_numpy(m).cuda(), Sa, Ss, True)
        torch.cuda.synchronize()
        ra, rs = oracle.macro_xs(op, m, e)
        assert np.array_equal(Sa.cpu().numpy(), ra) and np.array_equal(Ss.cpu().numpy(), rs)


def test_c3_scale_lookup_sampled(torch_cuda):
    """The 300-nuclide material at full size (grids of 20k-150k points): one
    million sorted lookups, a sample of 3000 checked against the oracle."""
    torch = torch_cuda
    prob = mcsynth.c3_problem()
    _say(f"c3 lookup data {prob.data_bytes() / 1e6:.0f} MB")
    t = Transport(prob)
    try:
        op = oracle.OracleProblem(prob)
        rng = np.random.default_rng(9)
        n = 1_000_000
        e = mcsynth.lookup_energies(rng, n)
        m = np.zeros(n, np.int32)
        Sa = torch.empty(n, dtype=torch.float64, device="cuda")
        Ss = torch.empty(n, dtype=torch.float64, device="cuda")
        mc.mc_lookup_macro(t.ctx, torch.from_numpy(e).cuda(), torch.from_numpy(m).cuda(), Sa, Ss, True)
        torch.cuda.synchronize()
        sel = rng.integers(0, n, 3000)
        ra, rs = oracle.macro_xs(op, m[sel], e[sel])
        ga, gs = Sa.cpu().numpy()[sel], Ss.cpu().numpy()[sel]
        assert np.max(np.abs(ga - ra) / ra) <= REL and np.max(np.abs(gs - rs) / rs) <= REL
        # sorted queues read shared grid windows; unsorted ones search per lane:
        # the same values bit for bit, all 1e6 of them
        Sa2 = torch.empty(n, dtype=torch.float64, device="cuda")
        Ss2 = torch.empty(n, dtype=torch.float64, device="cuda")
        mc.mc_lookup_macro(t.ctx, torch.from_numpy(e).cuda(), torch.from_numpy(m).cuda(), Sa2, Ss2, False)
        torch.cuda.synchronize()
        assert torch.equal(Sa, Sa2) and torch.equal(Ss, Ss2)
    finally:
        t.close()


def test_sorted_lookups_at_grid_points_and_bin_edges(c2, torch_cuda):
    """Sorted queues dense in energy (every lane of a wave in one or two hash
    bins): the fuel's grid points, their neighbours one ulp away and the hash
    bin edges one ulp either side, each energy many times over, in all three
    materials; equal to the oracle bit for bit."""
    torch = torch_cuda
    prob, t, op = c2
    fuel = prob.materials[0].nuclides[:3]
    pts = np.concatenate([prob.nuclides[k].E for k in fuel])
    pts = pts[(pts > mcsynth.EMIN) & (pts < mcsynth.EMAX)][::7]
    edges = mcsynth.EMIN * np.exp(np.arange(1, 8192) * np.log(mcsynth.EMAX / mcsynth.EMIN) / 8192)
    base = np.concatenate([pts, np.nextafter(pts, 0), np.nextafter(pts, np.inf),
                           np.nextafter(edges, 0), edges, np.nextafter(edges, np.inf)])
    e = np.repeat(base, 3)
    m = (np.arange(e.size) % 3).astype(np.int32)
    _say(f"sorted edge lookups n={e.size}")
    Sa = torch.empty(e.size, dtype=torch.float64, device="cuda")
    Ss = torch.empty(e.size, dtype=torch.float64, device="cuda")
    mc.mc_lookup_macro(t.ctx, torch.from_numpy(e).cuda(), torch.from_numpy(m).cuda(), Sa, Ss, True)
    torch.cuda.synchronize()
    ra, rs = oracle.macro_xs(op, m, e)
    assert np.array_equal(Sa.cpu().numpy(), ra) and np.array_equal(Ss.cpu().numpy(), rs)
