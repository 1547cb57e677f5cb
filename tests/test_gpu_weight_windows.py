"""GPU parity of weight windows and of the forward importance estimate against
the oracle (through the C ABI).

* Linear windows: every split copy depends on (seed, pid) and its line only,
  whichever slot runs it, so in an infinite medium and in a pure-absorber slab
  the GPU histories (collisions, crossings, draws and path length summed over
  all copies; fate, final energy and weight of the source particle's own
  copy) are those of the oracle, and the split / roulette counts and
  importance sums agree to summation order.
* Windows never bias: transmission through a pure absorber stays exp(-tau)
  with smaller errors; windowed and analog runs agree within 3 sigma.
* Network windows: FP32 ln I against the oracle's FP64 moves window edges by
  ~1e-6 relative, so nearly all (not all) same-seed histories are identical
  and the tallies agree within 3 sigma.
"""
import math
import sys

import numpy as np
import pytest

import mcsynth
import oracle
from oracle import mlp
from paper_2403_12345_amd import mc
from paper_2403_12345_amd.transport import Transport
from tests.stats import three_sigma

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    return torch


def _gpu_histories(torch, t, seed, first, n, **opts):
    log = torch.zeros(n * mc.HISTORY_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    t.run_batch(seed, first, n, history_log=log, **opts)
    torch.cuda.synchronize()
    return log.cpu().numpy().view(mc.HISTORY_DTYPE)


def _same(g, o):
    """Per history: identical fate, counts, draws and final energy; weights
    equal to the last ulps (window edges come from exp, whose last bit may
    differ between the device and the host library)."""
    return ((g["fate"] == o["fate"]) & (g["n_coll"] == o["n_coll"]) & (g["n_cross"] == o["n_cross"])
            & (g["n_draws"] == o["n_draws"]) & (g["E_final"] == o["E_final"])
            & np.isclose(g["weight"], o["weight"], rtol=1e-12, atol=0))


def _compare_histories(g, o):
    same = _same(g, o)
    assert np.all(same), (np.flatnonzero(~same)[:10], g[~same][:3], o[~same][:3])
    np.testing.assert_allclose(g["track"], o["track"], rtol=1e-12)


def _infinite_ww(depth=24, n_max=10):
    prob = mcsynth.c1_constant_problem(sig_c=10.0, sig_s=40.0, awr=12.0, density=0.01)
    prob.ww = mcsynth.WeightWindows(kind=mcsynth.WW_LINEAR, lin=(0.0, 3.0, 4.0), length=20.0, depth=depth,
                                    n_max=n_max)
    return prob


@pytest.mark.parametrize("in_flight", [0, 997, 64])
def test_infinite_medium_linear_windows_histories_identical(torch_cuda, in_flight):
    """Energy- and position-dependent windows in an infinite medium: splits and
    roulette happen; every history (summed over its copies, wherever they ran)
    and every tally sum equals the oracle's, with the default bank, a ragged
    bank refilled from the batch, and a bank so small that the copy bank and
    the per-slot stacks both fill up."""
    torch = torch_cuda
    prob = _infinite_ww()
    n = 4000
    _say(f"ww infinite identity in_flight={in_flight}")
    with Transport(prob) as t:
        g = _gpu_histories(torch, t, 11, 0, n, in_flight=in_flight)
        gl, _, _ = t.tallies(mc.MC_T_GLOBAL)
    r = oracle.run(oracle.OracleProblem(prob), 11, 0, n, history=True)
    _compare_histories(g, r.history)
    assert np.any(g["fate"] == mc.MC_FATE_ROULETTE)
    np.testing.assert_allclose(gl, r.glob / n, rtol=1e-11, atol=1e-300)
    assert gl[mc.MC_G_SPLIT] > 0 and gl[mc.MC_G_ROULETTE] > 0
    assert gl[mc.MC_G_SPLIT] * n == r.glob[oracle.G_SPLIT]
    assert gl[mc.MC_G_ROULETTE] * n == r.glob[oracle.G_ROULETTE]


def test_energy_dependent_xs_linear_windows_histories_identical(torch_cuda):
    torch = torch_cuda
    prob = mcsynth.c1_problem()
    prob.ww = mcsynth.WeightWindows(kind=mcsynth.WW_LINEAR, lin=(0.0, 2.0, 5.0), length=50.0)
    n = 2000
    _say("ww c1 identity")
    with Transport(prob) as t:
        g = _gpu_histories(torch, t, 1, 0, n)
    o = oracle.run(oracle.OracleProblem(prob), 1, 0, n, history=True).history
    _compare_histories(g, o)


def test_shallow_stack_and_event_cap_histories_identical(torch_cuda):
    """One pending split at most (further splits are skipped) and an event cap
    that loses copies (a lost copy hands over to the next pending one)."""
    torch = torch_cuda
    prob = _infinite_ww(depth=1, n_max=3)
    n = 3000
    _say("ww depth 1, event cap 6")
    with Transport(prob) as t:
        mc.mc_set_tuning(t.ctx, tail_particles=-1)
        g = _gpu_histories(torch, t, 5, 0, n, max_events=6, max_lost=n * 10)
        lost = t.stats()["lost"]
    o = oracle.run(oracle.OracleProblem(prob, max_events=6), 5, 0, n, history=True).history
    _compare_histories(g, o)
    assert lost > 0 and np.any(g["fate"] == mc.MC_FATE_LOST)


def _absorber(n_layers=20, sigma=0.02, ww=True, imp=(20, 1)):
    prob = mcsynth.slab_problem(sigma_t=(sigma,) * n_layers, thickness=(200.0 / n_layers,) * n_layers,
                                scatter_ratio=(0.0,) * n_layers)
    if ww:
        prob.ww = mcsynth.WeightWindows(kind=mcsynth.WW_LINEAR, lin=(0.0, sigma * 200.0, 0.0), length=200.0)
    if imp:
        prob.imp = mcsynth.ImportanceGrid(nx=imp[0], ne=imp[1], x0=0.0, x1=200.0)
    return prob


@pytest.mark.parametrize("in_flight", [0, 4096])
def test_absorber_slab_windows_and_importance_identical(torch_cuda, in_flight):
    """Beam into a 20-layer pure absorber, window checks at every crossing,
    importance grid on: histories, split counts and importance sums equal the
    oracle's."""
    torch = torch_cuda
    prob = _absorber(imp=(20, 4))
    n = 20_000
    _say(f"ww absorber identity in_flight={in_flight}")
    with Transport(prob) as t:
        g = _gpu_histories(torch, t, 9, 0, n, in_flight=in_flight)
        imp = t.importance()
        gl, _, _ = t.tallies(mc.MC_T_GLOBAL)
    r = oracle.run(oracle.OracleProblem(prob), 9, 0, n, history=True)
    _compare_histories(g, r.history)
    assert np.array_equal(imp[2], r.imp[2])
    np.testing.assert_allclose(imp[:2], r.imp[:2], rtol=1e-12, atol=0)
    np.testing.assert_allclose(gl, r.glob / n, rtol=1e-11, atol=1e-300)
    assert gl[mc.MC_G_SPLIT] > 0


def test_absorber_transmission_unbiased_with_windows(torch_cuda):
    sigma = 0.02
    truth = math.exp(-sigma * 200.0)
    k = mc.MC_G_LEAK_XHI
    res = {}
    for ww in (False, True):
        with Transport(_absorber(sigma=sigma, ww=ww, imp=None)) as t:
            for b in range(10):
                t.run_batch(21, b * 20_000, 20_000)
            g, s, _ = t.tallies(mc.MC_T_GLOBAL)
        assert abs(g[k] - truth) <= 3 * s[k], (ww, g[k], s[k], truth)
        res[ww] = s[k]
    assert res[True] < res[False] / 2


def test_importance_estimate_of_pure_absorber_on_gpu(torch_cuda):
    """Every transmitted particle entered every x-bin: the estimate of bin g is
    exp(-Sigma_t (L - x_g)), x_g its left edge (binomial error)."""
    sigma = 0.01
    prob = _absorber(n_layers=3, sigma=sigma, ww=False, imp=(20, 1))
    n = 500_000
    with Transport(prob) as t:
        t.run_batch(9, 0, n)
        num, den, cnt = t.importance()
    truth = np.exp(-sigma * (200.0 - np.arange(20) * 10.0))
    est = num / den
    se = np.sqrt(truth * (1 - truth) / den)
    n_fail, allowed, z = three_sigma(est, se, truth=truth)
    assert n_fail <= allowed, (n_fail, allowed, z)
    assert den[0] == n and np.array_equal(cnt, num)


def _scatter_slab():
    return mcsynth.slab_problem(sigma_t=(0.05, 0.08, 0.05), thickness=(60.0, 80.0, 60.0),
                                scatter_ratio=(0.7, 0.8, 0.7), awr=12.0)


def test_scattering_slab_windows_agree_with_analog_and_oracle(torch_cuda):
    torch = torch_cuda
    k = mc.MC_G_LEAK_XHI
    an = _scatter_slab()
    ww = _scatter_slab()
    ww.ww = mcsynth.WeightWindows(kind=mcsynth.WW_LINEAR, lin=(0.0, 8.0, 0.0), length=200.0)
    out = {}
    for name, prob in (("analog", an), ("ww", ww)):
        with Transport(prob) as t:
            for b in range(10):
                t.run_batch(31, b * 20_000, 20_000)
            out[name] = t.tallies(mc.MC_T_GLOBAL)[:2]
    (ga, sa), (gw, sw) = out["analog"], out["ww"]
    assert abs(gw[k] - ga[k]) <= 3 * math.hypot(sw[k], sa[k])
    assert sw[k] < sa[k]
    st = oracle.run_batches(oracle.OracleProblem(ww), 7, 10, 10_000)
    assert abs(gw[k] - st.mean["glob"][k]) <= 3 * math.hypot(sw[k], st.stderr["glob"][k])
    # same seed: the histories are the oracle's up to the last ulp of ln(xi)
    with Transport(ww) as t:
        g = _gpu_histories(torch, t, 7, 0, 5000)
    o = oracle.run(oracle.OracleProblem(ww), 7, 0, 5000, history=True).history
    assert np.mean(_same(g, o)) >= 0.99


def _net(scale=6.0, e_slope=0.5):
    """A fixed network with ln I rising by about 7 over the slab: first-layer
    units see depth with slopes 1 + j/64 (and, for odd j, the energy), the
    second layer passes them on, the output averages them.  Every weight is a
    BF16 value, so both sides use the same network."""
    j = np.arange(64)
    W1 = np.zeros((4, 64))
    W1[0] = 1.0 + j / 64.0
    W1[3] = e_slope * (j % 2)
    p = mlp.Params(W1, np.zeros(64), np.eye(64), np.zeros(64), np.full(64, scale / 64.0), 0.0)
    return p.flat()


def test_network_windows_match_oracle(torch_cuda):
    torch = torch_cuda
    prob = _scatter_slab()
    prob.ww = mcsynth.WeightWindows(kind=mcsynth.WW_MLP, mlp=_net(), length=200.0)
    op = oracle.OracleProblem(prob)
    k = mc.MC_G_LEAK_XHI
    _say("network windows")
    with Transport(prob) as t:
        g = _gpu_histories(torch, t, 41, 0, 5000)
        t.reset()
        for b in range(10):
            t.run_batch(43, b * 20_000, 20_000)
        gm, gs, _ = t.tallies(mc.MC_T_GLOBAL)
    o = oracle.run(op, 41, 0, 5000, history=True)
    assert o.glob[oracle.G_SPLIT] > 0 and o.glob[oracle.G_ROULETTE] > 0
    assert np.mean(_same(g, o.history)) >= 0.97
    st = oracle.run_batches(op, 47, 10, 10_000)
    for j in (k, mc.MC_G_TRACK, mc.MC_G_ABSORB):
        assert abs(gm[j] - st.mean["glob"][j]) <= 3 * math.hypot(gs[j], st.stderr["glob"][j]), j


def test_network_windows_keep_absorber_transmission_unbiased(torch_cuda):
    sigma = 0.02
    prob = _absorber(sigma=sigma, ww=False, imp=None)
    prob.ww = mcsynth.WeightWindows(kind=mcsynth.WW_MLP, mlp=_net(), length=200.0)
    k = mc.MC_G_LEAK_XHI
    with Transport(prob) as t:
        for b in range(10):
            t.run_batch(51, b * 20_000, 20_000)
        g, s, _ = t.tallies(mc.MC_T_GLOBAL)
    assert abs(g[k] - math.exp(-sigma * 200.0)) <= 3 * s[k]
    assert g[mc.MC_G_SPLIT] > 0


def test_invalid_window_settings_rejected(torch_cuda):
    prob = mcsynth.c1_constant_problem(sig_c=10.0, sig_s=40.0, awr=12.0, density=0.01)
    with Transport(prob) as t:
        for kw in ({"kind": 7}, {"kind": 1, "depth": 0}, {"kind": 1, "depth": 65}, {"kind": 1, "ratio": 1.0},
                   {"kind": 1, "n_max": 1}, {"imp_nx": 300, "imp_ne": 1}, {"imp_nx": 10, "imp_ne": 0},
                   {"imp_nx": 10, "imp_ne": 2, "imp_x0": 5.0, "imp_x1": 5.0}):
            with pytest.raises(mc.MCError) as e:
                mc.mc_set_weight_windows(t.ctx, **kw)
            assert e.value.code == mc.MC_EINVAL, kw
        with pytest.raises(mc.MCError) as e:
            mc.mc_get_importance(t.ctx, 4)
        assert e.value.code == mc.MC_ESTATE
        mc.mc_set_weight_windows(t.ctx, kind=mc.MC_WW_MLP)
        with pytest.raises(mc.MCError) as e:
            t.run_batch(1, 0, 100)
        assert e.value.code == mc.MC_ESTATE
        mc.mc_set_weight_windows(t.ctx)
        t.run_batch(1, 0, 100)
