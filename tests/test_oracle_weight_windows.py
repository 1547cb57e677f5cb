"""Pins for the oracle's weight windows (split / roulette with a per-history
stack of pending copies), its importance network forward pass and its
forward importance estimate.

Weight windows change the variance, never the expectation: the closed forms
of the analog game must still hold with them, with smaller errors.
"""
import math

import numpy as np
import pytest
import torch

import mcsynth
import oracle
from oracle import mlp
from tests.stats import three_sigma


def test_c_network_matches_numpy_network():
    rng = np.random.default_rng(0)
    p = mlp.init_params(1)
    p.b1 = rng.normal(0, 0.2, 64)
    p.b2 = rng.normal(0, 0.2, 64)
    p.b3 = 0.7
    f = np.stack([rng.uniform(0, 1, 500), rng.uniform(-1, 1, 500), rng.uniform(-1, 1, 500),
                  rng.uniform(0, 1, 500)], axis=1)
    ref, _ = mlp.forward(p, f)
    got = np.array([oracle.mlp_forward(p.flat(), row) for row in f])
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_c_bf16_matches_torch():
    rng = np.random.default_rng(2)
    a = rng.normal(size=2000) * 10.0 ** rng.integers(-10, 10, 2000)
    ref = torch.tensor(a.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal([oracle.bf16(v) for v in a], ref)


def test_child_lineages_are_distinct_and_nonzero():
    seen = set()
    for a in (0, 1, 12345):
        for s in range(20):
            for k in range(1, 10):
                v = oracle.child_lineage(a, s, k)
                assert v != 0
                seen.add((a, v))
    assert len(seen) == 3 * 20 * 9


def _absorber_slab(n_layers=20, sigma=0.02):
    return mcsynth.slab_problem(sigma_t=(sigma,) * n_layers, thickness=(200.0 / n_layers,) * n_layers,
                                scatter_ratio=(0.0,) * n_layers)


def test_weight_windows_keep_pure_absorber_transmission_unbiased():
    """Beam into a pure absorber cut into 20 layers (a window check at every
    crossing), importance exp(Sigma_t x): the transmission is exp(-tau) with
    and without windows, and the windows cut its standard error."""
    sigma = 0.02
    tau = sigma * 200.0
    prob = _absorber_slab(sigma=sigma)
    an = oracle.run_batches(oracle.OracleProblem(prob), 5, 10, 5000)
    prob.ww = mcsynth.WeightWindows(kind=mcsynth.WW_LINEAR, lin=(0.0, tau, 0.0), length=200.0)
    ww = oracle.run_batches(oracle.OracleProblem(prob), 5, 10, 5000)
    k = oracle.G_LEAK_XHI
    for st in (an, ww):
        assert abs(st.mean["glob"][k] - math.exp(-tau)) <= 3 * st.stderr["glob"][k]
    assert ww.stderr["glob"][k] < an.stderr["glob"][k] / 2
    assert ww.mean["glob"][oracle.G_SPLIT] > 0


def test_weight_windows_keep_infinite_medium_closed_form():
    """Energy-dependent importance in an infinite medium with constant cross
    sections: splits and roulette happen, the track length stays 1/Sigma_a."""
    prob = mcsynth.c1_constant_problem(sig_c=10.0, sig_s=40.0, awr=12.0, density=0.01)
    prob.ww = mcsynth.WeightWindows(kind=mcsynth.WW_LINEAR, lin=(0.0, 3.0, 4.0), length=20.0)
    st = oracle.run_batches(oracle.OracleProblem(prob), 11, 20, 2000)
    g, s = st.mean["glob"], st.stderr["glob"]
    assert abs(g[oracle.G_TRACK] - 10.0) <= 3 * s[oracle.G_TRACK]
    assert abs(g[oracle.G_ABSORB] + g[oracle.G_CUTOFF] - 1.0) <= 3 * math.hypot(s[oracle.G_ABSORB], s[oracle.G_CUTOFF])
    assert g[oracle.G_SPLIT] > 0 and g[oracle.G_ROULETTE] > 0


def test_weight_windows_agree_with_analog_in_a_scattering_slab():
    prob = mcsynth.slab_problem(sigma_t=(0.05, 0.08, 0.05), thickness=(60.0, 80.0, 60.0),
                                scatter_ratio=(0.7, 0.8, 0.7), awr=12.0)
    an = oracle.run_batches(oracle.OracleProblem(prob), 7, 10, 10_000)
    prob.ww = mcsynth.WeightWindows(kind=mcsynth.WW_LINEAR, lin=(0.0, 8.0, 0.0), length=200.0)
    ww = oracle.run_batches(oracle.OracleProblem(prob), 7, 10, 10_000)
    k = oracle.G_LEAK_XHI
    d = abs(ww.mean["glob"][k] - an.mean["glob"][k])
    assert d <= 3 * math.hypot(ww.stderr["glob"][k], an.stderr["glob"][k])
    assert ww.stderr["glob"][k] < an.stderr["glob"][k]


def test_split_generation_limit_bounds_splits_and_keeps_closed_form():
    """A copy made by `depth` splits along its line splits no further: with
    depth 1 and n_max 3 a history makes at most 2 copies, and the infinite
    medium track length stays 1/Sigma_a."""
    prob = mcsynth.c1_constant_problem(sig_c=10.0, sig_s=40.0, awr=12.0, density=0.01)
    prob.ww = mcsynth.WeightWindows(kind=mcsynth.WW_LINEAR, lin=(0.0, 3.0, 4.0), length=20.0, depth=1, n_max=3)
    op = oracle.OracleProblem(prob)
    n = 4000
    r = oracle.run(op, 13, 0, n, history=True)
    assert 0 < r.glob[oracle.G_SPLIT] <= 2 * n
    st = oracle.run_batches(op, 13, 20, 2000)
    assert abs(st.mean["glob"][oracle.G_TRACK] - 10.0) <= 3 * st.stderr["glob"][oracle.G_TRACK]


def test_history_record_keeps_the_source_copy_fate():
    """With windows, the record's fate, energy and weight are those of the
    source particle's own copy; roulette can end it, and its weight is then
    what it carried when it died (never above the window's survival weight)."""
    prob = mcsynth.c1_constant_problem(sig_c=10.0, sig_s=40.0, awr=12.0, density=0.01)
    prob.ww = mcsynth.WeightWindows(kind=mcsynth.WW_LINEAR, lin=(0.0, 3.0, 4.0), length=20.0)
    h = oracle.run(oracle.OracleProblem(prob), 17, 0, 3000, history=True).history
    assert set(np.unique(h["fate"])) <= {oracle.FATE_ABSORBED, oracle.FATE_CUTOFF, oracle.FATE_ROULETTE}
    assert np.any(h["fate"] == oracle.FATE_ROULETTE)
    assert np.all(h["weight"] > 0) and np.all(h["E_final"] > 0)


def test_forward_importance_of_a_pure_absorber():
    """Beam into a pure absorber: every transmitted particle entered every
    x-bin, so the forward estimate of bin g is exp(-Sigma_t (L - x_g)), x_g its
    left edge."""
    sigma = 0.01
    prob = _absorber_slab(n_layers=3, sigma=sigma)
    prob.imp = mcsynth.ImportanceGrid(nx=20, ne=1, x0=0.0, x1=200.0)
    op = oracle.OracleProblem(prob)
    n = 200_000
    r = oracle.run(op, 9, 0, n)
    num, den, cnt = r.imp
    x_left = np.arange(20) * 10.0
    truth = np.exp(-sigma * (200.0 - x_left))
    est = num / den
    # binomial error of the ratio (num counts particles reaching L among den)
    se = np.sqrt(truth * (1 - truth) / den)
    n_fail, allowed, z = three_sigma(est, se, truth=truth)
    assert n_fail <= allowed, (n_fail, allowed, z)
    assert den[0] == n and np.all(cnt == num)
