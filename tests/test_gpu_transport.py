"""GPU parity of the event-based transport loop against the history-based
oracle (through the C ABI).

* Infinite medium (no geometry): each history is a function of its Philox
  stream, its cross sections (bit-identical lookups) and its kinematics (only
  +, *, / with contraction off), so GPU and oracle histories are identical:
  same fate, collisions, draws and final energy bit for bit, path length to
  the last ulp of the logarithm.
* With geometry: tallies agree within 3 sigma (independent seeds), with the
  multiple-comparison allowance; same-seed reruns are bitwise identical.
* Closed forms (1/Sigma_a, lattice volume fractions, slab transmission) hold on
  the GPU as they do for the oracle.
"""
import math
import sys

import numpy as np
import pytest

import mcsynth
import oracle
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


def _compare_histories(g, o):
    assert np.array_equal(g["fate"], o["fate"])
    assert np.array_equal(g["n_coll"], o["n_coll"])
    assert np.array_equal(g["n_cross"], o["n_cross"])
    assert np.array_equal(g["n_draws"], o["n_draws"])
    assert np.array_equal(g["E_final"], o["E_final"])
    np.testing.assert_allclose(g["track"], o["track"], rtol=1e-12)


@pytest.mark.parametrize("in_flight,tail", [(0, 0), (0, -1), (997, 0), (997, -1)])
def test_c1_histories_identical_to_oracle(torch_cuda, in_flight, tail):
    """All 10^4 C1 histories: the whole bank in flight and a ragged bank of 997
    slots refilled from the batch, each with the one-launch tail (the default)
    and with every event in the event kernels (tail = -1)."""
    torch = torch_cuda
    prob = mcsynth.c1_problem()
    _say(f"c1 identity in_flight={in_flight} tail={tail}")
    with Transport(prob) as t:
        mc.mc_set_tuning(t.ctx, tail_particles=tail)
        g = _gpu_histories(torch, t, 1, 0, prob.histories, in_flight=in_flight)
    o = oracle.run(oracle.OracleProblem(prob), 1, 0, prob.histories, history=True).history
    _compare_histories(g, o)
    assert np.all(g["fate"] > 0)


@pytest.mark.parametrize("n_nuc,in_flight", [(60, 0), (300, 997)])
def test_many_nuclide_histories_identical_to_oracle(torch_cuda, n_nuc, in_flight):
    """Materials of more than 16 nuclides: the collision starts its walk for the
    target nuclide at a checkpoint of the running scattering sum written by the
    lookup; the histories must still be the oracle's, collision for
    collision."""
    torch = torch_cuda
    prob = mcsynth.infinite_many_nuclides_problem(n_nuclides=n_nuc, histories=3000)
    _say(f"infinite medium of {n_nuc} nuclides, identity, in_flight={in_flight}")
    with Transport(prob) as t:
        mc.mc_set_tuning(t.ctx, tail_particles=-1, sort_min=1024)
        g = _gpu_histories(torch, t, 7, 0, prob.histories, in_flight=in_flight)
    o = oracle.run(oracle.OracleProblem(prob), 7, 0, prob.histories, history=True).history
    _compare_histories(g, o)


def test_c1_same_seed_tallies_match_oracle_to_rounding(torch_cuda):
    """Same seed and pids: identical histories, so the batch tallies differ only
    in summation order and the last ulp of ln(xi)."""
    prob = mcsynth.c1_problem()
    op = oracle.OracleProblem(prob)
    with Transport(prob) as t:
        for b in range(5):
            t.run_batch(1, b * 2000, 2000)
        gtl, _, meta = t.tallies(mc.MC_T_FLUX_TRACK)
        gco, _, _ = t.tallies(mc.MC_T_FLUX_COLLISION)
        ggl, _, _ = t.tallies(mc.MC_T_GLOBAL)
    assert meta.n_batches == 5 and meta.histories == 10_000
    st = oracle.run_batches(op, 1, 5, 2000)
    np.testing.assert_allclose(gtl, st.mean["tl"], rtol=1e-11, atol=1e-300)
    np.testing.assert_allclose(gco, st.mean["coll"], rtol=1e-11, atol=1e-300)
    np.testing.assert_allclose(ggl, st.mean["glob"], rtol=1e-11, atol=1e-300)


def test_c1_tallies_within_three_sigma_independent_seeds(torch_cuda):
    prob = mcsynth.c1_problem()
    with Transport(prob) as t:
        for b in range(10):
            t.run_batch(101, b * 2000, 2000)
        gm, gs, _ = t.tallies(mc.MC_T_FLUX_TRACK)
        glm, gls, _ = t.tallies(mc.MC_T_GLOBAL)
    st = oracle.run_batches(oracle.OracleProblem(prob), 1, 10, 2000)
    n_fail, allowed, z = three_sigma(gm, gs, st.mean["tl"], st.stderr["tl"])
    assert n_fail <= allowed, (n_fail, allowed, z)
    for k in (mc.MC_G_TRACK, mc.MC_G_COLL_EST, mc.MC_G_NCOLL, mc.MC_G_TRACK_ABS):
        assert abs(glm[k] - st.mean["glob"][k]) <= 3 * math.hypot(gls[k], st.stderr["glob"][k])


def test_infinite_constant_xs_closed_form_on_gpu(torch_cuda):
    prob = mcsynth.c1_constant_problem(sig_c=10.0, sig_s=40.0, awr=238.0, density=0.01)
    with Transport(prob) as t:
        for b in range(20):
            t.run_batch(11, b * 2000, 2000)
        g, s, _ = t.tallies(mc.MC_T_GLOBAL)
    for k, truth in ((mc.MC_G_TRACK, 10.0), (mc.MC_G_COLL_EST, 10.0), (mc.MC_G_NCOLL, 5.0)):
        assert abs(g[k] - truth) <= 3 * s[k], (k, g[k], s[k])
    assert g[mc.MC_G_ABSORB] == 1.0


def test_lattice_homogeneous_closed_form_on_gpu(torch_cuda):
    nuc = mcsynth.constant_nuclide(10.0, 40.0, 238.0)
    mat = mcsynth.Material(nuclides=np.array([0], np.int32), densities=np.array([0.01]))
    prob = mcsynth.lattice_homogeneous_problem([nuc], mat)
    _say("lattice homogeneous")
    with Transport(prob) as t:
        for b in range(20):
            t.run_batch(21, b * 5000, 5000)
        m, s, _ = t.tallies(mc.MC_T_FLUX_TRACK)
        g, gs, _ = t.tallies(mc.MC_T_GLOBAL)
    assert abs(g[mc.MC_G_TRACK] - 10.0) <= 3 * gs[mc.MC_G_TRACK]
    frac = math.pi * 0.41 ** 2 / 1.26 ** 2
    n_fail, allowed, z = three_sigma(m, s, truth=np.full(289, frac / 289 * 10.0))
    assert n_fail <= allowed, (n_fail, allowed, z)
    assert g[mc.MC_G_LEAK] == 0.0 and g[mc.MC_G_NCROSS] > 10


def test_c2_tallies_match_oracle_and_rerun_is_bitwise(torch_cuda):
    prob = mcsynth.c2_problem()
    _say("c2 parity")
    with Transport(prob) as t:
        for b in range(10):
            t.run_batch(202, b * 20_000, 20_000)
        gm, gs, _ = t.tallies(mc.MC_T_FLUX_TRACK)
        cm, cs, _ = t.tallies(mc.MC_T_FLUX_COLLISION)
        glm, gls, _ = t.tallies(mc.MC_T_GLOBAL)
        t.reset()
        for b in range(10):
            t.run_batch(202, b * 20_000, 20_000)
        gm2, _, _ = t.tallies(mc.MC_T_FLUX_TRACK)
        glm2, _, _ = t.tallies(mc.MC_T_GLOBAL)
    assert np.array_equal(gm, gm2) and np.array_equal(glm, glm2)
    st = oracle.run_batches(oracle.OracleProblem(prob), 2, 10, 20_000)
    for (a, sa), (b, sb) in (((gm, gs), (st.mean["tl"], st.stderr["tl"])),
                             ((cm, cs), (st.mean["coll"], st.stderr["coll"]))):
        n_fail, allowed, z = three_sigma(a, sa, b, sb)
        assert n_fail <= allowed, (n_fail, allowed, z)
    for k in (mc.MC_G_TRACK, mc.MC_G_COLL_EST, mc.MC_G_NCOLL, mc.MC_G_NCROSS, mc.MC_G_TRACK_ABS):
        assert abs(glm[k] - st.mean["glob"][k]) <= 3 * math.hypot(gls[k], st.stderr["glob"][k]), k
    assert glm[mc.MC_G_ABSORB] + glm[mc.MC_G_CUTOFF] == pytest.approx(1.0, abs=1e-12)


def test_c2_tail_and_event_paths_agree(torch_cuda):
    """The one-launch tail and the event kernels run the same histories; the
    tallies differ only in summation order."""
    torch = torch_cuda
    prob = mcsynth.c2_problem()
    n = 50_000
    res = {}
    for tail in (-1, 0, 60_000):
        with Transport(prob) as t:
            mc.mc_set_tuning(t.ctx, tail_particles=tail)
            h = _gpu_histories(torch, t, 2, 0, n)
            m, _, _ = t.tallies(mc.MC_T_FLUX_TRACK)
            g, _, _ = t.tallies(mc.MC_T_GLOBAL)
            res[tail] = (h, m, g, t.stats())
    h0, m0, g0, s0 = res[-1]
    assert s0["tail_particles"] == 0 and res[60_000][3]["tail_particles"] == n
    for tail in (0, 60_000):
        h, m, g, _ = res[tail]
        for f in ("fate", "n_coll", "n_cross", "n_draws", "E_final"):
            assert np.array_equal(h[f], h0[f]), (tail, f)
        np.testing.assert_allclose(m, m0, rtol=1e-10)
        np.testing.assert_allclose(g, g0, rtol=1e-10)


def test_c2_same_seed_histories_mostly_identical(torch_cuda):
    """With geometry the device and host transcendental functions may differ
    in the last ulp, so a few histories can diverge; most stay identical."""
    torch = torch_cuda
    prob = mcsynth.c2_problem()
    n = 20_000
    with Transport(prob) as t:
        g = _gpu_histories(torch, t, 2, 0, n)
    o = oracle.run(oracle.OracleProblem(prob), 2, 0, n, history=True).history
    same = (g["n_draws"] == o["n_draws"]) & (g["E_final"] == o["E_final"]) & (g["fate"] == o["fate"])
    _say(f"c2 identical histories: {same.mean():.4f}")
    assert same.mean() > 0.9
    assert np.all(g["fate"] > 0)


def test_slab_transmission_closed_form_on_gpu(torch_cuda):
    prob = mcsynth.slab_problem(sigma_t=(0.01, 0.02, 0.005), thickness=(60.0, 80.0, 60.0),
                                scatter_ratio=(0.5, 0.8, 0.3), awr=12.0)
    tau = 0.01 * 60 + 0.02 * 80 + 0.005 * 60
    with Transport(prob) as t:
        for b in range(10):
            t.run_batch(5, b * 10_000, 10_000)
        g, s, _ = t.tallies(mc.MC_T_GLOBAL)
    assert abs(g[mc.MC_G_LEAK_XHI_UNC] - math.exp(-tau)) <= 3 * s[mc.MC_G_LEAK_XHI_UNC]
    assert g[mc.MC_G_LEAK] > g[mc.MC_G_LEAK_XHI] > g[mc.MC_G_LEAK_XHI_UNC]
    assert g[mc.MC_G_ABSORB] + g[mc.MC_G_LEAK] + g[mc.MC_G_CUTOFF] == pytest.approx(1.0, abs=1e-12)


def test_inactive_batch_and_ragged_sizes(torch_cuda):
    """no_tally leaves the binned flux tallies at zero and the global tallies
    unchanged; n = 1 and ragged in-flight sizes run."""
    prob = mcsynth.c1_problem()
    with Transport(prob) as t:
        t.run_batch(3, 0, 3001)
        g_on, _, _ = t.tallies(mc.MC_T_GLOBAL)
        t.reset()
        t.run_batch(3, 0, 3001, no_tally=True)
        g_off, _, _ = t.tallies(mc.MC_T_GLOBAL)
        f_off, _, _ = t.tallies(mc.MC_T_FLUX_TRACK)
        assert np.all(f_off == 0.0)
        assert np.array_equal(g_on, g_off)
        t.reset()
        t.run_batch(3, 5, 1)
        g1, _, meta = t.tallies(mc.MC_T_GLOBAL)
        assert meta.histories == 1 and g1[mc.MC_G_ABSORB] + g1[mc.MC_G_CUTOFF] == 1.0


def test_event_cap_reports_lost_particles(torch_cuda):
    torch = torch_cuda
    prob = mcsynth.c1_problem()
    with Transport(prob) as t:
        with pytest.raises(mc.MCError) as e:
            t.run_batch(1, 0, 500, max_events=3)
        assert e.value.code == mc.MC_ELOST
        h = _gpu_histories(torch, t, 1, 0, 500, max_events=3, max_lost=500)
    assert np.all((h["fate"] == mc.MC_FATE_LOST) | (h["n_coll"] <= 3))
    assert np.any(h["fate"] == mc.MC_FATE_LOST)


def test_invalid_inputs_rejected(torch_cuda):
    ctx = mc.mc_create(0)
    try:
        E = [np.array([1.0, 0.5, 2.0])]
        with pytest.raises(mc.MCError) as e:
            mc.mc_init_materials(ctx, E, [np.ones(3)], [np.ones(3)], [1.0], [[0]], [[0.1]], 16)
        assert e.value.code == mc.MC_EINVAL and "increasing" in str(e.value)
        with pytest.raises(mc.MCError) as e:
            mc.mc_run_batch(ctx, 1, 0, 10)
        assert e.value.code == mc.MC_ESTATE
        E = [np.array([1e-5, 1.0, 2e7])]
        with pytest.raises(mc.MCError) as e:
            mc.mc_init_materials(ctx, E, [np.ones(3)], [np.ones(3)], [1.0], [[0]], [[-0.1]], 16)
        assert e.value.code == mc.MC_EINVAL
    finally:
        mc.mc_destroy(ctx)


def test_core_of_assemblies_matches_oracle(torch_cuda):
    """A 3x3 core of three assembly types (open guide tubes, absorber rods,
    a water assembly) on the flat 51x51 lattice: same-seed histories mostly
    identical to the oracle's (device and host logarithms may differ in the
    last ulp), and the flux of every pin cell (a 51x51x1 mesh) within 3
    sigma of the oracle's on independent batches."""
    torch = torch_cuda
    prob = mcsynth.core_problem()
    n = 20_000
    _say("3x3 core of assemblies")
    with Transport(prob) as t:
        g = _gpu_histories(torch, t, 31, 0, n)
        t.reset()
        for b in range(20):
            t.run_batch(310, b * n, n)
        gm, gs, _ = t.tallies(mc.MC_T_FLUX_TRACK)
    o = oracle.run(oracle.OracleProblem(prob), 31, 0, n, history=True).history
    same = (g["n_draws"] == o["n_draws"]) & (g["E_final"] == o["E_final"]) & (g["fate"] == o["fate"])
    _say(f"core identical histories: {same.mean():.4f}")
    assert same.mean() > 0.9 and np.all(g["fate"] > 0)
    assert np.all(gm > 0.0)
    st = oracle.run_batches(oracle.OracleProblem(prob), 311, 20, n)
    # 2601 bins, each side's standard error from 20 batches: Student's t
    # allowance (2 x 19 degrees of freedom)
    n_fail, allowed, z = three_sigma(gm, gs, st.mean["tl"], st.stderr["tl"], dof=38)
    assert n_fail <= allowed, (n_fail, allowed, z)


def test_event_loop_counts_do_not_depend_on_launch_choices(torch_cuda):
    """The host runs the event loop one iteration behind the GPU and takes
    its choices (sort or not, bank size) from the previous iteration's queue
    lengths; the histories, and so the numbers of lookups, flights and
    iterations it reports, must not depend on them: every iteration counted
    once, sorted or not."""
    torch = torch_cuda
    prob = mcsynth.c2_problem()
    n = 60_000
    out = {}
    for name, tune in (("sorted", dict(sort_min=1)), ("unsorted", dict(sort_min=1 << 30)),
                       ("ragged", dict(sort_min=1, in_flight=7_777))):
        with Transport(prob) as t:
            mc.mc_set_tuning(t.ctx, tail_particles=-1, **tune)
            h = _gpu_histories(torch, t, 2, 0, n)
            out[name] = (h, t.stats())
    hs, ss = out["sorted"]
    hu, su = out["unsorted"]
    hr, sr = out["ragged"]
    for f in ("fate", "n_coll", "n_cross", "n_draws", "E_final"):
        assert np.array_equal(hs[f], hu[f]) and np.array_equal(hs[f], hr[f]), f
    # every history's lookups: one at its start and one after each collision
    # that leaves it alive (C2's materials change at crossings too)
    assert ss["lookups"] == su["lookups"] == sr["lookups"] > n
    assert ss["flights"] == su["flights"] == sr["flights"] == int(hs["n_coll"].sum() + hs["n_cross"].sum())
    # (an iteration whose predecessor had no lookups is not sorted: the
    # choice follows the previous lengths)
    assert 0.99 * ss["lookups"] <= ss["sorted_lookups"] <= ss["lookups"] and su["sorted_lookups"] == 0
    assert ss["iterations"] == su["iterations"] and sr["iterations"] > ss["iterations"]
    assert ss["tail_particles"] == su["tail_particles"] == sr["tail_particles"] == 0
