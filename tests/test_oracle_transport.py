"""Closed-form and invariant pins for the oracle's history-based transport.

Each test compares batch means with a value fixed by transport theory (or by
a symmetry of the problem), at three standard errors with the
multiple-comparison allowance of tests/stats.py.  Seeds are fixed, so each
test is deterministic.
"""
import math

import numpy as np
import pytest

import mcsynth
import oracle
from tests.stats import three_sigma


def _batches(prob, n_batches, per_batch, seed=None):
    op = oracle.OracleProblem(prob)
    return oracle.run_batches(op, prob.seed if seed is None else seed, n_batches, per_batch)


def test_infinite_constant_xs_track_length_and_collisions():
    """Infinite medium, constant cross sections: the expected track length per
    source particle is 1/Sigma_a, the expected number of collisions
    Sigma_t/Sigma_a, and the collision estimator of the total flux is also
    1/Sigma_a.  (A = 238 keeps every history far above the energy cutoff.)"""
    prob = mcsynth.c1_constant_problem(sig_c=10.0, sig_s=40.0, awr=238.0, density=0.01)
    Sa, St = 0.1, 0.5
    st = _batches(prob, 20, 2000)
    g, s = st.mean["glob"], st.stderr["glob"]
    for k, truth in ((oracle.G_TRACK, 1 / Sa), (oracle.G_COLL_EST, 1 / Sa),
                     (oracle.G_NCOLL, St / Sa), (oracle.G_TRACK_ABS, 1.0)):
        assert abs(g[k] - truth) <= 3 * s[k], (k, g[k], truth, s[k])
    assert g[oracle.G_ABSORB] == 1.0 and g[oracle.G_CUTOFF] == 0.0


def _hydrogen_bins(edges, E0, Sigma_t, c, e_cut):
    """Track-length flux per source particle in each energy bin for slowing
    down in hydrogen (A = 1) with constant cross sections, scattering ratio c:
    collided flux per unit energy (c / (Sigma_t E0)) (E0 / E)^c below E0, plus
    the uncollided 1/Sigma_t at E0."""
    out = np.zeros(edges.size - 1)
    for b in range(out.size):
        lo, hi = max(edges[b], e_cut), min(edges[b + 1], E0)
        if hi > lo:
            out[b] = c * E0 ** (c - 1) / Sigma_t * (hi ** (1 - c) - lo ** (1 - c)) / (1 - c)
        if edges[b] <= E0 < edges[b + 1]:
            out[b] += 1 / Sigma_t
    return out


def test_hydrogen_slowing_down_spectrum():
    c = 0.5
    prob = mcsynth.c1_constant_problem(sig_c=25.0, sig_s=25.0, awr=1.0, density=0.01, n_bins=50)
    St = 0.5
    st = _batches(prob, 20, 2500)
    truth = _hydrogen_bins(prob.tally.energy_edges, 2.0e6, St, c, prob.energy_cutoff)
    # bins reached by few histories (deep below the source energy) have skewed,
    # nearly empty batch tallies; test them together, the rest bin by bin
    well = truth > 1e-3
    n_fail, allowed, z = three_sigma(st.mean["tl"][well], st.stderr["tl"][well], truth=truth[well])
    assert n_fail <= allowed, (n_fail, allowed, z)
    rare_m = st.mean["tl"][~well].sum()
    rare_s = np.sqrt(np.sum(st.stderr["tl"][~well] ** 2))
    assert abs(rare_m - truth[~well].sum()) <= 3 * rare_s + 1e-4
    # bins above the source energy receive nothing
    assert np.all(st.mean["tl"][prob.tally.energy_edges[:-1] > 2.0e6] == 0.0)
    # the total is 1/Sigma_a less what the cutoff removes
    total = (1 / St) * (1 + c / (1 - c) * (1 - (prob.energy_cutoff / 2.0e6) ** (1 - c)))
    assert abs(st.mean["glob"][oracle.G_TRACK] - total) <= 3 * st.stderr["glob"][oracle.G_TRACK]


def test_absorption_balance_and_estimator_agreement_c1():
    """Energy-dependent data (the 4-nuclide infinite medium): every history ends
    in absorption or at the energy cutoff; the track-length estimate of
    absorption, sum w d Sigma_a, has the analog absorption as its expectation;
    track-length and collision estimators of the flux agree bin by bin."""
    prob = mcsynth.c1_problem()
    st = _batches(prob, 10, 1000)
    g, s = st.mean["glob"], st.stderr["glob"]
    assert g[oracle.G_ABSORB] + g[oracle.G_CUTOFF] == pytest.approx(1.0, abs=1e-15)
    assert abs(g[oracle.G_TRACK_ABS] - g[oracle.G_ABSORB]) <= 3 * math.hypot(
        s[oracle.G_TRACK_ABS], s[oracle.G_ABSORB])
    n_fail, allowed, z = three_sigma(st.mean["tl"], st.stderr["tl"], st.mean["coll"], st.stderr["coll"])
    assert n_fail <= allowed, (n_fail, allowed, z)


def test_homogeneous_lattice_is_infinite_medium():
    """One material everywhere, uniform source, reflective faces: the lattice is
    an infinite medium, so with constant cross sections the track length per
    source particle is 1/Sigma_a, and each pin's share of it is its volume
    fraction pi r^2 / (P^2 * 289)."""
    nuc = mcsynth.constant_nuclide(10.0, 40.0, 238.0)
    mat = mcsynth.Material(nuclides=np.array([0], np.int32), densities=np.array([0.01]))
    prob = mcsynth.lattice_homogeneous_problem([nuc], mat, histories=20_000)
    st = _batches(prob, 20, 2500)
    g, s = st.mean["glob"], st.stderr["glob"]
    assert abs(g[oracle.G_TRACK] - 10.0) <= 3 * s[oracle.G_TRACK]
    frac = math.pi * 0.41 ** 2 / 1.26 ** 2
    truth = np.full(289, frac / 289 * 10.0)
    n_fail, allowed, z = three_sigma(st.mean["tl"], st.stderr["tl"], truth=truth)
    assert n_fail <= allowed, (n_fail, allowed, z)
    # the sum over pins, with its own batch error
    tot = st.mean["tl"].sum()
    assert abs(tot - frac * 10.0) < 0.02 * frac * 10.0
    assert g[oracle.G_NCROSS] > 0


def test_c2_pin_flux_has_square_symmetry():
    """The C2 layout and source are invariant under the 8 symmetries of the
    square, so the per-pin flux is too (compared with the x-mirror and the
    transpose)."""
    prob = mcsynth.c2_problem(grid_range=(10_000, 60_000))
    st = _batches(prob, 10, 4000)
    m = st.mean["tl"].reshape(17, 17)
    s = st.stderr["tl"].reshape(17, 17)
    for mm, ss in ((m[:, ::-1], s[:, ::-1]), (m.T, s.T)):
        n_fail, allowed, z = three_sigma(m.ravel(), s.ravel(), mm.ravel(), ss.ravel())
        assert n_fail <= allowed, (n_fail, allowed, z)
    # absorption pins (material B) differ from fuel pins: the layout matters
    assert st.mean["glob"][oracle.G_ABSORB] == 1.0


def test_slab_pure_absorber_transmission():
    """A pure absorber under a normal beam transmits exp(-sum Sigma_t,i x_i)."""
    prob = mcsynth.slab_problem(sigma_t=(0.01, 0.02, 0.005), thickness=(60.0, 80.0, 60.0),
                                scatter_ratio=(0.0, 0.0, 0.0))
    st = _batches(prob, 10, 10_000)
    tau = 0.01 * 60 + 0.02 * 80 + 0.005 * 60
    k = oracle.G_LEAK_XHI
    assert abs(st.mean["glob"][k] - math.exp(-tau)) <= 3 * st.stderr["glob"][k]
    assert st.mean["glob"][oracle.G_NCOLL] == pytest.approx(1 - math.exp(-tau), abs=0.01)


def test_slab_uncollided_transmission_with_scattering():
    """With scattering the uncollided transmission is still exp(-tau_t)."""
    prob = mcsynth.slab_problem(sigma_t=(0.01, 0.02, 0.005), thickness=(60.0, 80.0, 60.0),
                                scatter_ratio=(0.5, 0.8, 0.3), awr=12.0)
    st = _batches(prob, 10, 10_000)
    tau = 0.01 * 60 + 0.02 * 80 + 0.005 * 60
    k = oracle.G_LEAK_XHI_UNC
    assert abs(st.mean["glob"][k] - math.exp(-tau)) <= 3 * st.stderr["glob"][k]
    assert st.mean["glob"][oracle.G_LEAK_XHI] > st.mean["glob"][k]


def test_oracle_result_independent_of_thread_count():
    prob = mcsynth.c2_problem(grid_range=(10_000, 12_000))
    op = oracle.OracleProblem(prob)
    a = oracle.run(op, 5, 100, 3000, threads=1)
    b = oracle.run(op, 5, 100, 3000, threads=8)
    assert np.array_equal(a.tl, b.tl) and np.array_equal(a.glob, b.glob)
