"""Pins of the oracle's reaction channels (per-nuclide reaction cross sections
tabulated on each nuclide's grid, the data a depletion tally gathers; paper
section 2, "Tallying") and of their track-length reaction-rate tally.

* A channel that copies the capture cross section gives the macroscopic
  capture cross section and, tallied, the track-length absorption sum: the
  same numbers bit for bit in one material.
* A constant channel c gives c times the sum of the densities, and tallied
  c * (sum of densities) * track length.
* Channels are linear: a channel 2 sigma_c + 3 sigma_s tallies 2 R_c + 3 R_s.
* The lookup of a channel equals per-nuclide numpy interpolation summed in
  material order, within the interpolation rounding bound.
* Constant cross sections in an infinite medium: the capture-copy channel's
  rate per source particle is the absorption probability, 1.
A transposed channel layout, a wrong nuclide offset or a dropped density
fails one of these.
"""
import numpy as np
import pytest

import mcsynth
import oracle


def _copy_channels(prob, extra=None):
    """Channels [sigma_c, sigma_s, 2 sigma_c + 3 sigma_s] (+ a constant column)."""
    chans = []
    for n in prob.nuclides:
        cols = [n.sig_c, n.sig_s, 2.0 * n.sig_c + 3.0 * n.sig_s]
        if extra is not None:
            cols.append(np.full(n.E.size, extra))
        chans.append(np.ascontiguousarray(np.stack(cols, 1)))
    prob.channels = chans
    return prob


def test_capture_copy_channel_equals_sigma_a_bitwise():
    prob = _copy_channels(mcsynth.c1_problem(), extra=1.5)
    op = oracle.OracleProblem(prob)
    rng = np.random.default_rng(3)
    E = mcsynth.lookup_energies(rng, 4000)
    Sa, Ss = oracle.macro_xs(op, 0, E)
    X = oracle.macro_channels(op, 0, E)
    assert np.array_equal(X[:, 0], Sa) and np.array_equal(X[:, 1], Ss)
    dens = prob.materials[0].densities
    ref = 0.0
    for d in dens:
        ref = ref + d * 1.5
    assert np.all(X[:, 3] == ref)


def test_channel_lookup_matches_numpy_interp():
    prob = mcsynth.with_channels(mcsynth.c2_problem(histories=1000), 4)
    op = oracle.OracleProblem(prob)
    rng = np.random.default_rng(11)
    E = mcsynth.lookup_energies(rng, 3000)
    for m, mat in enumerate(prob.materials):
        X = oracle.macro_channels(op, m, E)
        ref = np.zeros_like(X)
        bound = np.zeros_like(X)
        for q, d in zip(mat.nuclides, mat.densities):
            for x in range(4):
                v = np.interp(E, prob.nuclides[q].E, prob.channels[q][:, x])
                ref[:, x] += d * v
                bound[:, x] += d * np.abs(v)
        # lerp rounding (a few ulps per term) plus the ordered positive sum
        assert np.all(np.abs(X - ref) <= 1e-13 * bound + 1e-300)


def test_reaction_tally_identities_in_infinite_medium():
    prob = _copy_channels(mcsynth.c1_problem(histories=2000), extra=0.7)
    op = oracle.OracleProblem(prob)
    r = oracle.run(op, prob.seed, 0, 2000)
    rr = r.rr[0]
    # the capture copy is the track-length absorption sum, bit for bit
    assert rr[0] == r.glob[oracle.G_TRACK_ABS]
    # linearity (rounding only)
    assert abs(rr[2] - (2.0 * rr[0] + 3.0 * rr[1])) <= 1e-12 * rr[2]
    # constant channel: 0.7 * sum of densities * track length
    dsum = 0.0
    for d in prob.materials[0].densities:
        dsum = dsum + d * 0.7
    assert abs(rr[3] - dsum * r.glob[oracle.G_TRACK]) <= 1e-12 * rr[3]


def test_reaction_tally_per_material_in_lattice():
    """Three materials: per-material rates of the capture copy add up to the
    track-length absorption sum; a material's constant channel is its density
    sum times the track length spent in it (> 0 for every material)."""
    prob = _copy_channels(mcsynth.c2_problem(histories=3000), extra=1.0)
    op = oracle.OracleProblem(prob)
    r = oracle.run(op, prob.seed, 0, 3000)
    assert r.rr.shape == (3, 4)
    assert abs(r.rr[:, 0].sum() - r.glob[oracle.G_TRACK_ABS]) <= 1e-12 * r.glob[oracle.G_TRACK_ABS]
    track_in = np.array([r.rr[m, 3] / prob.materials[m].densities.sum() for m in range(3)])
    assert np.all(track_in > 0)
    assert abs(track_in.sum() - r.glob[oracle.G_TRACK]) <= 1e-10 * r.glob[oracle.G_TRACK]


def test_capture_copy_rate_is_absorption_probability():
    prob = mcsynth.c1_constant_problem(sig_c=10.0, sig_s=40.0, awr=238.0, density=0.01)
    prob = _copy_channels(prob)
    st = oracle.run_batches(oracle.OracleProblem(prob), prob.seed, 20, 1000)
    m, s = st.mean["rr"][0], st.stderr["rr"][0]
    assert abs(m[0] - 1.0) <= 3 * s[0] + 1e-12, (m[0], s[0])
