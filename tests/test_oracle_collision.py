"""Pins of the oracle's collision: which nuclide a scattering picks, and the
energy it leaves with.

A scattering picks its target nuclide with probability N_k sigma_s,k / Sigma_s
(the first nuclide, in material order, whose running sum of N_k sigma_s,k
reaches xi Sigma_s; paper section 2, the collision event).  With constant
cross sections that probability is the same at every collision, so the number
of scatterings on nuclide k among all of them is binomial with p_k.  An
elastic scattering off a target of mass ratio A at rest, isotropic in the
centre of mass, leaves E'/E uniform on [alpha, 1], alpha = ((A-1)/(A+1))^2,
so the lethargy gain ln(E/E') of a scattering on k has the textbook mean
xi_k = 1 + alpha ln(alpha) / (1 - alpha) (xi = 1 for A = 1) and a closed-form
second moment.

The mixtures are chosen so that a plausible slip in the selection fails: a
dropped density (p_k proportional to sigma_s,k), capture in place of
scattering (p_k proportional to N_k sigma_c,k), a pick one nuclide late or
early, or a mass ratio read at the wrong index.  Each test also checks that
those alternatives would be many standard errors away, so the pin has power.
"""
import math

import numpy as np

import mcsynth
import oracle


def _mixture(parts):
    """Infinite medium of constant-cross-section nuclides: parts = [(A, sigma_c,
    sigma_s, density)] in material order."""
    nucs = [mcsynth.constant_nuclide(sc, ss, A) for A, sc, ss, _ in parts]
    mat = mcsynth.Material(nuclides=np.arange(len(parts), dtype=np.int32),
                           densities=np.array([d for *_, d in parts], np.float64))
    return mcsynth.Problem(name="mixture", nuclides=nucs, materials=[mat],
                           geometry=mcsynth.Geometry(kind=mcsynth.GEOM_INFINITE, material=0),
                           source=mcsynth.Source(kind=mcsynth.SRC_POINT),
                           tally=mcsynth.Tally(mcsynth.TALLY_ENERGY, mcsynth.energy_edges(10)),
                           histories=1, batches=1, seed=21)


def _alpha(A):
    return ((A - 1.0) / (A + 1.0)) ** 2


def _xi_moments(A):
    """Mean and variance of ln(E/E') for E'/E ~ U[alpha, 1]."""
    a = _alpha(A)
    if a == 0.0:
        return 1.0, 1.0
    m1 = 1.0 + a * math.log(a) / (1.0 - a)
    # E[ln^2 x] for x ~ U[a, 1]: (2 - (a ln^2 a - 2 a ln a + 2 a)) / (1 - a)
    m2 = (2.0 - (a * math.log(a) ** 2 - 2.0 * a * math.log(a) + 2.0 * a)) / (1.0 - a)
    return m1, m2 - m1 * m1


def _binomial_z(count, n, p):
    return (count - n * p) / math.sqrt(max(n * p * (1.0 - p), 1e-300))


PARTS = [  # (A, sigma_c, sigma_s, N): N sigma_s = 0.015, 0.035, 0.05
    (1.0, 2.0, 7.5, 0.002),
    (12.0, 0.1, 3.5, 0.01),
    (56.0, 0.3, 2.5, 0.02),
]


def test_target_fractions_follow_density_times_scattering():
    prob = _mixture(PARTS)
    ns = oracle.scatter_stats(oracle.OracleProblem(prob), seed=31, first_pid=0, n=20_000)
    counts = ns[:, 0]
    n = counts.sum()
    assert n > 100_000, n
    ns_s = np.array([d * ss for _, _, ss, d in PARTS])
    p = ns_s / ns_s.sum()
    z = [_binomial_z(counts[k], n, p[k]) for k in range(3)]
    assert max(abs(v) for v in z) <= 3.0, (counts / n, p, z)
    # the slips listed above would be far off
    alternatives = {
        "density dropped": np.array([ss for _, _, ss, _ in PARTS]),
        "capture for scattering": np.array([d * sc for _, sc, _, d in PARTS]),
        "one nuclide late": np.array([0.0, ns_s[0], ns_s[1] + ns_s[2]]),
        "one nuclide early": np.array([ns_s[0] + ns_s[1], ns_s[2], 0.0]),
    }
    for name, w in alternatives.items():
        q = w / w.sum()
        za = max(abs(_binomial_z(counts[k], n, q[k])) for k in range(3) if 0.0 < q[k] < 1.0)
        assert za > 10.0, (name, za)


def test_lethargy_gain_per_target_is_the_textbook_xi():
    prob = _mixture(PARTS)
    ns = oracle.scatter_stats(oracle.OracleProblem(prob), seed=32, first_pid=0, n=20_000)
    for k, (A, *_rest) in enumerate(PARTS):
        cnt, s = ns[k]
        mean, var = _xi_moments(A)
        se = math.sqrt(var / cnt)
        assert abs(s / cnt - mean) <= 3.0 * se, (A, s / cnt, mean, se)
        # another nuclide's mass ratio would be far off
        for B, *_r in PARTS:
            if B != A:
                assert abs(s / cnt - _xi_moments(B)[0]) > 10.0 * se, (A, B)
    # mixture mean lethargy gain per scattering: sum_k p_k xi_k
    ns_s = np.array([d * ss for _, _, ss, d in PARTS])
    p = ns_s / ns_s.sum()
    mix_mean = sum(p[k] * _xi_moments(A)[0] for k, (A, *_r) in enumerate(PARTS))
    n = ns[:, 0].sum()
    # variance of one draw from the mixture
    m2 = sum(p[k] * (_xi_moments(A)[1] + _xi_moments(A)[0] ** 2) for k, (A, *_r) in enumerate(PARTS))
    se = math.sqrt((m2 - mix_mean ** 2) / n)
    assert abs(ns[:, 1].sum() / n - mix_mean) <= 3.0 * se


def test_non_scattering_nuclide_is_never_the_target():
    """A nuclide with sigma_s = 0 between two scatterers: its running-sum term is
    zero, so it can never be the first to reach xi Sigma_s; the scatterers share
    the collisions in the ratio of N sigma_s."""
    parts = [(1.0, 0.5, 5.0, 0.004), (238.0, 50.0, 0.0, 0.0001), (56.0, 0.3, 2.0, 0.02)]
    prob = _mixture(parts)
    ns = oracle.scatter_stats(oracle.OracleProblem(prob), seed=33, first_pid=0, n=10_000)
    assert ns[1, 0] == 0.0 and ns[1, 1] == 0.0
    n = ns[:, 0].sum()
    p0 = 0.02 / (0.02 + 0.04)
    assert abs(_binomial_z(ns[0, 0], n, p0)) <= 3.0


def test_scatter_stats_do_not_change_the_run():
    """The statistics run tracks the same histories as orc_run: the scattering
    count equals the collision count less the absorptions."""
    prob = _mixture(PARTS)
    op = oracle.OracleProblem(prob)
    ns = oracle.scatter_stats(op, seed=34, first_pid=0, n=2000)
    r = oracle.run(op, 34, 0, 2000)
    absorbed = r.glob[oracle.G_ABSORB]
    assert ns[:, 0].sum() == r.glob[oracle.G_NCOLL] - absorbed
