"""Pins for the oracle's cross-section lookup: grid index by brute force and by
numpy's searchsorted, interpolation by numpy.interp and on linear data, the
macroscopic sum by its error bound."""
import numpy as np
import pytest

import mcsynth
import oracle


def brute_index(grid, e):
    """Linear scan: the largest j with grid[j] <= e, clamped to [0, N-2]."""
    j = -1
    for k, g in enumerate(grid):
        if g <= e:
            j = k
    return min(max(j, 0), len(grid) - 2)


@pytest.mark.parametrize("n", [2, 3, 5, 17, 64])
def test_grid_index_brute_force_tiny(n):
    rng = np.random.default_rng(n)
    for _ in range(20):
        grid = np.sort(rng.uniform(0, 10, n))
        grid = np.unique(grid)
        if grid.size < 2:
            continue
        qs = np.concatenate([grid, np.nextafter(grid, -np.inf), np.nextafter(grid, np.inf),
                             rng.uniform(-1, 11, 50), [grid[0] - 1, grid[-1] + 1]])
        for e in qs:
            assert oracle.grid_index(grid, e) == brute_index(grid, e)


def test_grid_index_matches_searchsorted_on_real_grids():
    p = mcsynth.c2_problem(grid_range=(10_000, 12_000))
    rng = np.random.default_rng(0)
    for nuc in p.nuclides[:5]:
        qs = mcsynth.edge_case_energies(nuc, rng, 2000)[::7]
        ref = np.clip(np.searchsorted(nuc.E, qs, side="right") - 1, 0, nuc.E.size - 2)
        got = np.array([oracle.grid_index(nuc.E, e) for e in qs])
        assert np.array_equal(got, ref)


def _single_nuclide_problem(nuc):
    mat = mcsynth.Material(nuclides=np.array([0], np.int32), densities=np.array([1.0]))
    return mcsynth.Problem("one", [nuc], [mat], mcsynth.Geometry(), mcsynth.Source(),
                           mcsynth.Tally(mcsynth.TALLY_ENERGY, mcsynth.energy_edges(4)))


def test_micro_xs_exact_at_grid_points():
    rng = np.random.default_rng(1)
    nuc = mcsynth.make_nuclide(rng, 12.0, 2000)
    op = oracle.OracleProblem(_single_nuclide_problem(nuc))
    idx, sc, ss = oracle.micro_xs(op, 0, nuc.E[:-1])
    assert np.array_equal(idx, np.arange(nuc.E.size - 1))
    assert np.array_equal(sc, nuc.sig_c[:-1]) and np.array_equal(ss, nuc.sig_s[:-1])
    # the last grid point maps to the last interval with f = 1 exactly
    idx, sc, ss = oracle.micro_xs(op, 0, [nuc.E[-1]])
    assert idx[0] == nuc.E.size - 2 and sc[0] == nuc.sig_c[-1] and ss[0] == nuc.sig_s[-1]


def test_micro_xs_reproduces_linear_data():
    """sigma = alpha E + beta is reproduced by the interpolation to rounding."""
    E = mcsynth.log_uniform_grid(300)
    alpha, beta = 3.0e-6, 7.25
    nuc = mcsynth.Nuclide(E=E, sig_c=alpha * E + beta, sig_s=2 * alpha * E + 1.0, awr=1.0)
    op = oracle.OracleProblem(_single_nuclide_problem(nuc))
    q = mcsynth.lookup_energies(np.random.default_rng(2), 3000)
    _, sc, ss = oracle.micro_xs(op, 0, q)
    np.testing.assert_allclose(sc, alpha * q + beta, rtol=1e-13)
    np.testing.assert_allclose(ss, 2 * alpha * q + 1.0, rtol=1e-13)


def test_micro_xs_matches_numpy_interp_within_lerp_bound():
    rng = np.random.default_rng(3)
    nuc = mcsynth.make_nuclide(rng, 56.0, 5000, "clustered")
    op = oracle.OracleProblem(_single_nuclide_problem(nuc))
    q = mcsynth.edge_case_energies(nuc, rng, 3000)[::5]
    idx, sc, ss = oracle.micro_xs(op, 0, q)
    for tab, got in ((nuc.sig_c, sc), (nuc.sig_s, ss)):
        ref = np.interp(q, nuc.E, tab)
        scale = np.maximum(np.abs(tab[idx]), np.abs(tab[idx + 1]))
        assert np.all(np.abs(got - ref) <= 8 * np.finfo(float).eps * scale)


def test_macro_sum_within_positive_sum_bound():
    """All terms are >= 0, so any summation order is within (n-1) 2^-53 relative
    (plus the interpolation bound per term); numpy.interp gives each term."""
    p = mcsynth.c2_problem(grid_range=(10_000, 12_000))
    op = oracle.OracleProblem(p)
    rng = np.random.default_rng(4)
    q = mcsynth.lookup_energies(rng, 200)
    for m, mat in enumerate(p.materials):
        Sa, Ss = oracle.macro_xs(op, m, q)
        refa = sum(d * np.interp(q, p.nuclides[k].E, p.nuclides[k].sig_c)
                   for k, d in zip(mat.nuclides, mat.densities))
        refs = sum(d * np.interp(q, p.nuclides[k].E, p.nuclides[k].sig_s)
                   for k, d in zip(mat.nuclides, mat.densities))
        # bound: per-term lerp error (relative to the bracketing values) + summation
        bounda = sum(d * np.maximum(p.nuclides[k].sig_c[np.searchsorted(p.nuclides[k].E, q) - 1],
                                    p.nuclides[k].sig_c[np.searchsorted(p.nuclides[k].E, q)])
                     for k, d in zip(mat.nuclides, mat.densities))
        n = mat.nuclides.size
        assert np.all(np.abs(Sa - refa) <= (8 + n) * np.finfo(float).eps * bounda + 1e-300)
        np.testing.assert_allclose(Ss, refs, rtol=1e-12)


def test_macro_constant_xs_is_exact():
    nuc = mcsynth.constant_nuclide(0.5, 4.0, 1.0)
    mat = mcsynth.Material(nuclides=np.array([0], np.int32), densities=np.array([0.25]))
    p = mcsynth.Problem("c", [nuc], [mat], mcsynth.Geometry(), mcsynth.Source(),
                        mcsynth.Tally(mcsynth.TALLY_ENERGY, mcsynth.energy_edges(4)))
    op = oracle.OracleProblem(p)
    Sa, Ss = oracle.macro_xs(op, 0, mcsynth.lookup_energies(np.random.default_rng(5), 100))
    assert np.all(Sa == 0.125) and np.all(Ss == 1.0)
