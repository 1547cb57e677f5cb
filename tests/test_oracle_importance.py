"""Pins for the oracle's training-sample builder of the importance network.

* Pure absorber with a beam: the forward estimate of x-bin g is
  exp(-Sigma_t (L - x_g)) (x_g its left edge), so the targets are
  -Sigma_t (L - x_g) within the binomial error; the features are the bin
  centres, the weights the credit counts (no floor).
* Cells below the credit threshold or with empty sums give no sample, and the
  order is the cell order.
* The (y, z) replicas are uniform on [-1, 1].
"""
import numpy as np

import mcsynth
import oracle
from tests.stats import three_sigma


def _absorber(sigma=0.01):
    prob = mcsynth.slab_problem(sigma_t=(sigma,) * 3, thickness=(200.0 / 3,) * 3, scatter_ratio=(0.0,) * 3)
    prob.imp = mcsynth.ImportanceGrid(nx=20, ne=1, x0=0.0, x1=200.0)
    return prob


def test_absorber_targets_features_and_weights():
    sigma = 0.01
    r = oracle.run(oracle.OracleProblem(_absorber(sigma)), 3, 0, 200_000)
    num, den, cnt = r.imp
    X, T, W = oracle.importance_samples(num, den, cnt, 20, 1, 0.0, 200.0, 200.0, replicas=3, min_credits=10,
                                        rel_floor=0.0, seed=7)
    assert X.shape == (60, 4) and T.shape == (60,) and W.shape == (60,)
    centres = ((np.arange(20) + 0.5) * 10.0 / 200.0).astype(np.float32)
    assert np.array_equal(X[:, 0], np.repeat(centres, 3))
    assert np.all(X[:, 3] == np.float32(0.5))
    assert np.array_equal(W, np.repeat(cnt.astype(np.float32), 3))
    truth = np.exp(-sigma * (200.0 - np.arange(20) * 10.0))
    est = np.exp(T[::3].astype(np.float64))
    se = np.sqrt(truth * (1 - truth) / den)
    n_fail, allowed, z = three_sigma(est, se, truth=truth)
    assert n_fail <= allowed, (n_fail, allowed, z)
    assert np.all(np.abs(X[:, 1:3]) <= 1.0)
    assert len(set(map(tuple, X[:, 1:3].tolist()))) == 60


def test_threshold_and_empty_cells_are_skipped_in_cell_order():
    num = np.array([1.0, 2.0, 0.0, 3.0, 4.0, 5.0])
    den = np.array([2.0, 4.0, 1.0, 0.0, 8.0, 10.0])
    cnt = np.array([50.0, 5.0, 50.0, 50.0, 10.0, 11.0])
    X, T, W = oracle.importance_samples(num, den, cnt, 3, 2, 0.0, 30.0, 30.0, replicas=2, min_credits=10,
                                        rel_floor=0.5, seed=1)
    # kept: cells 0 (x 0, e 0), 4 (x 1, e 1), 5 (x 2, e 1)
    assert X.shape == (6, 4)
    assert np.array_equal(X[:, 0], np.float32([5, 5, 15, 15, 25, 25]) / np.float32(30.0))
    assert np.array_equal(X[:, 3], np.float32([0.25, 0.25, 0.75, 0.75, 0.75, 0.75]))
    np.testing.assert_allclose(T, np.log([0.5, 0.5, 0.5, 0.5, 0.5, 0.5]), rtol=1e-7)
    np.testing.assert_allclose(W, [1 / (1 / 50 + 0.25)] * 2 + [1 / (1 / 10 + 0.25)] * 2 + [1 / (1 / 11 + 0.25)] * 2,
                               rtol=1e-7)


def test_replicas_are_uniform_on_the_square():
    n = 400
    ones = np.ones(n)
    X, _, _ = oracle.importance_samples(ones, ones, 20 * ones, 20, 20, 0.0, 1.0, 1.0, replicas=5, min_credits=1,
                                        rel_floor=0.0, seed=11)
    yz = X[:, 1:3].astype(np.float64)
    m = yz.size
    # mean 0 and variance 1/3 of U(-1, 1); deciles within binomial error
    assert abs(yz.mean()) < 4 * np.sqrt(1 / 3 / m)
    assert abs((yz ** 2).mean() - 1 / 3) < 4 * np.sqrt(4 / 45 / m)
    for q in np.linspace(-0.8, 0.8, 9):
        p = (q + 1) / 2
        assert abs(np.mean(yz < q) - p) < 4 * np.sqrt(p * (1 - p) / m)
