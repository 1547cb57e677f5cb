"""Pins for the oracle's collision kinematics and direction update (textbook
two-body elastic scattering off a target at rest)."""
import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("A", [1.0, 2.0, 12.0, 56.0, 238.0])
def test_elastic_energy_range_and_endpoints(A):
    alpha = ((A - 1) / (A + 1)) ** 2
    E = 1.0e6
    e_fwd, mu_fwd = oracle.elastic(A, E, 1.0)
    assert e_fwd == pytest.approx(E, rel=1e-15) and mu_fwd == pytest.approx(1.0, rel=1e-15)
    if A > 1:
        e_back, mu_back = oracle.elastic(A, E, -1.0)
        assert e_back == pytest.approx(alpha * E, rel=1e-13)
        assert mu_back == pytest.approx(-1.0, rel=1e-13)
    for mu in np.linspace(-1 + 1e-12, 1, 101):
        e, m = oracle.elastic(A, E, mu)
        assert alpha * E * (1 - 1e-14) <= e <= E * (1 + 1e-14)
        assert -1 - 1e-14 <= m <= 1 + 1e-14


@pytest.mark.parametrize("A", [1.0, 12.0, 238.0])
def test_elastic_means(A):
    """Isotropic in the centre of mass: E[E'/E] = (1 + alpha)/2 and the mean lab
    cosine is 2/(3A) (textbook results)."""
    alpha = ((A - 1) / (A + 1)) ** 2
    # Gauss-Legendre quadrature over mu_cm in [-1, 1] (uniform density 1/2)
    x, w = np.polynomial.legendre.leggauss(64)
    ratio = np.array([oracle.elastic(A, 1.0, m)[0] for m in x])
    mul = np.array([oracle.elastic(A, 1.0, m)[1] for m in x])
    assert np.sum(w * ratio) / 2 == pytest.approx((1 + alpha) / 2, rel=1e-12)
    # the lab cosine has a kink at A = 1 (mu_lab = sqrt((1+mu)/2)); use many points
    if A == 1.0:
        m = (np.arange(200000) + 0.5) / 100000 - 1
        mul = np.array([oracle.elastic(A, 1.0, v)[1] for v in m[::50]])
        assert mul.mean() == pytest.approx(2 / 3, rel=2e-3)
    else:
        assert np.sum(w * mul) / 2 == pytest.approx(2 / (3 * A), rel=1e-9)


def test_rotate_keeps_unit_norm_and_angle():
    rng = np.random.default_rng(11)
    for _ in range(500):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        if rng.uniform() < 0.1:
            d = np.array([0.0, 0.0, 1.0 if rng.uniform() < 0.5 else -1.0])
        mu = rng.uniform(-1, 1)
        phi = rng.uniform(0, 2 * np.pi)
        n = oracle.rotate(d, mu, phi)
        assert np.linalg.norm(n) == pytest.approx(1.0, abs=1e-12)
        assert np.dot(n, d) == pytest.approx(mu, abs=1e-12)


def test_rotate_azimuth_is_uniform():
    """For a fixed direction and mu, phi uniform spreads the new directions
    evenly around the old one: their mean is mu * d."""
    d = np.array([0.3, -0.4, np.sqrt(1 - 0.25)])
    mu = 0.2
    phis = (np.arange(720) + 0.5) * (2 * np.pi / 720)
    out = np.array([oracle.rotate(d, mu, p) for p in phis])
    np.testing.assert_allclose(out.mean(axis=0), mu * d, atol=1e-12)
