"""Pins of the oracle's windowed-multipole cross sections (Doppler broadening
on the fly through the Faddeeva function).

* The Faddeeva function (a rational series) against scipy.special.wofz over
  the upper half plane.
* Zero-temperature limit: with T -> 0 every pole term tends to i / (u - p),
  so the broadened cross section tends to the plain rational function of u.
* Doppler broadening keeps each resonance's area in u: the integral over u
  of E * sigma_res is pi * r for a real residue r at every temperature, while
  the peak falls as T rises.
* The macroscopic value is the density-weighted sum of the nuclides'.
A wrong sqrt(pi) beta factor, a sign of the pole shift, a dropped 1/E or a
wrong window fails one of these.
"""
import numpy as np
import pytest
import scipy.special as sp

import mcsynth
import oracle

KB = 8.617333262e-5


def test_faddeeva_matches_wofz():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.uniform(-30, 30, 4000), np.sinh(rng.uniform(-9, 9, 2000))])
    y = np.concatenate([10 ** rng.uniform(-6, 2, 4000), 10 ** rng.uniform(-6, 4, 2000)])
    z = x + 1j * y
    w = oracle.faddeeva(z)
    ref = sp.wofz(z)
    rel = np.abs(w - ref) / np.abs(ref)
    assert np.max(rel) < 1e-10, np.max(rel)
    assert abs(oracle.faddeeva([0.5j])[0] - sp.erfcx(0.5)) < 1e-14


def _single_pole(e_r=100.0, gamma_e=1.0, h=1000.0, phase=0.0):
    a = np.sqrt(e_r)
    g = gamma_e / (4 * a)
    r = h * g * e_r * np.exp(1j * phase)
    return mcsynth.MultipoleNuclide(poles=np.array([a - 1j * g]), res_c=np.array([r]), res_s=np.array([0.5 * r]),
                                    u_lo=np.sqrt(mcsynth.EMIN), u_hi=np.sqrt(mcsynth.EMAX),
                                    win=np.array([[0, 1]], np.int32), bg_c=np.zeros((1, 3)),
                                    bg_s=np.array([[0.0, 3.0, 0.0]]), awr=56.0), a, g, r


def test_zero_temperature_limit():
    nd, a, g, r = _single_pole(phase=0.3)
    E = np.linspace(95.0, 105.0, 401)
    Sa, Ss = oracle.multipole_macro([nd], [0], [1.0], 1e-9, E)
    u = np.sqrt(E)
    plain = np.real(r * 1j / (u - (a - 1j * g))) / E
    np.testing.assert_allclose(Sa, plain, rtol=1e-6, atol=1e-9)
    np.testing.assert_allclose(Ss, 0.5 * plain + 3.0, rtol=1e-6, atol=1e-9)


@pytest.mark.parametrize("T", [300.0, 3000.0])
def test_broadening_keeps_resonance_area(T):
    nd, a, g, r = _single_pole()
    u = np.linspace(a - 3.0, a + 3.0, 600_001)
    Sa, _ = oracle.multipole_macro([nd], [0], [1.0], T, u ** 2)
    area = np.trapezoid(Sa * u ** 2, u)
    # the tails beyond +-3 in u hold r g (1/3 + 1/3) of the area (Lorentzian
    # wings, which broadening leaves in place to first order)
    deficit = np.pi * np.real(r) - area
    assert 0 < deficit <= 1.02 * 2 * g / 3 * np.real(r), (area, np.pi * r)
    peak_cold = oracle.multipole_macro([nd], [0], [1.0], 1.0, [a * a])[0][0]
    peak_hot = oracle.multipole_macro([nd], [0], [1.0], T, [a * a])[0][0]
    assert peak_hot < peak_cold


def test_macro_is_density_weighted_sum():
    nucs, ids, dens = mcsynth.multipole_material(n_nuclides=12, data_seed=5)
    rng = np.random.default_rng(8)
    E = mcsynth.lookup_energies(rng, 500)
    Sa, Ss = oracle.multipole_macro(nucs, ids, dens, 600.0, E)
    ra, rs = np.zeros_like(E), np.zeros_like(E)
    for q in range(12):
        a, s = oracle.multipole_macro(nucs, [q], [1.0], 600.0, E)
        ra += dens[q] * a
        rs += dens[q] * s
    np.testing.assert_allclose(Sa, ra, rtol=1e-12)
    np.testing.assert_allclose(Ss, rs, rtol=1e-12)
    assert np.all(Sa > 0) and np.all(Ss > 0)
