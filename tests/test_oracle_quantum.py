"""Pins of the oracle's quantum-corrected spectra (Sect. 3.1: the photon
spectrum S(gamma, x), the rate function T_syn and the Gaunt factor g_Q of
P_syn; Sect. 3.2: the pair creation rate T_BW and the energy split of the
pair) against what the paper and the mathematics fix:

* the classical limit chi -> 0 (T_syn -> 5/(2 sqrt3); the spectrum becomes
  the classical synchrotron spectrum of the default sampler);
* the exact first-order expansion the paper quotes, T_syn = 5/(2 sqrt3)
  (1 - 8 sqrt3/15 chi), and the textbook one of the radiated power,
  g_Q = 1 - 55 sqrt3/16 chi;
* the paper's claim that its T_syn fit holds to ~1 % for chi <~ 30 and its
  T_BW fit to ~10 % for chi <~ 100;
* the two asymptotes of T_BW the paper quotes: 0.23 exp(-8/(3 chi)) (with
  the exact constant 3 sqrt3/(16 sqrt2)) and 0.38 chi^(-1/3);
* the small-chi pair split: the electron fraction is Gaussian about 1/2 with
  variance 3 chi/64 (the exponent 2/(3 chi v(1-v)) expanded about v = 1/2);
* the inverse distribution functions invert the distribution functions, and
  their means reproduce the Gaunt factor through <x>/gamma = 2/3 chi g_Q/T_syn.
"""
import math

import numpy as np

from oracle import oracle as O

T0 = 5.0 / (2.0 * math.sqrt(3.0))


def test_emission_rate_classical_limit_and_first_order():
    assert abs(O.qsyn_T(1e-7) / T0 - 1.0) < 2e-7
    chi = 1e-5
    slope = (O.qsyn_T(chi) - T0) / chi
    assert abs(slope / (-4.0 / 3.0) - 1.0) < 1e-3          # T0 * 8 sqrt3/15 = 4/3


def test_emission_rate_matches_the_paper_fit():
    for chi in np.logspace(-3, math.log10(30.0), 16):
        assert abs(O.tsyn(chi) / O.qsyn_T(chi) - 1.0) < 0.01, chi


def test_gaunt_factor_limit_first_order_and_monotone():
    assert abs(O.qsyn_g(1e-7) - 1.0) < 1e-6
    chi = 1e-5
    slope = (O.qsyn_g(chi) - 1.0) / chi
    assert abs(slope / (-55.0 * math.sqrt(3.0) / 16.0) - 1.0) < 2e-3
    g = [O.qsyn_g(c) for c in np.logspace(-3, 2, 11)]
    assert all(0.0 < b < a <= 1.0 for a, b in zip(g, g[1:]))


def test_photon_spectrum_classical_limit():
    chi = 1e-7
    for xi in (1e-3, 0.05, 0.3, 1.0, 2.5, 6.0):
        d = 1.5 * chi * xi / (1.0 + 1.5 * chi * xi)           # x = xi x_c, x_c = 3/2 gamma chi
        assert abs(O.qsyn_cdf(chi, d)[0] - O.sync_cdf(xi)) < 1e-6, xi


def test_photon_inverse_inverts_and_mean_matches_gaunt():
    for chi in (0.05, 1.0, 20.0):
        r = np.array([1e-6, 0.01, 0.3, 0.5, 0.77, 0.99, 1 - 1e-6])
        d = O.qsyn_inverse(chi, r)
        assert np.all(np.diff(d) > 0) and np.all((d > 0) & (d < 1))
        assert np.allclose(O.qsyn_cdf(chi, d), r, rtol=1e-9, atol=1e-12)
        # <d> by midpoint strata of r; compare 2/3 chi g_Q / T_syn
        m = 400
        mean = O.qsyn_inverse(chi, (np.arange(m) + 0.5) / m).mean()
        assert abs(mean / (2.0 / 3.0 * chi * O.qsyn_g(chi) / O.qsyn_T(chi)) - 1.0) < 5e-3, chi


def test_pair_rate_asymptotes_and_the_paper_fit():
    erber = 3.0 * math.sqrt(3.0) / (16.0 * math.sqrt(2.0))
    chi = 0.005
    assert abs(O.qbw_T(chi) / math.exp(-8.0 / (3.0 * chi)) / erber - 1.0) < 2e-3
    assert abs(O.qbw_T(1e4) * 1e4 ** (1.0 / 3.0) / 0.38 - 1.0) < 0.01
    for chi in np.logspace(-1.5, 2, 15):
        assert abs(O.tbw(chi) / O.qbw_T(chi) - 1.0) < 0.11, chi


def test_pair_split_small_chi_width_and_symmetry():
    chi = 0.01
    m = 600
    r = (np.arange(m) + 0.5) / m
    v = O.qbw_inverse(chi, r)
    assert np.allclose(v + v[::-1], 1.0, atol=1e-12)
    var = ((v - 0.5) ** 2).mean()
    assert abs(var / (3.0 * chi / 64.0) - 1.0) < 0.03
    for c in (0.3, 3.0):
        rr = np.array([1e-4, 0.1, 0.35, 0.6, 0.95])
        vv = O.qbw_inverse(c, rr)
        assert np.all(np.diff(vv) > 0)
        assert np.allclose(O.qbw_cdf(c, vv), rr, rtol=1e-9, atol=1e-12)
