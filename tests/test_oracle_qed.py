"""Oracle pins for the QED pieces (Sect. 3; Sect. 4 radiation reaction)."""
import math

import numpy as np
import pytest
from scipy import integrate, special, stats

from oracle import oracle as O

ALPHA_EM = 1 / 137.035999084


# ---------------------------------------------------------------- rate fits
def test_tsyn_limit_and_slope():
    # Sect. 3.1: T_syn -> 5/(2 sqrt 3) for chi << 1 and the linear coefficient
    # reproduces T_syn = 5/(2 sqrt3) (1 - 8 sqrt3/15 chi) + O(chi^2).
    t0 = 5 / (2 * math.sqrt(3))
    assert math.isclose(O.tsyn(0.0), t0, rel_tol=1e-15)
    h = 1e-6
    slope = (O.tsyn(h) - O.tsyn(-h)) / (2 * h) / t0
    assert math.isclose(slope, -8 * math.sqrt(3) / 15, rel_tol=1e-6)
    # decreasing, and ~chi^(-1/3) at large chi (exponent of the fit: -2/6)
    assert O.tsyn(10) < O.tsyn(1) < O.tsyn(0.1)
    r = math.log(O.tsyn(1e6) / O.tsyn(1e5)) / math.log(10)
    assert math.isclose(r, -1 / 3, rel_tol=1e-4)


def test_tbw_asymptotes():
    # Sect. 3.2: T_BW -> 0.23 exp(-8/(3 chi)) for chi << 1 and -> 0.38 chi^(-1/3)
    # for chi >> 1; the fit's 0.22 ~ (0.23/0.38)^3 = 0.2217.
    for chi in (5e-3, 2e-2):
        assert math.isclose(O.tbw(chi) / (0.23 * math.exp(-8 / (3 * chi))), 1.0, rel_tol=2e-3)
    big = 1e7
    assert math.isclose(O.tbw(big) * big ** (1 / 3), 0.38, rel_tol=3e-3)
    assert abs((0.23 / 0.38) ** 3 - 0.22) < 2e-3
    assert O.tbw(0.0) == 0.0


# ------------------------------------------------------- synchrotron spectrum
def _cdf_scipy(xi):
    """C(xi) = int_0^xi F1, F1(t) = int_t^inf K_{5/3}: by parts,
    int_0^xi F1 = xi F1(xi) + int_0^xi t K_{5/3}(t) dt, normalised by 5 pi/3."""
    f1 = integrate.quad(lambda t: special.kv(5 / 3, t), xi, 1, limit=400)[0] + \
        integrate.quad(lambda t: special.kv(5 / 3, t), 1, np.inf, limit=400)[0] if xi < 1 else \
        integrate.quad(lambda t: special.kv(5 / 3, t), xi, np.inf, limit=400)[0]
    g = integrate.quad(lambda v: 3 * v ** 5 * special.kv(5 / 3, v ** 3), 0, xi ** (1 / 3), limit=400)[0]
    return (xi * f1 + g) * 3 / (5 * math.pi)


@pytest.mark.parametrize("xi", [1e-6, 1e-4, 1e-2, 0.3, 1.0, 3.0, 10.0])
def test_sync_cdf_matches_bessel_quadrature(xi):
    assert math.isclose(O.sync_cdf(xi), _cdf_scipy(xi), rel_tol=1e-9)


def test_sync_cdf_small_argument_asymptote():
    # dN/dxi ~ int_xi^inf K_{5/3} ~ (3/2) 2^(2/3) Gamma(5/3) xi^(-2/3) as xi -> 0,
    # so C(xi) -> (27/(20 pi)) 2^(5/3) Gamma(5/3) xi^(1/3).
    a = 27 / (20 * math.pi) * 2 ** (5 / 3) * special.gamma(5 / 3)
    for xi in (1e-15, 1e-12):
        assert math.isclose(O.sync_cdf(xi), a * xi ** (1 / 3), rel_tol=2e-3)


def test_sync_inverse_mean_and_roundtrip():
    # mean of the classical spectrum: Gamma(2/3)Gamma(7/3) / (5 pi/3) = 8/(15 sqrt 3)
    r = (np.arange(100000) + 0.5) / 100000
    x = O.sync_inverse(r)
    assert math.isclose(x.mean(), 8 / (15 * math.sqrt(3)), rel_tol=2e-4)
    for ri, xi in zip(r[::9973], x[::9973]):
        assert math.isclose(O.sync_cdf(xi), ri, rel_tol=1e-10)


# ---------------------------------------------------------- emission in PIC
def _frozen_beam(gamma, n, lam_scale, rc_scale, flags, steps, N=64):
    """n electrons at fixed gamma moving up in zero field (periodic, frozen)."""
    cfg = dict(n_cells=N, init_kind=2, b=0.1, r_curv_cm=1e7, lambda_c_scale=lam_scale, r_curv_scale=rc_scale,
               h_gap_frac=1.0, flags=flags, seed=11)
    o = O.Oracle(cfg)
    u = math.sqrt(gamma ** 2 - 1)
    rng = np.random.default_rng(5)
    lep = dict(cell=rng.integers(0, N, n), xi=rng.random(n), u=np.full(n, u), w=np.full(n, -1.0),
               id=np.arange(1, n + 1, dtype=np.uint64))
    o.set_state(lep)
    o.set_field(np.zeros(N), 0.0)
    o.step(steps)
    return o


def test_emission_rate_and_curvature_power():
    # Sect. 3.1: photon rate alpha_em gamma/R~ T_syn(chi) per particle (eq. tau_syn
    # with b sin psi = gamma lambda_C/R_curv) and, for chi << 1, mean radiated
    # power (2/3) alpha_em lambda~ gamma^4 / R~^2 (eq. P_curv).
    F = O.FLAGS
    flags = F["FIELD_FROZEN"] | F["PERIODIC"] | F["RECOIL_OFF"] | F["CONV_OFF"] | F["TRACK_ALL"]
    gamma, n, steps = 300.0, 4000, 40
    o = _frozen_beam(gamma, n, 1.7e5, 1.4e-5, flags, steps)
    lr = o.lam / o.rc
    chi = gamma ** 2 * lr
    assert chi < 0.01
    c = o.counts()
    dtau = ALPHA_EM * gamma / o.rc * O.tsyn(chi) * o.dt
    expected = n * steps * (-math.expm1(-dtau))
    assert abs(c["n_emit"] - expected) < 3.5 * math.sqrt(expected)
    # power: e_rad / (n t) vs (2/3) alpha_em lam gamma^4 / R^2, corrected by T_syn(chi)/T_syn(0)
    p_meas = o.e_rad / (n * steps * o.dt)
    p_curv = 2 / 3 * ALPHA_EM * o.lam * gamma ** 4 / o.rc ** 2 * O.tsyn(chi) / O.tsyn(0.0)
    # relative spread of the estimator: sqrt(<x^2>)/<x> / sqrt(N_events)
    rel = math.sqrt(1 + 1.0) / math.sqrt(c["n_emit"])
    assert abs(p_meas / p_curv - 1) < 3.5 * rel


def test_emitted_spectrum_ks():
    F = O.FLAGS
    flags = F["FIELD_FROZEN"] | F["PERIODIC"] | F["RECOIL_OFF"] | F["CONV_OFF"] | F["TRACK_ALL"]
    gamma = 300.0
    o = _frozen_beam(gamma, 3000, 1.7e5, 1.4e-5, flags, 200)
    ph = o.photons()
    xc = 1.5 * gamma ** 3 * o.lam / o.rc
    xi = np.abs(ph["x"]) / xc
    assert xi.size > 500
    grid = np.logspace(-8, 1.6, 400)
    cdf = np.array([O.sync_cdf(g) for g in grid])
    res = stats.kstest(xi, lambda q: np.interp(np.log(q), np.log(grid), cdf))
    assert res.pvalue > 0.01


def test_radiation_reaction_equilibrium():
    # Sect. 4 eq. gam_rad: acceleration balances curvature drag at
    # gamma_rad = (3 E R~^2 / (2 alpha_em lambda~))^(1/4) (chi << 1 here).
    F = O.FLAGS
    N, E0 = 256, 100.0
    cfg = dict(n_cells=N, init_kind=2, b=0.1, r_curv_cm=1e7, lambda_c_scale=350.0, r_curv_scale=1.4e-5,
               h_gap_frac=1.0, flags=F["FIELD_FROZEN"] | F["PERIODIC"] | F["CONV_OFF"], seed=3)
    o = O.Oracle(cfg)
    n = 200
    rng = np.random.default_rng(1)
    lep = dict(cell=rng.integers(0, N, n), xi=rng.random(n), u=np.zeros(n), w=np.full(n, 1.0),
               id=np.arange(1, n + 1, dtype=np.uint64))
    o.set_state(lep)
    o.set_field(np.full(N, E0), E0)
    g_rad = (3 * E0 * o.rc ** 2 / (2 * ALPHA_EM * o.lam)) ** 0.25
    chi = g_rad ** 2 * o.lam / o.rc
    assert chi < 0.02
    steps_to_eq = int(3 * g_rad / E0 / o.dt)
    o.step(steps_to_eq)
    gs = []
    for _ in range(10):
        o.step(50)
        u = o.leptons()["u"]
        gs.append(np.sqrt(1 + u ** 2).mean())
    g_eq = float(np.mean(gs))
    # the quantum-suppressed rate T_syn(chi)/T_syn(0) raises the balance point by (T0/T)^(1/4)
    corr = (O.tsyn(0.0) / O.tsyn(chi)) ** 0.25
    assert abs(g_eq / (g_rad * corr) - 1) < 0.03


# ---------------------------------------------------------- pair conversion
def test_conversion_distance_distribution_and_mfp():
    # Photons born along B at n0 = 0 with fixed energy x: conversion rate
    # alpha_em (b/lambda~) sin(psi) T_BW(x b sin psi), sin psi = |sin(s/R~)|.
    F = O.FLAGS
    N = 8192
    cfg = dict(n_cells=N, init_kind=2, b=0.1, r_curv_cm=1e7, lambda_c_scale=1.7e5, r_curv_scale=1.4e-5,
               h_gap_frac=1.0, flags=F["FIELD_FROZEN"] | F["EMIT_OFF"] | F["RECORD"], seed=9)
    o = O.Oracle(cfg)
    n, x = 3000, 200.0
    pho = dict(cell=np.zeros(n, np.int32), xi=np.full(n, 0.0), x=np.full(n, x), w=np.ones(n),
               n0=np.zeros(n, np.int64), id=np.arange(1, n + 1, dtype=np.uint64))
    o.set_state(dict(cell=[], xi=[], u=[], w=[], id=[]), pho)
    o.set_field(np.zeros(N), 0.0)
    steps = 1500
    o.step(steps)
    ev = o.events()
    conv_steps = ev["step"][ev["kind"] == 1]
    # survival by brute-force accumulation of the per-step hazard
    haz = []
    for m in range(steps):
        s = (m + 1) * o.dt
        sp = abs(math.sin(s / o.rc))
        chi = x * 0.1 * sp
        haz.append(ALPHA_EM * (0.1 / o.lam) * sp * O.tbw(chi) * o.dt)
    p_conv = -np.expm1(-np.array(haz))
    surv = np.concatenate([[1.0], np.cumprod(1 - p_conv)])
    cdf = 1 - surv[1:]
    emp = np.array([(conv_steps <= m).sum() for m in range(steps)]) / n
    # one-sample KS distance with the discrete CDF
    assert np.max(np.abs(emp - cdf)) < 1.63 / math.sqrt(n)
    # Sect. 3.2 eq. lmfp_pair (Lambert-W estimate, chi << 1): within a factor 2
    lam_c, b = o.lam, 0.1
    z = 0.4 * (lam_c * x ** 2 * b / (ALPHA_EM * o.rc)) ** (-1 / 3)
    l_est = 8 / 9 * o.rc / (x * b) / special.lambertw(z).real
    median = np.median(conv_steps + 1) * o.dt
    assert 0.5 < median / l_est < 2.0
