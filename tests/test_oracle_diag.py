"""Pins of the oracle's discharge diagnostics (oracle/diag.py and the return
flux of oracle.c) against what their definitions fix (Sect. 5, Figs. 3, 5, 7):
brute force over small states, closed forms for uniform and mono-energetic
plasmas, and a return flux whose every absorbed lepton is known."""
import math

import numpy as np

from oracle import diag
from oracle.oracle import Oracle, FLAGS as OF


def _brute(lep, pho, N, B):
    nb = (N + B - 1) // B
    acc = [[[0.0] * 3 for _ in range(6)] for _ in range(nb)]
    for c, u, w in zip(lep["cell"], lep["u"], lep["w"]):
        if w == 0.0:
            continue
        b = min(max(int(c), 0), N - 1) // B
        grp = (0 if w < 0 else 2) + (0 if u > 0 else 1)
        g = math.sqrt(1.0 + u * u)
        acc[b][grp][0] += abs(w)
        acc[b][grp][1] += abs(w) * g
        acc[b][grp][2] += abs(w) / g ** 3
    for c, x, w in zip(pho["cell"], pho["x"], pho["w"]):
        if x == 0.0 or abs(x) <= 2.0:
            continue
        b = min(max(int(c), 0), N - 1) // B
        grp = 4 if x > 0 else 5
        acc[b][grp][0] += w
        acc[b][grp][1] += w * abs(x)
    return np.array(acc)


def _state(rng, nl, npho, N):
    lep = dict(cell=rng.integers(0, N, nl), u=rng.normal(0, 30, nl) * (rng.random(nl) < 0.9),
               w=rng.choice([-2.0, -1.0, 0.0, 1.0, 0.5], nl))
    pho = dict(cell=rng.integers(0, N, npho), x=rng.choice([-1, 1], npho) * 10 ** rng.uniform(-1, 4, npho),
               w=rng.choice([1.0, 2.0], npho))
    pho["x"][::17] = 0.0
    return lep, pho


def test_profile_sums_equal_brute_force():
    rng = np.random.default_rng(3)
    N, B = 300, 32   # a ragged last bin
    lep, pho = _state(rng, 2000, 700, N)
    got = diag.profile_sums(lep, pho, N, B)
    ref = _brute(lep, pho, N, B)
    assert got.shape == (10, 6, 3)
    assert np.allclose(got, ref, rtol=1e-13, atol=0.0)


def test_uniform_cold_plasma_closed_form():
    # ppc_ref electrons and positrons of unit weight at rest in every cell:
    # multiplicity 1 per species (u = 0 counts as moving down), gamma 1
    N, B, ppc = 256, 64, 8
    cell = np.repeat(np.arange(N), 2 * ppc)
    w = np.tile(np.r_[-np.ones(ppc), np.ones(ppc)], N)
    lep = dict(cell=cell, u=np.zeros(cell.size), w=w)
    pho = dict(cell=np.zeros(0, int), x=np.zeros(0), w=np.zeros(0))
    p = diag.profile(diag.profile_sums(lep, pho, N, B), B, ppc)
    assert np.array_equal(p[:, 1, 0], np.ones(4)) and np.array_equal(p[:, 3, 0], np.ones(4))
    assert np.array_equal(p[:, 0, 0], np.zeros(4)) and np.array_equal(p[:, 2, 0], np.zeros(4))
    assert np.array_equal(p[:, 1, 1], np.ones(4)) and np.array_equal(p[:, 1, 2], np.ones(4))


def test_monoenergetic_beam_moments():
    # one gamma for every lepton: <gamma> = gamma, <gamma^-3> = gamma^-3
    gam = 1234.5
    u = math.sqrt(gam * gam - 1.0)
    N, B, ppc = 128, 16, 4
    lep = dict(cell=np.arange(N), u=np.full(N, u), w=np.full(N, 3.0))
    pho = dict(cell=np.zeros(0, int), x=np.zeros(0), w=np.zeros(0))
    p = diag.profile(diag.profile_sums(lep, pho, N, B), B, ppc)
    assert np.allclose(p[:, 2, 0], 3.0 * 16 / (16 * 4), rtol=0, atol=0)
    assert np.allclose(p[:, 2, 1], gam, rtol=1e-14)
    assert np.allclose(p[:, 2, 2], gam ** -3, rtol=1e-12)


def test_peak_in_zone_and_field_extremes():
    N, B, ppc, dx = 512, 32, 4, 0.25
    H = 0.5 * N * dx                        # zone: bins 0..7 (centres below H)
    cell = np.r_[np.arange(N), np.full(50, 5 * B + 3), np.full(80, 12 * B)]   # bump in bin 5, a bigger one above H
    u = np.r_[np.full(N, 10.0), np.full(50, -2.0), np.full(80, 1.0)]
    w = np.r_[np.ones(N), -np.ones(50), np.ones(80)]
    lep = dict(cell=cell, u=u, w=w)
    pho = dict(cell=np.array([5 * B + 1, 5 * B + 2, 6 * B]), x=np.array([5.0, -300.0, 7.0]), w=np.array([1.0, 2.0, 4.0]))
    E = np.sin(np.arange(N) * 0.1)
    pk = diag.peak(diag.profile_sums(lep, pho, N, B), E, B, dx, H, ppc)
    assert pk["h"] == (5 + 0.5) * B * dx
    assert pk["m_pairs"] == (B + 50) / (B * ppc)
    g_fast, g_slow = math.sqrt(101.0), math.sqrt(5.0)
    assert math.isclose(pk["g3"], (B * g_fast ** -3 + 50 * g_slow ** -3) / (B + 50), rel_tol=1e-13)
    assert pk["m_photons"] == 3.0 / (B * ppc)
    assert pk["e_min"] == np.min(E) and pk["e_max"] == np.max(E)


def test_return_flux_of_known_absorptions():
    # leptons in cell 0 moving down fast enough to cross h = 0 in one step
    # (|beta| 0.45 > xi), zero field: every one is absorbed in step 1 with its
    # initial momentum, so the flux is fixed by their gammas and weights
    N = 256
    cfg = dict(n_cells=N, init_kind=2, alpha=0.0, flags=OF["FIELD_FROZEN"] | OF["QED_OFF"], seed=1,
               ppc_ref=4, inj_rate=0.0)
    o = Oracle(cfg)
    gam = np.array([1.5, 10 ** 1.31, 10 ** 2.06, 10 ** 4.44, 10 ** 7.93, 10 ** 8.6])
    u = -np.sqrt(gam ** 2 - 1.0)
    w = np.array([-1.0, 1.0, -2.0, 0.5, -1.0, 3.0])
    lep = dict(cell=np.zeros(6, np.int32), xi=np.full(6, 0.1), u=u, w=w, id=np.arange(1, 7, dtype=np.uint64))
    o.set_state(lep, None, 0.0, 0)
    o.set_field(np.zeros(N), 0.0)
    o.step(1)
    assert o.counts()["n_absorbed"] == 6
    r = o.return_spectrum()
    ref = np.zeros(66)
    for gi, wi in zip(gam, w):
        ref[min(int(math.floor(8 * math.log10(gi))), 63)] += abs(wi)
    ref[64] = np.abs(w).sum()
    ref[65] = float((np.abs(w) * gam).sum())
    assert np.array_equal(r[:64], ref[:64])
    assert r[64] == ref[64] and math.isclose(r[65], ref[65], rel_tol=1e-14)
    assert np.array_equal(o.return_spectrum(), np.zeros(66))   # reading cleared it


def test_waterfall_row_constant_and_linear_fields():
    # constant E: every bin holds E0^2; E = cell index k: the mean of k^2 over
    # k0 .. k1-1 is (S(k1-1) - S(k0-1)) / (k1 - k0) with S(n) = n(n+1)(2n+1)/6
    N, B = 300, 64                           # bins of 64, 64, 64, 64, 44 cells
    assert np.array_equal(diag.waterfall_row(np.full(N, -2.5), B), np.full(5, 6.25))
    S = lambda n: n * (n + 1) * (2 * n + 1) / 6.0
    ref = []
    for b in range(5):
        k0, k1 = b * B, min(N, (b + 1) * B)
        ref.append((S(k1 - 1) - S(k0 - 1)) / (k1 - k0))
    assert np.allclose(diag.waterfall_row(np.arange(N, dtype=np.float64), B), ref, rtol=1e-15, atol=0.0)


def test_waterfall_row_brute_force_ragged():
    rng = np.random.default_rng(11)
    E = rng.normal(0, 50, 1000).astype(np.float32)
    for B in (1, 7, 37, 1000, 4096):
        nb = (E.size + B - 1) // B
        ref = [sum(float(e) * float(e) for e in E[b * B:(b + 1) * B]) / len(E[b * B:(b + 1) * B]) for b in range(nb)]
        assert np.allclose(diag.waterfall_row(E, B), ref, rtol=1e-13, atol=0.0)


def test_e_power_spectrum_closed_forms():
    # a cosine of integer mode m on M = N cells puts A^2 M / 4 into bin m and
    # nothing elsewhere; a constant puts A^2 M into bin 0; Parseval holds for
    # any field, also zero-padded (N = 1000 -> M = 1024)
    M, m, A = 1024, 37, 3.0
    j = np.arange(M)
    P = diag.e_power_spectrum(A * np.cos(2 * np.pi * m * j / M))
    assert P.shape == (M // 2 + 1,)
    ref = np.zeros(M // 2 + 1)
    ref[m] = A * A * M / 4
    assert np.allclose(P, ref, rtol=1e-12, atol=1e-9)
    P0 = diag.e_power_spectrum(np.full(M, A))
    assert math.isclose(P0[0], A * A * M, rel_tol=1e-14) and np.max(np.abs(P0[1:])) < 1e-12
    rng = np.random.default_rng(4)
    E = rng.normal(0, 2, 1000)
    P = diag.e_power_spectrum(E)
    full = np.r_[P, P[1:-1][::-1]]                       # the mirrored half of a real field
    assert math.isclose(full.sum(), float((E * E).sum()), rel_tol=1e-12)
    # brute-force DFT of the padded field at a few wavenumbers
    x = np.r_[E, np.zeros(24)]
    for k in (0, 1, 77, 512):
        X = sum(x[i] * complex(math.cos(2 * math.pi * i * k / 1024), -math.sin(2 * math.pi * i * k / 1024))
                for i in range(1024))
        assert math.isclose(P[k], abs(X) ** 2 / 1024, rel_tol=1e-9)


def test_spectra_bins_beam_and_brute_force():
    thr = diag.spectrum_edges_sq()
    assert thr.size == 89 and math.isclose(thr[0], 1e-4) and math.isclose(thr[-1], 1e18, rel_tol=1e-15)
    # a mono-energetic beam: all weight in the bin of its |u|, by species
    g = 1234.5
    u = math.sqrt(g * g - 1)
    b = int(math.floor(8 * (math.log10(u) + 2))) + 1
    lep = dict(u=np.r_[np.full(10, u), np.full(4, -u)], w=np.r_[-np.ones(10), 2 * np.ones(4)])
    pho = dict(x=np.array([0.0, 5.0, -5.0]), w=np.array([7.0, 1.0, 3.0]))
    S = diag.spectra(lep, pho)
    assert S[0, b] == 10 and S[1, b] == 8 and S[0].sum() == 10 and S[1].sum() == 8
    bx = int(math.floor(8 * (math.log10(5.0) + 2))) + 1
    assert S[2, bx] == 4 and S[2].sum() == 4
    # edges: a value whose square is an edge goes up; below 1e-2 and above 1e9
    # go to the end bins
    rng = np.random.default_rng(8)
    uu = np.r_[0.0, 1e-3, 10 ** rng.uniform(-3, 10, 500), 2e9]
    ww = rng.choice([-1.0, 1.0, 0.5], uu.size)
    S = diag.spectra(dict(u=uu, w=ww), None)
    ref = np.zeros((3, 90))
    for ui, wi in zip(uu, ww):
        k = sum(1 for t in thr if ui * ui >= t)
        ref[0 if wi < 0 else 1, k] += abs(wi)
    assert np.array_equal(S, ref)
    assert S[:, 0].sum() == sum(abs(w) for x, w in zip(uu, ww) if x < 1e-2)


def test_phase_space_brute_force_and_marginals():
    rng = np.random.default_rng(9)
    N, B = 300, 32
    lep, pho = _state(rng, 1500, 600, N)
    ph = diag.phase_space(lep, pho, N, B)
    assert ph.shape == (3, 10, 180)
    thr = diag.spectrum_edges_sq()
    ref = np.zeros_like(ph)
    for c, u, w in zip(lep["cell"], lep["u"], lep["w"]):
        if w == 0.0:
            continue
        b = sum(1 for t in thr if u * u >= t)
        ref[0 if w < 0 else 1, min(max(int(c), 0), N - 1) // B, 90 + b if u > 0 else 89 - b] += abs(w)
    for c, x, w in zip(pho["cell"], pho["x"], pho["w"]):
        if x == 0.0:
            continue
        b = sum(1 for t in thr if x * x >= t)
        ref[2, min(max(int(c), 0), N - 1) // B, 90 + b if x > 0 else 89 - b] += w
    assert np.allclose(ph, ref, rtol=1e-14, atol=0.0)
    # marginals: over momentum it is the profile's weight per bin and species
    # (photons: all, not only |x| > 2); over space, the |p| spectrum folded
    S = diag.spectra(lep, pho)
    folded = ph.sum(axis=1)[:, 90:] + ph.sum(axis=1)[:, 89::-1]
    assert np.allclose(folded, S, rtol=1e-13, atol=0.0)
    prof = diag.profile_sums(lep, None, N, B)
    assert np.allclose(ph[0].sum(axis=1), prof[:, 0, 0] + prof[:, 1, 0], rtol=1e-13)
    assert np.allclose(ph[1].sum(axis=1), prof[:, 2, 0] + prof[:, 3, 0], rtol=1e-13)
