"""Discharge diagnostics of the HIP path (profile, peak, return flux; Sect. 5,
Figs. 3, 5, 7) against the oracle's definitions on identical states."""
import math
import sys

import numpy as np
import pytest

from paper_2608_21920_amd import Gap, workloads
from paper_2608_21920_amd import gap as G
from paper_2608_21920_amd.inputs import LEPTON_DTYPE, leptons_as_oracle, photons_as_oracle
from oracle import diag
from oracle.oracle import Oracle, FLAGS as OF

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def grown(torch_gpu):
    cfg = dict(workloads.TINY)
    g = Gap(cfg)
    g.step(300)
    assert g.counts()["n_pho"] > 0
    yield g, cfg
    g.close()


@pytest.mark.parametrize("bin_cells", [64, 37, 1])
def test_profile_and_peak_match_oracle(grown, bin_cells):
    g, cfg = grown
    _say("case: profile and peak of the tiny gap at step 300, bins of %d cells" % bin_cells)
    g.set_profile_bin(bin_cells)
    L, P = leptons_as_oracle(g.leptons()), photons_as_oracle(g.photons())
    N, ppc = cfg["n_cells"], int(cfg.get("ppc_ref", 16))
    d = g.derived()
    sums = diag.profile_sums(L, P, N, bin_cells)
    ref = diag.profile(sums, bin_cells, ppc)
    got = g.profile()
    assert got.shape == ref.shape
    assert np.array_equal(got[:, :, 0], ref[:, :, 0])          # sums of weights: exact in FP64
    assert np.allclose(got[:, :, 1:], ref[:, :, 1:], rtol=1e-12, atol=0.0)
    pk, rp = g.peak(), diag.peak(sums, g.field().astype(np.float64), bin_cells, cfg.get("dx", 0.25), d["H"], ppc)
    _say("  peak m = %.4g at h = %.4g, <gamma^-3> = %.4g" % (pk["m_pairs"], pk["h"], pk["g3"]))
    assert pk["h"] == rp["h"] and pk["m_pairs"] == rp["m_pairs"] and pk["m_photons"] == rp["m_photons"]
    assert math.isclose(pk["g3"], rp["g3"], rel_tol=1e-12)
    assert pk["e_min"] == rp["e_min"] and pk["e_max"] == rp["e_max"]


def test_profile_of_one_tube_of_a_batch(torch_gpu):
    _say("case: profile of each tube of a 3-tube handle vs plain handles")
    cfgs = [dict(workloads.TINY, n_cells=384, seed=5), dict(workloads.TINY, n_cells=1000, alpha=-1.0, seed=6),
            dict(workloads.TINY, n_cells=130, b=0.2, seed=7)]
    gb = Gap(cfgs)
    gb.step(120)
    gb.set_profile_bin(32)
    for t, c in enumerate(cfgs):
        gp = Gap(c)
        gp.step(120)
        gp.set_profile_bin(32)
        a, b = gb.profile(t), gp.profile()
        assert np.array_equal(a[:, :, 0], b[:, :, 0]), t
        assert np.allclose(a, b, rtol=1e-12, atol=0.0), t
        gp.close()
    gb.close()


def test_return_flux_of_known_absorptions(torch_gpu):
    # the oracle pin's state: six leptons in cell 0 moving down, zero frozen
    # field, no QED; all are absorbed in step 1 with their initial momenta
    _say("case: return flux of six known absorptions")
    N = 256
    cfg = dict(n_cells=N, init_kind=2, alpha=0.0, flags=G.FIELD_FROZEN | G.QED_OFF, seed=1, ppc_ref=4,
               inj_rate=0.0)
    gam = np.array([1.5, 10 ** 1.31, 10 ** 2.06, 10 ** 4.44, 10 ** 7.93, 10 ** 8.6])
    L = np.zeros(6, LEPTON_DTYPE)
    L["cell"], L["frac"] = 0, int(0.1 * (1 << 24))
    L["u"] = (-np.sqrt(gam ** 2 - 1.0)).astype(np.float32)
    L["w"] = [-1.0, 1.0, -2.0, 0.5, -1.0, 3.0]
    L["id"] = np.arange(1, 7, dtype=np.uint64)
    g = Gap(cfg)
    g.set_particles(L)
    g.set_field(np.zeros(N, np.float32), 0.0)
    g.return_spectrum()                      # clear
    g.step(1)
    assert g.counts()["n_absorbed"] == 6
    r = g.return_spectrum()
    o = Oracle(dict(cfg, flags=OF["FIELD_FROZEN"] | OF["QED_OFF"]))
    o.set_state(leptons_as_oracle(L), None, 0.0, 0)
    o.set_field(np.zeros(N), 0.0)
    o.step(1)
    ro = o.return_spectrum()
    assert np.array_equal(r[:65], ro[:65])
    assert math.isclose(r[65], ro[65], rel_tol=1e-6)        # gamma in FP32 on the GPU
    assert np.array_equal(g.return_spectrum(), np.zeros(66))
    g.close()


def test_return_flux_counts_every_absorption(torch_gpu):
    # tiny gap: every lepton weighs 1, so the returned weight over a run is
    # the number of absorbed leptons, and the gamma moment is at least it
    _say("case: return flux over 200 steps of the tiny gap")
    g = Gap(dict(workloads.TINY, seed=4))
    g.step(50)
    c0 = g.counts()
    g.return_spectrum()
    g.step(200)
    r, c1 = g.return_spectrum(), g.counts()
    n_abs = c1["n_absorbed"] - c0["n_absorbed"]
    _say("  absorbed %d, returned weight %.1f" % (n_abs, r[64]))
    assert n_abs > 0
    assert r[64] == float(n_abs) and r[:64].sum() == r[64]
    assert r[65] >= r[64]
    g.close()


def test_waterfall_matches_definition_and_oracle(torch_gpu):
    # every third step, bins of 37 cells (ragged): each record equals the
    # definition applied to the field read back after that step, and follows
    # the oracle's own run within the field tolerance
    _say("case: waterfall of the tiny gap, every 3 steps, bins of 37 cells, 40 steps")
    cfg = dict(workloads.TINY, seed=2)
    g = Gap(cfg)
    o = Oracle(cfg)
    g.set_waterfall(3, 37, 64)
    want, want_o = {}, {}
    for _ in range(40):
        g.step(1)
        o.step(1)
        s = g.counts()["step"]
        if s % 3 == 0:
            want[s] = diag.waterfall_row(g.field(), 37)
            want_o[s] = diag.waterfall_row(o.field(), 37)
    steps, e2 = g.waterfall()
    assert list(steps) == sorted(want)
    assert e2.shape == (len(want), (cfg["n_cells"] + 36) // 37)
    for s, row in zip(steps, e2):
        assert np.allclose(row, want[s], rtol=1e-12, atol=0.0), s
        assert np.max(np.abs(row - want_o[s])) <= 1e-4 * np.max(want_o[s]), s
    steps2, e22 = g.waterfall()                      # reading emptied it
    assert steps2.size == 0 and e22.shape[0] == 0
    g.close()


def test_waterfall_ring_keeps_the_last_records(torch_gpu):
    _say("case: waterfall ring of 4 records over 10 steps, then off")
    g = Gap(dict(workloads.TINY, n_cells=256, seed=3))
    s0 = g.counts()["step"]
    g.set_waterfall(1, 64, 4)
    g.step(10)
    steps, e2 = g.waterfall()
    assert list(steps) == [s0 + 7, s0 + 8, s0 + 9, s0 + 10]
    assert e2.shape == (4, 4) and np.all(np.isfinite(e2)) and np.all(e2 >= 0.0)
    g.set_waterfall(0)
    with pytest.raises(G.GapError):
        g.waterfall()
    g.close()


def test_waterfall_of_each_tube_of_a_batch(torch_gpu):
    _say("case: waterfall of each tube of a 3-tube handle vs plain handles")
    cfgs = [dict(workloads.TINY, n_cells=384, seed=5), dict(workloads.TINY, n_cells=1000, alpha=-1.0, seed=6),
            dict(workloads.TINY, n_cells=130, b=0.2, seed=7)]
    gb = Gap(cfgs)
    gb.set_waterfall(2, 32, 16)
    gb.step(20)
    for t, c in enumerate(cfgs):
        gp = Gap(c)
        gp.set_waterfall(2, 32, 16)
        gp.step(20)
        sa, a = gb.waterfall(t)
        sb, b = gp.waterfall()
        assert np.array_equal(sa, sb) and np.array_equal(a, b), t
        gp.close()
    gb.close()


def test_e_spectrum_matches_definition(grown):
    g, cfg = grown
    _say("case: E power spectrum of the tiny gap at step 300")
    P = g.e_spectrum()
    ref = diag.e_power_spectrum(g.field())
    assert P.shape == ref.shape == (513,)
    assert np.max(np.abs(P - ref)) <= 1e-11 * np.max(ref)


def test_e_spectrum_of_a_set_cosine_and_a_ragged_grid(torch_gpu):
    _say("case: E power spectrum of a frozen cosine field (4096 cells) and of 130 cells")
    N, m, A = 4096, 111, 2.5
    g = Gap(dict(workloads.TINY, n_cells=N, flags=G.FIELD_FROZEN | G.QED_OFF))
    E = (A * np.cos(2 * np.pi * m * np.arange(N) / N)).astype(np.float32)
    g.set_field(E, 0.0)
    P = g.e_spectrum()
    ref = diag.e_power_spectrum(E)
    assert np.max(np.abs(P - ref)) <= 1e-11 * np.max(ref)
    assert math.isclose(P[m], A * A * N / 4, rel_tol=1e-6)
    assert np.max(np.delete(P, m)) < 1e-9 * P[m]
    g.close()
    g = Gap(dict(workloads.TINY, n_cells=130, seed=3))
    g.step(40)
    P, ref = g.e_spectrum(), diag.e_power_spectrum(g.field())
    assert P.shape == (129,) and np.max(np.abs(P - ref)) <= 1e-11 * np.max(ref)
    g.close()


def test_momentum_spectra_match_oracle(grown):
    g, cfg = grown
    _say("case: momentum spectra of the tiny gap at step 300")
    L, P = leptons_as_oracle(g.leptons()), photons_as_oracle(g.photons())
    S, ref = g.spectra(), diag.spectra(L, P)
    assert S.shape == (3, 90)
    assert np.array_equal(S, ref)                       # unit weights: exact sums in FP64
    c = g.counts()
    assert S[0].sum() + S[1].sum() == c["n_lep"] and S[2].sum() == c["n_pho"]


def test_momentum_spectra_of_a_set_beam_and_of_a_batch_tube(torch_gpu):
    _say("case: momentum spectra of a loaded beam and of each tube of a batch")
    N = 256
    g = Gap(dict(workloads.TINY, n_cells=N, flags=G.QED_OFF))
    L = np.zeros(9, LEPTON_DTYPE)
    L["cell"], L["frac"] = np.arange(9) * 20, 0
    L["u"] = np.array([1e-3, 0.01, 0.0999, 1.0, 1e3, -1e3, 3.0e7, 1e9, 4e9], np.float32)
    L["w"] = [1.0, -1.0, 2.0, -0.5, 1.0, -1.0, 1.0, -1.0, 3.0]
    L["id"] = np.arange(1, 10, dtype=np.uint64)
    g.set_particles(L)
    S, ref = g.spectra(), diag.spectra(leptons_as_oracle(L), None)
    assert np.array_equal(S, ref)
    assert S[1, 0] == 1.0 and S[1, 89] == 3.0 and S[0, 89] == 1.0    # 1e9 in float32 is >= 1e9
    g.close()
    cfgs = [dict(workloads.TINY, n_cells=384, seed=5), dict(workloads.TINY, n_cells=130, b=0.2, seed=7)]
    gb = Gap(cfgs)
    gb.step(150)
    for t, c in enumerate(cfgs):
        gp = Gap(c)
        gp.step(150)
        assert np.array_equal(gb.spectra(t), gp.spectra()), t
        gp.close()
    gb.close()


@pytest.mark.parametrize("bin_cells", [64, 37])
def test_phase_space_matches_oracle(grown, bin_cells):
    g, cfg = grown
    _say("case: phase space of the tiny gap at step 300, bins of %d cells" % bin_cells)
    g.set_profile_bin(bin_cells)
    L, P = leptons_as_oracle(g.leptons()), photons_as_oracle(g.photons())
    ph, ref = g.phase_space(), diag.phase_space(L, P, cfg["n_cells"], bin_cells)
    assert ph.shape == ref.shape == (3, (cfg["n_cells"] + bin_cells - 1) // bin_cells, 180)
    assert np.array_equal(ph, ref)                      # unit weights: exact sums in FP64
    S = g.spectra()
    assert np.array_equal(ph.sum(axis=1)[:, 90:] + ph.sum(axis=1)[:, 89::-1], S)


def test_phase_space_of_one_tube_of_a_batch(torch_gpu):
    _say("case: phase space of each tube of a 2-tube handle vs plain handles")
    cfgs = [dict(workloads.TINY, n_cells=384, seed=5), dict(workloads.TINY, n_cells=130, b=0.2, seed=7)]
    gb = Gap(cfgs)
    gb.step(150)
    gb.set_profile_bin(16)
    for t, c in enumerate(cfgs):
        gp = Gap(c)
        gp.step(150)
        gp.set_profile_bin(16)
        assert np.array_equal(gb.phase_space(t), gp.phase_space()), t
        gp.close()
    gb.close()
