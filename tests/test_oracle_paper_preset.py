"""The paper-setup preset (Sect. 6.1) against the scales the paper prints for
it: R_curv = 30 H_gap, gamma_gap = H^2/2 ~ 3e7 (E_rot = H), and
gamma_rad / gamma_gap ~ 0.3, with gamma_rad the radiation-reaction limit
(3 E R~^2 / (2 alpha_em lambda~))^(1/4) at E = E_rot (Sect. 4).  The units
(skin depth, lambda~, R~, H) are the oracle's own derived numbers."""
import math

from paper_2608_21920_amd import workloads
from oracle.oracle import Oracle, FLAGS


def test_paper_preset_scales():
    o = Oracle(dict(workloads.PAPER))
    assert workloads.PAPER["flags"] & FLAGS["FILTER"]
    assert abs(o.rc / o.H / 30.0 - 1) < 2e-3
    g_gap = o.H ** 2 / 2
    assert abs(g_gap / 3e7 - 1) < 0.01
    g_rad = (3 * o.H * o.rc ** 2 / (2 * (1 / 137.035999084) * o.lam)) ** 0.25
    assert abs(g_rad / g_gap - 0.3) < 0.01
    # two electrons per cell everywhere and two protons per cell below H
    # (charge 0 below H, n_co above), a thermal atmosphere at 0.3 m_e c^2
    kh = math.ceil(o.H / 0.25 - 1e-9)
    assert o.counts()["n_lep"] == 2 * o.N
    assert o.proton_counts()["n_pro"] == 2 * kh
    assert workloads.PAPER["atm_ppc"] > 0 and workloads.PAPER["atm_temp"] == 0.3
