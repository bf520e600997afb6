"""Oracle pins: Philox4x32-10 and the unit system (CPU only)."""
import math
import os

import numpy as np

from oracle import oracle as O


def test_philox_known_answers(golden_dir):
    rows = [ln.split() for ln in open(os.path.join(golden_dir, "philox4x32_10_kat.txt"))
            if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(t, 16) for t in r]
        assert O.philox(v[0:4], v[4:6]) == v[6:10]


def test_philox_uniformity():
    # chi^2 of the 24-bit uniforms of 40000 consecutive counters over 64 bins
    u = np.array([O.u24(O.philox([i, 0, 7, (2 << 16)], [0, 0])[0]) for i in range(40000)])
    assert u.min() > 0 and u.max() < 1
    h, _ = np.histogram(u, bins=64, range=(0, 1))
    chi2 = ((h - 625.0) ** 2 / 625.0).sum()
    assert chi2 < 110  # 63 dof, p ~ 2e-4


def test_u24_midpoints():
    assert O.u24(0) == 0.5 / 2 ** 24
    assert O.u24(0xFFFFFFFF) == 1.0 - 0.5 / 2 ** 24
    assert O.u24(0x100) == 1.5 / 2 ** 24


def _derived(b, r_curv=1e7):
    o = O.Oracle(dict(n_cells=8, init_kind=2, b=b, r_curv_cm=r_curv))
    return o


def test_skin_depth_order_of_magnitude():
    # Sect. 2.2: c/omega_p,co ~ 3 cm for B = 1e12 G and P = 1 s
    o = _derived(1e12 / 4.414e13)
    assert 2.5 < o.d_cm < 3.5


def test_gyro_radius_and_threshold_scales():
    # Sect. 4: r_g ~ 1e-9 cm (so r_g/R_curv ~ 1e-15 at R_curv = 1e6 cm) and
    # gamma_thr = (4/3 R_curv/(b r_g))^(1/3) ~ 3e5 for R_curv = 1e6 cm.  With
    # b r_g = lambda_C, in skin-depth units gamma_thr = (4 R~/(3 lambda~))^(1/3).
    o = _derived(1e12 / 4.414e13, r_curv=1e6)
    r_g = 2.99792458e10 / (1.75882e7 * 1e12)
    assert 1e-9 < r_g < 3e-9
    g_thr = (4 * o.rc / (3 * o.lam)) ** (1 / 3)
    assert 2.5e5 < g_thr < 4e5
    # independent of b: b r_g = lambda_C
    o2 = _derived(0.3, r_curv=1e6)
    assert math.isclose((4 * o2.rc / (3 * o2.lam)) ** (1 / 3), g_thr, rel_tol=1e-12)


def test_paper_gap_energy():
    # Sect. 6.1: H_gap / (c/omega_p) ~ 7400 gives gamma_gap = H^2/2 ~ 3e7 in
    # skin-depth units (E_rot = H, gamma_gap = E_rot H / 2 for the linear ramp).
    # The oracle's initial field for the vacuum-below-H state ramps 0 -> H.
    o = O.Oracle(dict(n_cells=4096, dx=7400 / (0.8 * 4096), init_kind=0, ppc_init=1, ppc_ref=1,
                      b=0.02, r_curv_cm=1e7))
    E = o.field()
    assert math.isclose(E.max(), o.H, rel_tol=2e-3)
    gamma_gap = 0.5 * o.H * E.max()
    assert 2e7 < gamma_gap < 3.5e7
