"""Pins of the oracle's current filter (Sect. 6.1: binomial 3-point shape,
8 passes per step): the binomial coefficients of eight passes, uniform
arrays and sums kept at the ends, one pass against loops, and the cold
Langmuir mode, whose leapfrog frequency obeys sin^2(w dt / 2) ~ T(k) with
the filter's transfer function T(k) = cos^16(k dx / 2)."""
import math

import numpy as np

from oracle import oracle as O

F = O.FLAGS


def test_eight_passes_give_binomial_coefficients():
    x = np.zeros(41)
    x[20] = 1.0
    y = O.binomial_filter(x)
    ref = np.zeros(41)
    for j in range(17):
        ref[12 + j] = math.comb(16, j) / 2.0 ** 16
    assert np.array_equal(y, ref)


def test_uniform_arrays_and_sums_are_kept():
    rng = np.random.default_rng(5)
    for periodic in (False, True):
        assert np.array_equal(O.binomial_filter(np.full(57, -3.25), periodic=periodic), np.full(57, -3.25))
        x = rng.normal(0, 1, 57)
        y = O.binomial_filter(x, periodic=periodic)
        assert abs(y.sum() - x.sum()) < 1e-12 * np.abs(x).sum()
        assert np.max(np.abs(y)) < np.max(np.abs(x))      # smoothing


def test_one_pass_against_loops():
    rng = np.random.default_rng(6)
    x = rng.normal(0, 1, 23)
    for periodic in (False, True):
        ref = []
        for i in range(23):
            l = x[i - 1] if i > 0 else (x[-1] if periodic else x[0])
            r = x[i + 1] if i < 22 else (x[0] if periodic else x[-1])
            ref.append(0.25 * l + 0.5 * x[i] + 0.25 * r)
        assert np.allclose(O.binomial_filter(x, passes=1, periodic=periodic), ref, rtol=1e-15, atol=1e-16)


def _lep(cell, xi, u, w):
    return dict(cell=cell.astype(np.int32), xi=xi, u=u, w=w, id=np.arange(1, cell.size + 1, dtype=np.uint64))


def _langmuir_omega(flags, N, ppc, m, steps):
    o = O.Oracle(dict(n_cells=N, init_kind=2, alpha=0.0, flags=flags))
    cell = np.repeat(np.arange(N), ppc)
    xi = np.tile((np.arange(ppc) + 0.5) / ppc, N)
    kx = 2 * math.pi * m / (N * 0.25)
    o.set_state(_lep(cell, xi, 1e-4 * np.sin(kx * (cell + xi) * 0.25), -np.ones(N * ppc)))
    hc = (np.arange(N) + 0.5) * 0.25
    amp = []
    for _ in range(steps):
        o.step(1)
        amp.append(float((o.field() * np.sin(kx * hc)).sum()))
    s = np.asarray(amp) - np.mean(amp)
    idx = np.where((s[:-1] < 0) & (s[1:] >= 0))[0]
    t = [(i + s[i] / (s[i] - s[i + 1])) * o.dt for i in idx]
    return 2 * math.pi / ((t[-1] - t[0]) / (len(t) - 1)), o.dt, kx


def test_filtered_langmuir_mode_follows_the_transfer_function():
    # a short mode (k dx = 0.49) that the filter slows strongly; the shape
    # factors of deposit and gather cancel in the ratio
    N, ppc, m = 512, 16, 40             # ppc_ref = 16: neutral with the eta_co background
    base = F["QED_OFF"] | F["PERIODIC"]
    wu, dt, kx = _langmuir_omega(base, N, ppc, m, 700)
    wf, _, _ = _langmuir_omega(base | F["FILTER"], N, ppc, m, 700)
    T = math.cos(kx * 0.25 / 2) ** 16
    ratio = math.sin(wf * dt / 2) ** 2 / math.sin(wu * dt / 2) ** 2
    assert abs(ratio / T - 1) < 1e-4, (ratio, T)
    assert wf < 0.85 * wu
