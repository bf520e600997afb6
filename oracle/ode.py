"""Concurrency model of the discharge (Sect. 5.2, eqs. dis1-dis4; App. B).

Test infrastructure only.  State (m_pm, m_x, eps, j) in units of t_esc = 1:

    dm_pm/dt = 2 m_x / t_pm - m_pm / t_esc
    dm_x/dt  = -m_x / t_pm + (m_pm / t_x) H(|eps| - 1) - m_x / t_esc
    deps/dt  = (alpha - j) / t_esc
    dj/dt    = -j / t_esc + m_pm eps g3 / t_acc

H is the Heaviside step with H(0) = 0.  Solved with the implicit Radau IIA
(order 5) integrator, as the paper does (Sect. 5.4).  The optional current
cap |j| <= m_pm (the bulk flow cannot exceed c, Sect. 5.3) is a variant.
"""
from __future__ import annotations

import numpy as np
from scipy.integrate import solve_ivp


def rhs(t, y, alpha, t_pm, t_x, t_acc, g3, t_esc=1.0):
    m, mx, eps, j = y
    gate = 1.0 if abs(eps) > 1.0 else 0.0
    return [2.0 * mx / t_pm - m / t_esc,
            -mx / t_pm + m / t_x * gate - mx / t_esc,
            (alpha - j) / t_esc,
            -j / t_esc + m * eps * g3 / t_acc]


def solve(alpha=2.0, t_pm=1e-3, t_x=1e-3, t_acc=4e-8, g3=8e-8, t_end=60.0, cap=False,
          rtol=1e-8, atol=1e-12, max_step=1e-2, y0=(1.0, 0.0, 1.0, 0.0)):
    """Integrate the model piecewise: the Heaviside gate is held fixed on each
    piece and flipped at the event |eps| = 1, so the implicit integrator never
    sees the discontinuity.  Returns (t, y) arrays over the whole interval."""
    ts, ys = [np.array([0.0])], [np.array(y0, dtype=float).reshape(4, 1)]
    t0, y = 0.0, np.array(y0, dtype=float)
    gate = 1.0 if abs(y[2]) > 1.0 else 0.0

    def f(t, yy):
        m, mx, eps, j = yy
        dj = -j + m * eps * g3 / t_acc
        if cap and abs(j) >= m and np.sign(dj) == np.sign(j):
            dj = 0.0
        return [2.0 * mx / t_pm - m, -mx / t_pm + m / t_x * gate - mx, alpha - j, dj]

    def crossing(t, yy):
        return abs(yy[2]) - 1.0
    crossing.terminal = True

    n_pieces = 0
    while t0 < t_end and n_pieces < 100000:
        crossing.direction = -1.0 if gate else 1.0
        s = solve_ivp(f, (t0, t_end), y, method="Radau", rtol=rtol, atol=atol, max_step=max_step,
                      events=crossing)
        if s.status < 0:
            raise RuntimeError(s.message)
        ts.append(s.t[1:])
        ys.append(s.y[:, 1:])
        t0, y = s.t[-1], s.y[:, -1].copy()
        if s.status == 1:
            gate = 0.0 if gate else 1.0
            # step just past the switching surface along the flow
            t0 = np.nextafter(t0, np.inf)
        n_pieces += 1

    class Sol:
        pass
    out = Sol()
    out.t = np.concatenate(ts)
    out.y = np.concatenate(ys, axis=1)
    out.pieces = n_pieces
    return out


def cycles(sol, t_skip_cycles=1):
    """Per-cycle peak multiplicity M_pm and cycle lengths.

    A cycle's peak is the maximum of m_pm between successive ignitions, an
    ignition being an upward crossing of m_pm through 10 |alpha|-independent
    level 10 (the decay phase ends near m_pm ~ |alpha|, Sect. 5.3)."""
    t, m = sol.t, sol.y[0]
    lvl = 10.0
    up = np.where((m[:-1] < lvl) & (m[1:] >= lvl))[0]
    peaks, tpk = [], []
    for a, b in zip(up[:-1], up[1:]):
        k = a + int(np.argmax(m[a:b]))
        peaks.append(m[k])
        tpk.append(t[k])
    peaks = np.array(peaks[t_skip_cycles:])
    tpk = np.array(tpk[t_skip_cycles:])
    return peaks, np.diff(tpk)
