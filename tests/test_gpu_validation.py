"""Model-vs-PIC check of the discharge on the GPU (Sect. 5 and the ringing
frequency of App. B.5, eq. omega_osc).

Once the pair cascade has screened the gap, the field rings at the plasma
frequency of the pairs, omega_osc = omega_p,co sqrt(M <gamma^-3>) (omega_p,co
= 1 in these units), with M the pair multiplicity and <gamma^-3> the pairs'
inertia measure; the paper finds the kinetic runs in reasonable (rough)
agreement with it.  The bar here is SURVEY's factor 2: in every screened
window of a long run of the tiny gap, the dominant angular frequency of E at
the cells of the multiplicity peak lies within a factor 2 of
sqrt(M <gamma^-3>) measured there by the library's own diagnostics
(GAP_DIAG_PEAK).  Parity with the paper is unpinned (its runs use other
parameters and physics); this checks the model relation on our own run.
"""
import numpy as np
import pytest

from paper_2608_21920_amd import Gap, workloads
from paper_2608_21920_amd import gap as G

pytestmark = pytest.mark.gpu

BIN = 64


def _run(steps, every=100):
    cfg = dict(workloads.TINY, flags=G.MERGE_ON, cap_leptons=1 << 20, cap_photons=1 << 20, merge_every=16,
               merge_frac=0.9)
    g = Gap(cfg)
    g.set_profile_bin(BIN)
    d = g.derived()
    E = np.zeros((steps, cfg["n_cells"]), np.float32)
    peaks = []
    for n in range(steps):
        g.step(1)
        E[n] = g.field()
        if (n + 1) % every == 0:
            pk = g.peak()
            peaks.append((n + 1, pk["m_pairs"], pk["h"], pk["g3"], pk["e_max"]))
    assert g.counts()["err"] == 0
    g.close()
    return E, np.array(peaks), d


def _omega_peak(x, dt):
    """Dominant angular frequency of the columns of x (time along axis 0),
    each detrended by a quadratic, Hann-windowed; power summed over columns;
    the two lowest bins excluded."""
    n = x.shape[0]
    t = np.arange(n)
    y = x - np.stack([np.polyval(np.polyfit(t, x[:, j], 2), t) for j in range(x.shape[1])], axis=1)
    P = (np.abs(np.fft.rfft(y * np.hanning(n)[:, None], axis=0)) ** 2).sum(axis=1)
    f = np.fft.rfftfreq(n, dt) * 2.0 * np.pi
    k = 2 + int(np.argmax(P[2:]))
    return f[k]


def test_ringing_frequency_follows_pair_plasma_frequency():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("case: tiny gap with merging, 2600 steps, ringing vs sqrt(M <gamma^-3>)", flush=True)
    E, pk, d = _run(2600)
    dt, dx = d["dt"], 0.25
    e0 = float(np.abs(E[50]).max())
    W = 600
    checked = []
    for a in range(800, 2600 - W + 1, 200):
        rows = pk[(pk[:, 0] > a) & (pk[:, 0] <= a + W)]
        screened = np.abs(E[a:a + W]).max() < 0.25 * e0
        if rows.size == 0 or rows[:, 1].min() < 10.0 or not screened:
            continue
        pred = float(np.mean(np.sqrt(rows[:, 1] * rows[:, 3])))
        mid = rows[len(rows) // 2]
        b = int(mid[2] / (BIN * dx))                      # the peak's bin
        cells = slice(b * BIN, (b + 1) * BIN)
        meas = _omega_peak(E[a:a + W, cells].astype(np.float64), dt)
        print("  window %d-%d: peak M %.1f at h %.0f, <g^-3> %.3g; predicted %.3f measured %.3f" % (
            a, a + W, mid[1], mid[2], mid[3], pred, meas), flush=True)
        checked.append((a, pred, meas))
        assert 0.5 <= meas / pred <= 2.0, (a, pred, meas)
    assert len(checked) >= 2, checked


def _paper_first_cycle():
    """The paper preset (its Sect. 6.1 setup) from the initial state through
    the first discharge until the gap ignites again.  Every 500 steps: the
    peak pair multiplicity in the gap zone with its height and <gamma^-3>
    (GAP_DIAG_PEAK), and the pair multiplicity averaged over the bins below
    H (GAP_DIAG_PROFILE); the return flux summed over the run.  Four windows
    of 2048 steps in the saturation phase sample E at the cells of the peak's
    bin every step."""
    cfg = dict(workloads.PAPER)
    g = Gap(cfg)
    g.set_profile_bin(BIN)
    d = g.derived()
    H, dt = d["H"], d["dt"]
    nb = int(H / (BIN * 0.25))                          # bins wholly below H
    win_at = [int(round(f * H / dt)) for f in (0.3, 0.45, 0.6, 0.75)]
    rec, wins = [], []
    ret = np.zeros(G.RETURN_BINS + 2)
    m_max, exited, emptied, t_ign = 0.0, None, False, []
    step = 0
    while step < int(6.5 * H / dt):
        if win_at and step >= win_at[0]:
            win_at.pop(0)
            p0 = g.peak()
            b = min(int(p0["h"] / (BIN * 0.25)), nb - 1)
            Ew = np.zeros((2048, BIN))
            for k in range(2048):
                g.step(1)
                Ew[k] = g.field()[b * BIN:(b + 1) * BIN]
            p1 = g.peak()
            wins.append((step * dt / H, np.sqrt(p0["m_pairs"] * p0["g3"]), np.sqrt(p1["m_pairs"] * p1["g3"]),
                         _omega_peak(Ew, dt), Ew.std() / H))
            step += 2048
        g.step(500)
        step += 500
        pk = g.peak()
        mz = float(g.profile()[:nb, :4, 0].sum(axis=1).mean())
        ret += g.return_spectrum()
        t = step * dt / H
        rec.append((t, pk["m_pairs"], pk["h"], pk["g3"], mz))
        if mz >= 10.0 and (not t_ign or emptied):
            t_ign.append(t)
            emptied = False
            if len(t_ign) == 2:
                break
        m_max = max(m_max, mz)
        if exited is None and t_ign and mz < 0.1 * m_max:
            exited = t
        if exited is not None and mz < 3.0:
            emptied = True
        if len(rec) % 40 == 0:
            print("  t %.2f t_esc: peak M %.1f at h %.0f, <g^-3> %.2e; zone mean %.1f" % rec[-1], flush=True)
    c = g.counts()
    g.close()
    return np.array(rec), wins, ret, t_ign, exited, c, cfg


def test_paper_preset_discharge_against_the_papers_kinetic_run():
    """The paper's printed kinetic-run values for its fiducial setup
    (Sect. 6.2 observed dynamics, 6.3 peak multiplicity, 6.6 oscillations),
    each with a factor-2 band unless stated:

    * peak multiplicity in the gap zone 1e3 to 1e4, gap-averaged a few 1e2;
    * M_pm ~ 5e2 at t = 0.5 t_esc;
    * <gamma^-3> below 1e-10 while the gap loads (median over
      0.02..0.12 t_esc; bar 1e-9);
    * the pair cloud leaves the zone near 1.1 t_esc (the zone mean falls
      below a tenth of its maximum within 0.9..1.6 t_esc);
    * ringing from t ~ 0.2 t_esc with dE/E_rot ~ 1e-2 (bar 3e-3..3e-2 at
      0.3 t_esc), at omega_osc = sqrt(M <gamma^-3>) (factor 2), sweeping up
      through saturation;
    * a cycle shorter than the model's ln(M_pm / alpha) t_esc (Sect. 5.3,
      eq. t_cycle), longer than the flush time of ~ t_esc.
    """
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("case: paper preset, first discharge and re-ignition against the paper's kinetic run", flush=True)
    rec, wins, ret, t_ign, t_exit, c, cfg = _paper_first_cycle()
    assert c["err"] == 0
    t, mpk, g3, mz = rec[:, 0], rec[:, 1], rec[:, 3], rec[:, 4]
    first = t <= (t_exit if t_exit else t[-1])
    at_half = mpk[np.argmin(np.abs(t - 0.5))]
    loading = np.median(g3[(t >= 0.02) & (t <= 0.12)])
    print("  peak M %.0f, zone mean %.0f, M at 0.5 t_esc %.0f, loading <g^-3> %.1e, exit %s, ignitions %s" % (
        mpk[first].max(), mz[first].max(), at_half, loading, t_exit, t_ign), flush=True)
    for w in wins:
        print("  window at %.2f t_esc: sqrt(M g3) %.3f .. %.3f, measured omega %.3f, dE/E_rot %.1e" % w, flush=True)
    gam = 10.0 ** ((np.arange(G.RETURN_BINS) + 0.5) / 8.0)
    dn = ret[:G.RETURN_BINS]
    hot = gam > 10.0
    mode = gam[hot][np.argmax(dn[hot])]
    tail = (gam > 1e4) & (gam < 1e6) & (dn > 0)
    slope = -np.polyfit(np.log(gam[tail]), np.log(dn[tail]), 1)[0] if tail.sum() > 3 else np.nan
    print("  return flux: mode above gamma 10 at %.0f, tail slope s %.2f over 1e4..1e6" % (mode, slope), flush=True)
    assert 500.0 <= mpk[first].max() <= 2e4
    assert 100.0 <= mz[first].max() <= 2000.0
    assert 250.0 <= at_half <= 1000.0
    assert loading < 1e-9
    assert t_exit is not None and 0.9 <= t_exit <= 1.6
    assert len(wins) == 4
    for tw, p0, p1, om, amp in wins:
        assert 0.5 <= om / np.sqrt(p0 * p1) <= 2.0, (tw, p0, p1, om)
    assert all(b[3] > a[3] for a, b in zip(wins[:-1], wins[1:]))
    assert 3e-3 <= wins[0][4] <= 3e-2
    assert len(t_ign) == 2
    cyc = t_ign[1] - t_ign[0]
    assert 1.5 <= cyc <= np.log(mpk[first].max() / abs(cfg["alpha"])), cyc
