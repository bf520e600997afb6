"""Pins of the FP64 adjoint of the frozen-QED window (oracle/adjoint.py).

The adjoint is checked against what does not depend on it: the closed form of
the vacuum drive (Sect. 2.2, E_s advanced by alpha s_co dt each step) and
central finite differences of the frozen map itself, with the QED off and
with a dense QED realisation (emission, photon births, conversions and pairs
inside the window)."""
import numpy as np
import pytest

from oracle.oracle import FLAGS, Oracle
from oracle import adjoint as A
from paper_2608_21920_amd import workloads

# Test-only QED preset in which photons convert within a few steps of their
# birth and pairs are born with gamma ~ 5: every kind of event occurs many
# times inside a short window (b = 1, R~ ~ 1 d, lambda~/R~ ~ 7e-3).
DENSE_QED = dict(n_cells=256, init_kind=1, ppc_init=8, alpha=1.5, b=1.0, lambda_c_scale=7.4e7,
                 r_curv_scale=4.3e-8, inj_rate=0.5, seed=3)


def _state(cfg, steps):
    o = Oracle(dict(cfg, flags=cfg.get("flags", 0) | FLAGS["INJ_FIXED"]))
    o.step(steps)
    return A.export_state(o)


def test_replay_reproduces_the_recorded_window():
    st = _state(DENSE_QED, 60)
    rec = A.Window(DENSE_QED, 25, st)
    rep = A.Window(DENSE_QED, 25, st, events=rec.events)
    assert rec.loss == rep.loss
    for a, b in zip(rec.snaps, rep.snaps):
        assert np.array_equal(a["E"], b["E"]) and a["Es"] == b["Es"]
        # replayed photon births enter the store in log order, and pairs
        # follow their photons: compare by id
        ia, ib = np.argsort(a["L"]["id"]), np.argsort(b["L"]["id"])
        for k in ("cell", "xi", "u", "w", "id"):
            assert np.array_equal(a["L"][k][ia], b["L"][k][ib]), k
        ia, ib = np.argsort(a["P"]["id"]), np.argsort(b["P"]["id"])
        for k in ("cell", "xi", "x", "w", "n0", "id"):
            assert np.array_equal(a["P"][k][ia], b["P"][k][ib]), k
    ev = rec.events
    assert (ev["kind"] == 0).sum() > 1000 and (ev["kind"] == 1).sum() > 100 and (ev["kind"] == 2).sum() > 1000


def test_vacuum_drive_closed_form():
    # no particles: E^m_k = E^0_k + alpha s_co dt m, so
    # dL/dalpha = 1/(W N) sum_m sum_k 2 E^m_k s_co dt m
    cfg = dict(n_cells=100, init_kind=2, alpha=1.5, flags=FLAGS["QED_OFF"])
    W = 50
    win = A.Window(cfg, W, None)
    ad = A.adjoint(win)
    N, dt, s_co = win.N, win.dt, win.s_co
    ref = sum(2.0 * win.snaps[m]["E"].sum() * s_co * dt * m for m in range(1, W + 1)) / (W * N)
    assert abs(ad["dL_dalpha"] / ref - 1) < 1e-12
    assert ad["dL_dninj"] == 0.0


def test_adjoint_matches_finite_differences_without_qed():
    cfg = dict(workloads.TINY, n_cells=128, ppc_init=8, inj_rate=0.5, flags=FLAGS["QED_OFF"])
    st = _state(cfg, 100)
    win = A.Window(cfg, 30, st)
    ad = A.adjoint(win)
    fd = A.finite_differences(cfg, 30, st, win.events, h=1e-4)
    assert abs(ad["dL_dalpha"] / fd["dL_dalpha"] - 1) < 1e-5
    assert abs(ad["dL_dninj"] / fd["dL_dninj"] - 1) < 1e-5


@pytest.mark.parametrize("W", [2, 40])
def test_adjoint_matches_finite_differences_with_frozen_qed(W):
    st = _state(DENSE_QED, 60)
    win = A.Window(DENSE_QED, W, st)
    ad = A.adjoint(win)
    fd = A.finite_differences(DENSE_QED, W, st, win.events, h=1e-4)
    assert abs(ad["dL_dalpha"] / fd["dL_dalpha"] - 1) < 1e-5
    assert abs(ad["dL_dninj"] / fd["dL_dninj"] - 1) < 1e-5


def test_adjoint_on_the_tiny_preset_with_injection():
    # the rescaled tiny gap after its first emissions: QED-frozen window of
    # 40 steps, gradients of the time-averaged field energy
    cfg = dict(workloads.TINY, n_cells=256, ppc_init=8, inj_rate=0.5)
    st = _state(cfg, 450)
    win = A.Window(cfg, 40, st)
    assert (win.events["kind"] == 0).sum() > 100
    ad = A.adjoint(win)
    fd = A.finite_differences(cfg, 40, st, win.events, h=1e-4)
    assert abs(ad["dL_dalpha"] / fd["dL_dalpha"] - 1) < 1e-5
    assert abs(ad["dL_dninj"] / fd["dL_dninj"] - 1) < 1e-5
