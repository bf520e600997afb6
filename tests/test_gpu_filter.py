"""The current filter (Sect. 6.1; GAP_FILTER) on the HIP path against the
FP64 oracle's: the field over 100 steps of the tiny gap, the filtered cold
Langmuir mode against the filter's transfer function, a filtered tube in a
batch, and the cases the flag refuses."""
import math
import sys

import numpy as np
import pytest

from paper_2608_21920_amd import Gap, workloads
from paper_2608_21920_amd import gap as G
from oracle.oracle import Oracle

from gpu_util import rel_field_err

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


def _filtered(cfg):
    return dict(cfg, flags=cfg.get("flags", 0) | G.FILTER)


def test_filtered_field_parity_100_steps_tiny(torch_gpu):
    _say("case: filtered field parity over 100 steps, tiny gap")
    cfg = _filtered(workloads.TINY)
    g, o = Gap(cfg), Oracle(cfg)
    assert np.array_equal(g.field(), o.field().astype(np.float32))     # no filtering at the set state
    worst = 0.0
    for n in range(100):
        g.step(1)
        o.step(1)
        err = rel_field_err(g.field(), o.field())
        worst = max(worst, err)
        assert err <= 1e-5, (n, err)
    assert rel_field_err(g.node_field(), o.node_field()) <= 1e-5
    _say("  worst rel field err %.3e" % worst)
    # the filter changed the field: an unfiltered run differs by far more
    u = Gap(workloads.TINY)
    u.step(100)
    assert rel_field_err(u.field(), o.field()) > 1e-3
    assert g.counts()["err"] == 0
    u.close()
    g.close()


def _langmuir(flags, N, ppc, m, steps):
    g = Gap(dict(n_cells=N, init_kind=2, alpha=0.0, flags=flags, cap_leptons=1 << 16))
    cell = np.repeat(np.arange(N), ppc)
    frac = np.tile(((np.arange(ppc) + 0.5) / ppc * 2 ** 24).astype(np.uint32), N)
    kx = 2 * math.pi * m / (N * 0.25)
    rec = np.zeros(N * ppc, G.LEPTON_DTYPE)
    rec["cell"], rec["frac"], rec["w"] = cell, frac, -1.0
    rec["u"] = 1e-4 * np.sin(kx * (cell + frac / 2 ** 24) * 0.25)
    rec["id"] = np.arange(1, N * ppc + 1)
    g.set_particles(rec)
    hc = (np.arange(N) + 0.5) * 0.25
    amp = []
    for _ in range(steps):
        g.step(1)
        amp.append(float((g.field().astype(np.float64) * np.sin(kx * hc)).sum()))
    dt = g.derived()["dt"]
    g.close()
    s = np.asarray(amp) - np.mean(amp)
    idx = np.where((s[:-1] < 0) & (s[1:] >= 0))[0]
    t = [(i + s[i] / (s[i] - s[i + 1])) * dt for i in idx]
    return 2 * math.pi / ((t[-1] - t[0]) / (len(t) - 1)), dt, kx


def test_filtered_langmuir_follows_the_transfer_function(torch_gpu):
    _say("case: filtered cold Langmuir mode (k dx = 0.49), periodic")
    base = G.QED_OFF | G.PERIODIC
    wu, dt, kx = _langmuir(base, 512, 16, 40, 700)
    wf, _, _ = _langmuir(base | G.FILTER, 512, 16, 40, 700)
    T = math.cos(kx * 0.25 / 2) ** 16
    ratio = math.sin(wf * dt / 2) ** 2 / math.sin(wu * dt / 2) ** 2
    _say("  omega %.5f -> %.5f, ratio %.6f, transfer %.6f" % (wu, wf, ratio, T))
    assert abs(ratio / T - 1) < 1e-3


def test_filtered_tube_in_a_batch(torch_gpu):
    _say("case: filtered and unfiltered tubes in one handle vs plain handles")
    cfgs = [_filtered(dict(workloads.TINY, n_cells=384, seed=5)), dict(workloads.TINY, n_cells=1000, seed=6),
            _filtered(dict(workloads.TINY, n_cells=130, alpha=-1.0, seed=7))]
    gb = Gap(cfgs)
    gb.step(60)
    for t, c in enumerate(cfgs):
        gp = Gap(c)
        gp.step(60)
        assert np.array_equal(gb.field(t), gp.field()), t
        assert np.array_equal(gb.node_field(t), gp.node_field()), t
        gp.close()
    gb.close()


def test_filter_refusals(torch_gpu):
    _say("case: filter refused below 16 cells and for the differentiable window")
    with pytest.raises(G.GapError):
        Gap(_filtered(dict(workloads.TINY, n_cells=12)))
    g = Gap(_filtered(dict(workloads.TINY, n_cells=256)))
    with pytest.raises(G.GapError):
        g.window_forward(10, 5)
    g.close()


def test_graph_replays_with_filter_and_waterfall(torch_gpu):
    # the filter kernel and the waterfall record are inside the captured
    # steps; every replay, with eager work between, matches eager stepping
    _say("case: graph replays of filtered steps with the waterfall on")
    import torch
    cfg = _filtered(dict(workloads.TINY, n_cells=512))
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ga = Gap(cfg, stream=s)
        gb = Gap(cfg, stream=s)
        for g in (ga, gb):
            g.set_waterfall(4, 32, 64)
        for r in range(5):
            ga.step_graph(16)
            ga.sync()
            gb.step(16)
            assert np.array_equal(ga.field(), gb.field()), r
            sa, a = ga.waterfall()
            sb, b = gb.waterfall()
            assert np.array_equal(sa, sb) and np.array_equal(a, b), r
            assert sa.size == 4, r
        ga.close()
        gb.close()


@pytest.mark.parametrize("alpha", [2.0, -2.0])
def test_paper_preset_field_parity(torch_gpu, alpha):
    # the paper's setup (b = 0.02, R_curv = 30 H, filter on, 38730 cells,
    # protons and the thermal atmosphere), with its fiducial alpha and the
    # tested -2
    _say("case: paper preset, alpha %+.0f, field parity over 100 steps" % alpha)
    cfg = dict(workloads.PAPER, alpha=alpha, cap_leptons=1 << 20, cap_photons=1 << 20, merge=False)
    g, o = Gap(cfg), Oracle(cfg)
    for n in range(100):
        g.step(1)
        o.step(1)
        err = rel_field_err(g.field(), o.field())
        assert err <= 1e-5, (n, err)
    cg, co, pc = g.counts(), o.counts(), o.proton_counts()
    assert cg["n_lep"] == co["n_lep"] and cg["err"] == 0
    assert (cg["n_pro"], cg["n_atm_e"], cg["n_atm_p"]) == (pc["n_pro"], pc["n_atm_e"], pc["n_atm_p"])
    assert abs(g.es() - o.Es) <= 1e-12 * max(1.0, abs(o.Es))
    g.close()
