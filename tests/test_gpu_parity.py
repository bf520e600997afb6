"""Parity of the HIP path with the FP64 oracle (runs on the MI355X).

Every GPU call goes through the C ABI (ctypes binding).  The bars:
 * integer work (initial state, node charge on an identical state) bit-exact;
 * field within 1e-5 of max|E| at every step of the first 100 (FP32 vs FP64);
 * Monte Carlo events: identical realisation while the two sides agree,
   statistical agreement afterwards.
"""
import math
import sys

import numpy as np
import pytest

from paper_2608_21920_amd import Gap, workloads
from paper_2608_21920_amd import gap as G
from paper_2608_21920_amd.inputs import random_state
from oracle.oracle import Oracle, FLAGS as OF

from gpu_util import by_id, gpu_leptons_as_oracle, gpu_photons_as_oracle, rel_field_err

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


TINY = workloads.TINY


def test_initial_state_bit_exact(torch_gpu):
    _say("case: initial state, tiny gap")
    g, o = Gap(TINY), Oracle(TINY)
    L = by_id(gpu_leptons_as_oracle(g.leptons()))
    R = by_id(o.leptons())
    assert L["id"].size == R["id"].size == 32768
    for k in ("cell", "xi", "u", "w", "id"):
        assert np.array_equal(L[k], R[k]), k
    assert np.array_equal(g.rho(), o.rho())
    assert np.array_equal(g.field(), o.field().astype(np.float32))
    assert np.array_equal(g.node_field(), o.node_field().astype(np.float32))
    g.close()


def test_field_parity_100_steps_tiny(torch_gpu):
    _say("case: field parity over 100 steps, tiny gap")
    g, o = Gap(TINY), Oracle(TINY)
    worst = 0.0
    for n in range(100):
        g.step(1)
        o.step(1)
        err = rel_field_err(g.field(), o.field())
        worst = max(worst, err)
        assert err <= 1e-5, (n, err)
    cg, co = g.counts(), o.counts()
    _say("worst rel field err %.3e; gpu emit %d pho %d, oracle emit %d pho %d" %
         (worst, cg["n_emit"], cg["n_pho"], co["n_emit"], co["n_pho"]))
    assert cg["err"] == 0
    # the Monte Carlo realisation is the same: emission decisions agree up to
    # FP32/FP64 near-ties of u < p
    assert abs(cg["n_emit"] - co["n_emit"]) <= max(2, 1e-3 * co["n_emit"])
    assert abs(cg["n_lep"] - co["n_lep"]) <= 2
    assert abs(g.es() - o.Es) <= 1e-12 * max(1.0, abs(o.Es))
    # photons: same ids; energies within the table accuracy
    P, Q = by_id(gpu_photons_as_oracle(g.photons())), by_id(o.photons())
    common, ia, ib = np.intersect1d(P["id"], Q["id"], return_indices=True)
    assert common.size >= 0.999 * max(P["id"].size, Q["id"].size)
    assert np.all(P["n0"][ia] == Q["n0"][ib])
    assert np.allclose(P["x"][ia], Q["x"][ib], rtol=2e-4, atol=0)
    g.close()


def test_identical_state_deposit_bit_exact(torch_gpu):
    # a seeded synthetic state (mixed charges and weights, ragged grid) loaded
    # into both sides: node charge bit-exact, field identical after FP32 rounding
    for seed, n, N in ((21, 200000, 1000), (22, 5000, 130)):
        _say("case: identical-state deposit, seed %d, %d leptons on %d cells" % (seed, n, N))
        L, _ = random_state(seed, n, 0, N, weights=(-1.0, 1.0, -2.0, 2.0, -0.5, 0.75))
        cfg = dict(TINY, n_cells=N, init_kind=2)
        g, o = Gap(cfg), Oracle(cfg)
        g.set_particles(L)
        o.set_state(gpu_leptons_as_oracle(L))
        assert np.array_equal(g.rho(), o.rho())
        assert np.array_equal(g.field(), o.field().astype(np.float32))
        g.close()


def test_vacuum_drive(torch_gpu):
    _say("case: vacuum drive")
    cfg = dict(n_cells=300, init_kind=2, alpha=1.5, flags=G.QED_OFF)
    g = Gap(cfg)
    g.step(1000)
    d = g.derived()
    es = g.es()
    # 1000 FP64 additions: round-off bound 1000 ulp(|E_s|)
    assert abs(es - (-1.5 * d["dt"] * 1000)) <= 1000 * np.spacing(abs(es))
    E = g.field()
    k = np.arange(300)
    assert np.allclose(E, (es + (k + 0.5) * 0.25).astype(np.float32), rtol=0, atol=2e-5)
    g.close()


def test_ragged_and_minimal_grids(torch_gpu):
    # N not a multiple of the tile width, and the smallest grid
    for n in (1000, 130, 2):
        _say("case: ragged grid N=%d" % n)
        cfg = dict(TINY, n_cells=n, ppc_init=4)
        g, o = Gap(cfg), Oracle(cfg)
        for _ in range(30):
            g.step(1)
            o.step(1)
            assert rel_field_err(g.field(), o.field()) <= 1e-5
        assert g.counts()["err"] == 0
        g.close()


def test_empty_gap_and_injection(torch_gpu):
    _say("case: empty gap with surface injection")
    cfg = dict(TINY, n_cells=512, init_kind=2, inj_rate=0.1, flags=G.QED_OFF)
    g, o = Gap(cfg), Oracle(cfg)
    for _ in range(200):
        g.step(1)
        o.step(1)
    cg, co = g.counts(), o.counts()
    assert cg["n_injected"] == co["n_injected"] == 320
    assert cg["n_lep"] == co["n_lep"]
    assert rel_field_err(g.field(), o.field()) <= 1e-5
    L, R = by_id(gpu_leptons_as_oracle(g.leptons())), by_id(o.leptons())
    assert np.array_equal(L["id"], R["id"])
    assert np.array_equal(L["cell"], R["cell"])
    assert np.max(np.abs(L["xi"] - R["xi"])) < 1e-4
    g.close()


def test_cold_langmuir_gpu(torch_gpu):
    _say("case: cold Langmuir, periodic")
    N, ppc = 1024, 16
    cfg = dict(n_cells=N, init_kind=2, alpha=0.0, flags=G.QED_OFF | G.PERIODIC, cap_leptons=1 << 16)
    g = Gap(cfg)
    cell = np.repeat(np.arange(N), ppc)
    frac = np.tile(((np.arange(ppc) + 0.5) / ppc * 2 ** 24).astype(np.uint32), N)
    kx = 2 * math.pi / (N * 0.25)
    h = (cell + frac / 2 ** 24) * 0.25
    rec = np.zeros(N * ppc, G.LEPTON_DTYPE)
    rec["cell"], rec["frac"], rec["u"], rec["w"] = cell, frac, 1e-4 * np.sin(kx * h), -1.0
    rec["id"] = np.arange(1, N * ppc + 1)
    g.set_particles(rec)
    hc = (np.arange(N) + 0.5) * 0.25
    amp = []
    for _ in range(480):
        g.step(1)
        amp.append(float((g.field().astype(np.float64) * np.sin(kx * hc)).sum()))
    s = np.asarray(amp) - np.mean(amp)
    idx = np.where((s[:-1] < 0) & (s[1:] >= 0))[0]
    dt = g.derived()["dt"]
    t = [(i + s[i] / (s[i] - s[i + 1])) * dt for i in idx]
    w = 2 * math.pi / ((t[-1] - t[0]) / (len(t) - 1))
    w_disc = 2 / dt * math.asin(dt / 2)
    assert abs(w / w_disc - 1) < 3e-4
    g.close()


def test_hyperbolic_motion_gpu(torch_gpu):
    _say("case: hyperbolic motion, frozen field")
    N, E0 = 4096, 0.8
    cfg = dict(n_cells=N, init_kind=2, flags=G.QED_OFF | G.FIELD_FROZEN, cap_leptons=1024)
    g = Gap(cfg)
    rec = np.zeros(1, G.LEPTON_DTYPE)
    rec["cell"], rec["frac"], rec["u"], rec["w"], rec["id"] = 10, 0, 0.0, 1.0, 1
    g.set_particles(rec)
    g.set_field(np.full(N, E0, np.float32), E0)
    o = Oracle(dict(cfg, flags=OF["QED_OFF"] | OF["FIELD_FROZEN"]))
    o.set_state(gpu_leptons_as_oracle(rec))
    o.set_field(np.full(N, E0), E0)
    for _ in range(10):
        g.step(100)
        o.step(100)
    a, b = g.leptons(), o.leptons()
    xa = a["cell"][0] + a["frac"][0] / 2 ** 24
    xb = b["cell"][0] + b["xi"][0]
    # 1000 FP32 kicks accumulate at most ~1000 * 2^-24 relative round-off
    assert abs(a["u"][0] - b["u"][0]) / b["u"][0] < 1000 * 2.0 ** -24
    assert abs(xa - xb) < 1e-3
    g.close()


def test_deterministic_and_order_independent(torch_gpu):
    _say("case: determinism and re-sort independence")
    cfg = dict(TINY, n_cells=512)
    runs = []
    for rb in (0, 1, 7):
        g = Gap(dict(cfg, rebucket_every=rb))
        g.step(220)
        runs.append((by_id(gpu_leptons_as_oracle(g.leptons())), g.field(), g.rho()))
        g.close()
    for L, E, r in runs[1:]:
        for k in ("cell", "xi", "u", "w", "id"):
            assert np.array_equal(L[k], runs[0][0][k]), k
        assert np.array_equal(E, runs[0][1])
        assert np.array_equal(r, runs[0][2])


def test_batched_tubes_equal_plain_runs(torch_gpu):
    _say("case: batched tubes bitwise equal to plain runs")
    cfgs = [dict(TINY, n_cells=384, seed=5), dict(TINY, n_cells=1000, alpha=-1.0, seed=6, ppc_init=8),
            dict(TINY, n_cells=130, b=0.2, seed=7)]
    gb = Gap(cfgs)
    gb.step(160)
    for t, c in enumerate(cfgs):
        gp = Gap(c)
        gp.step(160)
        A, B = by_id(gpu_leptons_as_oracle(gb.leptons(t))), by_id(gpu_leptons_as_oracle(gp.leptons()))
        for k in ("cell", "xi", "u", "w", "id"):
            assert np.array_equal(A[k], B[k]), (t, k)
        assert np.array_equal(gb.field(t), gp.field())
        assert gb.es(t) == gp.es()
        gp.close()
    gb.close()


def test_graph_replay_equals_eager(torch_gpu):
    _say("case: graph replay equals eager steps")
    import torch
    cfg = dict(TINY, n_cells=512, rebucket_every=8)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ga = Gap(cfg, stream=s)
        for _ in range(6):
            ga.step_graph(16)
            ga.sync()
            _ = ga.counts()   # eager work between replays
        gb = Gap(cfg, stream=s)
        gb.step(96)
        A, B = by_id(gpu_leptons_as_oracle(ga.leptons())), by_id(gpu_leptons_as_oracle(gb.leptons()))
        for k in ("cell", "xi", "u", "w", "id"):
            assert np.array_equal(A[k], B[k]), k
        assert np.array_equal(ga.field(), gb.field())
        ga.close()
        gb.close()


def test_store_overflow_reports_ecap(torch_gpu):
    # a photon store far too small for the cascade: births past the cap are
    # dropped, the tail stays inside the store, the step reports GAP_ECAP
    _say("case: photon store overflow (cap 3000)")
    cfg = dict(TINY, n_cells=512, cap_photons=3000)
    g = Gap(cfg)
    with pytest.raises(G.GapError) as ei:
        for _ in range(6):
            g.step(50)
            g.sync()
    assert ei.value.code == -3
    P = g.photons()
    c = g.counts()
    assert c["n_dropped"] > 0
    assert P.size <= 3000 + 2 * 4 * 1024 + 1024
    g.close()


def test_graph_recapture_while_a_replay_is_in_flight(torch_gpu):
    # one re-sort per 16-step replay flips the store buffers, so the second of
    # two back-to-back replays captures a new graph while the first still
    # runs; the old graph is released only after both streams are idle
    _say("case: back-to-back graph replays that re-capture")
    import torch
    cfg = dict(TINY, n_cells=512)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ga = Gap(cfg, stream=s)
        ga.set_launch(8, 16, 64, 16)
        for _ in range(4):
            ga.step_graph(16)
        ga.sync()
        gb = Gap(cfg, stream=s)
        gb.step(64)
        A, B = by_id(gpu_leptons_as_oracle(ga.leptons())), by_id(gpu_leptons_as_oracle(gb.leptons()))
        for k in ("cell", "xi", "u", "w", "id"):
            assert np.array_equal(A[k], B[k]), k
        assert np.array_equal(ga.field(), gb.field())
        assert ga.counts()["err"] == 0
        ga.close()
        gb.close()


def test_state_change_ends_the_cold_window(torch_gpu):
    # Photons of x = 10 born at step 0 in a frozen zero field: their
    # conversion probability is about 2e-27 at age 41, so the re-sort (every
    # 40 steps) classes them as unable to draw before the next one; at age
    # ~1000 it is about 0.15 per step.  Mid-window, jump the step index by
    # 1000: the state change must end that classification (the photon pass
    # then takes every probability), and the next steps equal those of a
    # fresh handle loaded with the same state and step, whose re-sort
    # classifies from scratch.
    _say("case: step index jump mid re-sort window, 1e5 photons of x = 10")
    from paper_2608_21920_amd.inputs import LEPTON_DTYPE, PHOTON_DTYPE
    N, n = 8192, 100_000
    cfg = dict(n_cells=N, init_kind=2, b=0.1, r_curv_cm=1e7, lambda_c_scale=1.7e5, r_curv_scale=1.4e-5,
               h_gap_frac=1.0, flags=G.FIELD_FROZEN | G.EMIT_OFF, seed=9, cap_photons=1 << 20, cap_leptons=1 << 21,
               rebucket_every=40)
    P = np.zeros(n, PHOTON_DTYPE)
    P["cell"] = np.arange(n) % 64
    P["x"], P["w"], P["n0"] = 10.0, 1.0, 0
    P["id"] = np.arange(1, n + 1, dtype=np.uint64) * np.uint64(2654435761)
    g = Gap(cfg)
    g.set_particles(np.zeros(0, LEPTON_DTYPE), P)
    g.set_field(np.zeros(N, np.float32), 0.0)
    g.step(5)
    c0 = g.counts()
    assert c0["n_conv"] == 0 and c0["n_pho"] == n
    L0, P0, es = g.leptons(), g.photons(), g.es()
    jump = c0["step"] + 1000
    g.set_es_step(es, jump)
    h = Gap(cfg)
    h.set_particles(L0, P0)
    h.set_field(np.zeros(N, np.float32), es)
    h.set_es_step(es, jump)
    hc0 = h.counts()
    g.step(10)
    h.step(10)
    ga, ha = g.counts(), h.counts()
    assert ga["err"] == 0 and ha["err"] == 0
    _say("  conversions after the jump: %d" % (ga["n_conv"] - c0["n_conv"]))
    assert ga["n_conv"] - c0["n_conv"] > 1000
    for k in ("n_conv", "n_pho_exit", "n_conv_eval"):
        assert ga[k] - c0[k] == ha[k] - hc0[k], k
    A, B = by_id(gpu_leptons_as_oracle(g.leptons())), by_id(gpu_leptons_as_oracle(h.leptons()))
    for k in ("cell", "xi", "u", "w", "id"):
        assert np.array_equal(A[k], B[k]), k
    A, B = by_id(gpu_photons_as_oracle(g.photons())), by_id(gpu_photons_as_oracle(h.photons()))
    for k in ("cell", "xi", "x", "w", "n0", "id"):
        assert np.array_equal(A[k], B[k]), k
    g.close()
    h.close()
