"""Parity at full size, in the launch configuration that the benchmark
times: the production gap (65536 cells, caps 5e7 per species) and the
full-scale gap (262144 cells, b = 0.2, caps 2e8), each grown by the
simulation itself to 2e7 particles, then stepped by the plain eager path.

 * One step from the grown state on both sides (the oracle loads the GPU's
   whole state, ~2e7 particles): the node charge of the loaded state is
   bit-exact, the field after the step within 1e-5 of max|E| (the field bar
   of the 100-step comparison), E_s to FP64 round-off, and every particle
   (by id) within the FP32-vs-FP64 tolerance of a single step; the node
   charge the lepton pass deposited is bit-exact against the oracle's deposit
   of the GPU's post-step leptons.
 * Counter balance over the step (births, conversions, injection, absorption,
   outflow and exits account for every change of the store sizes) and
   unique ids.
 * Graph replay of 20 steps on a second handle loaded with the same state
   (its stores re-sorted from scratch) equals 20 eager steps bitwise.
"""
import sys

import numpy as np
import pytest

from paper_2608_21920_amd import Gap, workloads
from paper_2608_21920_amd.inputs import leptons_as_oracle, photons_as_oracle
from oracle.oracle import Oracle

from gpu_util import by_id, rel_field_err

pytestmark = pytest.mark.gpu

GROW_TO = 2.0e7
WORKLOADS = {"production": workloads.PRODUCTION, "full": workloads.FULL}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", params=sorted(WORKLOADS))
def grown(request):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cfg = dict(WORKLOADS[request.param])
    _say("case: %s gap (%d cells) grown to %.0e particles" % (request.param, cfg["n_cells"], GROW_TO))
    s = torch.cuda.Stream()
    g = Gap(cfg, stream=s)
    while True:
        c = g.counts()
        if c["n_lep"] + c["n_pho"] >= GROW_TO:
            break
        assert c["step"] < 200000 and c["err"] == 0
        g.step(2000)
        g.sync()
    _say("  grown: step %d, %d leptons, %d photons" % (c["step"], c["n_lep"], c["n_pho"]))
    yield g, s, cfg
    g.close()


def _match(A, B):
    """Index pairs of equal ids in two id-sorted dicts."""
    _, ia, ib = np.intersect1d(A["id"], B["id"], assume_unique=True, return_indices=True)
    return ia, ib


def test_one_step_from_grown_state_matches_oracle(grown):
    g, _, CFG = grown
    c0 = g.counts()
    n = c0["step"]
    L0, P0 = g.leptons(), g.photons()
    assert L0.size == c0["n_lep"] and P0.size == c0["n_pho"]
    E0, Es0 = g.field(), g.es()
    # the injection accumulator is not exported: give both sides the same one
    g.set_injection(0.0, c0["n_injected"])
    o = Oracle(CFG)
    o.set_state(leptons_as_oracle(L0), photons_as_oracle(P0), Es0, n)
    o.set_injection(0.0, c0["n_injected"])
    _say("  loaded %d + %d particles into the oracle at step %d" % (L0.size, P0.size, n))
    # the GPU's field of the grown state is the exact field of its leptons
    assert np.array_equal(g.rho(), o.rho())
    assert np.array_equal(E0, o.field().astype(np.float32))

    g.step(1)
    o.step(1)
    c1, co = g.counts(), o.counts()
    assert c1["err"] == 0
    d = {k: c1[k] - c0[k] for k in c0}
    ev = max(10, 1e-5 * (c0["n_lep"] + c0["n_pho"]))      # FP32/FP64 near-ties of an event decision
    _say("  gpu: emit %d conv %d inj %d abs %d exit %d; oracle: emit %d conv %d inj %d abs %d exit %d" % (
        d["n_emit"], d["n_conv"], d["n_injected"], d["n_absorbed"], d["n_pho_exit"], co["n_emit"], co["n_conv"],
        co["n_injected"], co["n_absorbed"], co["n_pho_exit"]))
    assert d["n_injected"] == co["n_injected"] - c0["n_injected"]
    assert abs(d["n_emit"] - co["n_emit"]) <= ev and abs(d["n_conv"] - co["n_conv"]) <= ev
    assert abs(c1["n_lep"] - co["n_lep"]) <= 2 * ev and abs(c1["n_pho"] - co["n_pho"]) <= 2 * ev

    # field and surface field
    err = rel_field_err(g.field(), o.field())
    _say("  field rel err %.3e, Es gpu %.12e oracle %.12e" % (err, g.es(), o.Es))
    assert err <= 1e-5
    assert abs(g.es() - o.Es) <= 1e-12 * max(1.0, abs(o.Es))

    # leptons, by id
    A, B = by_id(leptons_as_oracle(g.leptons())), by_id(o.leptons())
    ia, ib = _match(A, B)
    assert ia.size >= max(A["id"].size, B["id"].size) - 2 * ev
    prev = by_id(leptons_as_oracle(L0))
    u_before = np.zeros(ia.size)
    jp, kp = _match({"id": B["id"][ib]}, prev)
    u_before[jp] = prev["u"][kp]
    fresh = np.ones(ia.size, bool)
    fresh[jp] = False                                   # pair children and injected leptons
    pos_err = np.abs((A["cell"][ia] + A["xi"][ia]) - (B["cell"][ib] + B["xi"][ib]))
    du = np.abs(A["u"][ia] - B["u"][ib])
    kick = np.max(np.abs(E0)) * g.derived()["dt"]
    tol_u = np.where(fresh, 1e-6 * np.abs(B["u"][ib]) + 1e-6,
                     1e-6 * (np.abs(B["u"][ib]) + kick) + 3e-4 * np.abs(B["u"][ib] - u_before))
    bad = (pos_err > 1e-5) | (du > tol_u) | (A["w"][ia] != B["w"][ib])
    _say("  leptons: %d matched, %d fresh, %d outside tolerance; max pos err %.2e cells" % (
        ia.size, fresh.sum(), bad.sum(), pos_err.max()))
    assert bad.sum() <= ev

    # photons, by id
    A, B = by_id(photons_as_oracle(g.photons())), by_id(o.photons())
    ia, ib = _match(A, B)
    assert ia.size >= max(A["id"].size, B["id"].size) - 2 * ev
    born = B["n0"][ib] == n + 1
    pos_err = np.abs((A["cell"][ia] + A["xi"][ia]) - (B["cell"][ib] + B["xi"][ib]))
    dx = np.abs(A["x"][ia] - B["x"][ib])
    tol_x = np.where(born, 2e-4 * np.abs(B["x"][ib]), 0.0)
    bad = (pos_err > 1e-5) | (dx > tol_x) | (A["n0"][ia] != B["n0"][ib]) | (A["w"][ia] != B["w"][ib])
    _say("  photons: %d matched, %d born this step, %d outside tolerance" % (ia.size, born.sum(), bad.sum()))
    assert bad.sum() <= ev
    del o

    # the node charge the lepton pass deposited, against the oracle's deposit
    # of the GPU's post-step leptons
    L1 = g.leptons()
    o2 = Oracle(CFG)
    o2.set_state(leptons_as_oracle(L1), None, g.es(), c1["step"])
    assert np.array_equal(g.rho(), o2.rho())
    assert np.array_equal(g.field(), o2.field().astype(np.float32))


def test_counter_balance_and_unique_ids(grown):
    g, _, CFG = grown
    c0 = g.counts()
    g.step(5)
    c1 = g.counts()
    d = {k: c1[k] - c0[k] for k in c0}
    assert c1["err"] == 0 and d["n_dropped"] == 0 and d["n_merged"] == 0
    assert d["n_lep"] == 2 * d["n_conv"] + d["n_injected"] - d["n_absorbed"] - d["n_outflow"]
    assert d["n_pho"] == d["n_pho_born"] - d["n_conv"] - d["n_pho_exit"]
    L, P = g.leptons(), g.photons()
    assert L.size == c1["n_lep"] and P.size == c1["n_pho"]
    assert np.unique(L["id"]).size == L.size and np.unique(P["id"]).size == P.size
    assert np.all((L["frac"] < (1 << 24)) & (L["cell"] >= 0) & (L["cell"] < CFG["n_cells"]))
    assert np.all(np.isfinite(L["u"])) and np.all(np.isfinite(P["x"]))


def test_graph_replay_on_reloaded_state_equals_eager(grown):
    import torch
    g, s, CFG = grown
    c0 = g.counts()
    L0, P0 = g.leptons(), g.photons()
    g.set_injection(0.0, c0["n_injected"])
    with torch.cuda.stream(s):
        h = Gap(CFG, stream=s)
        h.set_particles(L0, P0)
        h.set_es_step(g.es(), c0["step"])
        h.set_injection(0.0, c0["n_injected"])
        assert np.array_equal(h.field(), g.field())
        ch0 = h.counts()
        g.step(20)
        h.step_graph(20)
        h.sync()
        A, B = by_id(leptons_as_oracle(g.leptons())), by_id(leptons_as_oracle(h.leptons()))
        for k in ("cell", "xi", "u", "w", "id"):
            assert np.array_equal(A[k], B[k]), k
        A, B = by_id(photons_as_oracle(g.photons())), by_id(photons_as_oracle(h.photons()))
        for k in ("cell", "xi", "x", "w", "n0", "id"):
            assert np.array_equal(A[k], B[k]), k
        assert np.array_equal(g.field(), h.field())
        assert g.es() == h.es()
        ca, cb = g.counts(), h.counts()
        for k in ("n_lep", "n_pho", "step"):
            assert ca[k] == cb[k], k
        for k in ("n_emit", "n_conv", "n_absorbed", "n_pho_exit", "n_injected"):
            assert ca[k] - c0[k] == cb[k] - ch0[k], k
        h.close()
