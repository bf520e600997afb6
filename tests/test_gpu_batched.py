"""Batched form: an ensemble of uneven tubes in one set of launches, captured
in a graph, with launch shapes from the autotuner; every tube's state is
bitwise that of a plain single-tube run."""
import sys

import numpy as np
import pytest

from paper_2608_21920_amd import Gap, workloads

from gpu_util import by_id, gpu_leptons_as_oracle

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


def _same(ga, ta, gb, tb):
    A, B = by_id(gpu_leptons_as_oracle(ga.leptons(ta))), by_id(gpu_leptons_as_oracle(gb.leptons(tb)))
    for k in ("cell", "xi", "u", "w", "id"):
        assert np.array_equal(A[k], B[k]), k
    assert np.array_equal(ga.field(ta), gb.field(tb))
    assert ga.es(ta) == gb.es(tb)


def test_autotune_changes_no_result(torch_gpu):
    _say("case: autotune on the tiny gap")
    cfg = dict(workloads.TINY, n_cells=512)
    a = Gap(cfg)
    a.step(40)
    ch = a.autotune(8)
    _say("  chosen", ch)
    assert ch["grid_leptons"] % 8 == 0 and ch["grid_photons"] % 8 == 0 and ch["resort_every"] >= 4
    n = a.counts()["step"]
    a.step(30)
    b = Gap(cfg)
    b.step(n + 30)
    _same(a, 0, b, 0)
    assert a.counts()["err"] == 0
    a.close()
    b.close()


def test_ensemble_graph_equals_single_tubes(torch_gpu):
    import torch
    _say("case: 12-tube ensemble from the batched recipe, graph replays vs single tubes")
    cfgs = [dict(c, n_cells=c["n_cells"] // 8, cap_leptons=c["cap_leptons"] // 8, cap_photons=c["cap_photons"] // 8)
            for c in workloads.batched_tubes(12, seed=1)]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        gb = Gap(cfgs, stream=s)
        gb.autotune(4)
        n0 = gb.counts(0)["step"]
        for _ in range(3):
            gb.step_graph(20)
            gb.sync()
        steps = gb.counts(0)["step"]
        assert steps == n0 + 60
        for t in (0, 5, 11):
            g1 = Gap(cfgs[t], stream=s)
            g1.step(steps)
            _same(gb, t, g1, 0)
            g1.close()
        assert gb.counts(0)["err"] == 0
        gb.close()


def test_launch_shapes_change_no_result(torch_gpu):
    from paper_2608_21920_amd import gap as G
    _say("case: explicit launch shapes on the tiny gap")
    cfg = dict(workloads.TINY, n_cells=512)
    a, b = Gap(cfg), Gap(cfg)
    a.set_launch(8, 16, 64, 5)
    a.step(70)
    b.step(70)
    _same(a, 0, b, 0)
    for bad in ((0, 16, 64, 5), (12, 16, 64, 5), (8, 16, 64, 0), (8, 16, 64, 100000), (8, 1 << 20, 64, 5)):
        with pytest.raises(G.GapError):
            a.set_launch(*bad)
    a.close()
    b.close()


def test_autotune_keeps_the_drift_bound(torch_gpu):
    # the tuning trials leave many steps since the last re-sort when the
    # re-sort interval candidates are tried; those steps must count toward
    # the next re-sort (else particles drift out of their tile windows and
    # the library reports GAP_ETILE)
    _say("case: autotune with 16-step trials on the tiny gap")
    g = Gap(dict(workloads.TINY))
    g.step(50)
    ch = g.autotune(16)
    _say("  chosen", ch)
    g.step(20)
    g.sync()
    assert g.counts()["err"] == 0
    g.close()


def test_launch_shape_sweep_recaptures_equal_single_tubes(torch_gpu):
    """The batched launch-shape sweep as a regression test of the graph
    lifecycle: eight cycles of a new launch shape (which drops the captured
    graph), then two replays whose length holds one re-sort, so the store
    parity flips and each replay captures a new graph while the previous
    replay may still run, then eager steps and reads.  Every tube must equal
    a single-tube run of the same number of eager steps, bitwise."""
    import torch
    _say("case: 6-tube ensemble, 8 launch-shape cycles with re-capture")
    cfgs = [dict(c, n_cells=c["n_cells"] // 8, cap_leptons=c["cap_leptons"] // 8, cap_photons=c["cap_photons"] // 8)
            for c in workloads.batched_tubes(6, seed=1)]
    shapes = [(256, 512, 512, 68), (512, 256, 1024, 34), (1024, 1024, 256, 136), (256, 256, 256, 17),
              (512, 1024, 512, 68), (1024, 512, 1024, 34), (256, 1024, 256, 136), (512, 512, 512, 40)]
    s = torch.cuda.Stream()
    total = 0
    with torch.cuda.stream(s):
        gb = Gap(cfgs, stream=s)
        for cyc, shp in enumerate(shapes):
            _say("  cycle %d shape %s" % (cyc, shp))
            gb.set_launch(*shp)
            n = shp[3] + (cyc & 1)
            gb.step_graph(n)
            gb.step_graph(n)
            gb.step(3)
            total += 2 * n + 3
            c = gb.counts(cyc % len(cfgs))
            assert c["err"] == 0 and c["step"] == total
        gb.sync()
        for t in (0, 3, 5):
            g1 = Gap(cfgs[t], stream=s)
            g1.step(total)
            _same(gb, t, g1, 0)
            g1.close()
        gb.close()


def _qed_active(cfg):
    """A tube of the batched recipe at its own size, with the tiny gap's QED
    rescale so that emission, transport and conversion all run within 100
    steps."""
    # photon store as large as the lepton store: the QED-active tube makes
    # more photons than the recipe's physical run is sized for, and a cap
    # reached on one side only would split the two runs
    cap = max(cfg["cap_leptons"], 1 << 20)
    return dict(cfg, lambda_c_scale=workloads.TINY["lambda_c_scale"], r_curv_scale=workloads.TINY["r_curv_scale"],
                cap_leptons=cap, cap_photons=cap)


def test_batched_tubes_match_the_oracle(torch_gpu):
    """Tubes of the 256-tube recipe, at full size, stepped together in one
    handle (concatenated launches), against the FP64 oracle run of each tube
    alone: the field within 1e-5 of max|E| at every one of 100 steps, the
    Monte Carlo counts equal up to FP32/FP64 near-ties, and the photons by
    id.  QED-active: 1e4-1e5 emissions and 1e3 conversions per tube."""
    from oracle.oracle import Oracle
    from gpu_util import gpu_photons_as_oracle, rel_field_err
    recipe = workloads.batched_tubes(256, seed=1)
    pick = (76, 3, 109)                 # the three smallest of the recipe
    cfgs = [_qed_active(recipe[i]) for i in pick]
    _say("case: batched tubes %s vs the oracle, 100 steps" % (pick,))
    g = Gap(cfgs)
    orcs = [Oracle(c) for c in cfgs]
    worst = [0.0] * len(cfgs)
    for n in range(100):
        g.step(1)
        for t, o in enumerate(orcs):
            o.step(1)
            err = rel_field_err(g.field(t), o.field())
            worst[t] = max(worst[t], err)
            assert err <= 1e-5, (pick[t], n, err)
    for t, o in enumerate(orcs):
        cg, co = g.counts(t), o.counts()
        _say("  tube %d: worst field err %.2e; emit %d/%d born %d/%d conv %d/%d leptons %d/%d" % (
            pick[t], worst[t], cg["n_emit"], co["n_emit"], cg["n_pho_born"], co["n_pho_born"], cg["n_conv"],
            co["n_conv"], cg["n_lep"], co["n_lep"]))
        assert cg["err"] == 0 and co["err"] == 0
        assert cg["n_dropped"] == 0 and co["n_dropped"] == 0
        assert co["n_emit"] > 10000 and co["n_conv"] > 500
        for k in ("n_emit", "n_pho_born", "n_conv"):
            assert abs(cg[k] - co[k]) <= max(2, 1e-3 * co[k]), (pick[t], k)
        assert abs(cg["n_lep"] - co["n_lep"]) <= max(4, 2e-3 * co["n_lep"])
        assert abs(g.es(t) - o.Es) <= 1e-9 * max(1.0, abs(o.Es))
        P, Q = by_id(gpu_photons_as_oracle(g.photons(t))), by_id(o.photons())
        common, ia, ib = np.intersect1d(P["id"], Q["id"], return_indices=True)
        assert common.size >= 0.998 * max(P["id"].size, Q["id"].size)
        assert np.all(P["n0"][ia] == Q["n0"][ib])
        # energies within the table accuracy, except photons of leptons whose
        # history split at an FP32/FP64 near-tie (a draw on the other side of
        # u < p changes the lepton's later momentum and so its later photons)
        rel = np.abs(P["x"][ia] - Q["x"][ib]) / np.abs(Q["x"][ib])
        _say("  tube %d: %d common photons, %d outside 2e-4, median rel %.1e" % (
            pick[t], common.size, int((rel > 2e-4).sum()), float(np.median(rel))))
        for k in np.argsort(rel)[-3:]:
            _say("    n0 %d x gpu %.7e oracle %.7e" % (Q["n0"][ib[k]], P["x"][ia[k]], Q["x"][ib[k]]))
        assert (rel > 2e-4).sum() <= max(4, 2e-3 * common.size)
        assert np.median(rel) <= 1e-6
    g.close()
