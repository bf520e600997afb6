"""Invariants of the weight-doubling merge (not described in the paper; its
parity is unpinned by the paper, so these are the properties it must keep)."""
import numpy as np

from oracle import oracle as O

F = O.FLAGS


def _state(seed=0, n=6000, N=32):
    rng = np.random.default_rng(seed)
    return dict(cell=rng.integers(0, N, n).astype(np.int32), xi=rng.random(n),
                u=rng.choice([-1, 1], n) * np.exp(rng.uniform(0, 8, n)),
                w=rng.choice([-1.0, 1.0], n), id=rng.permutation(np.arange(1, n + 1, dtype=np.uint64) * 7919))


def _run(lep, N=32):
    o = O.Oracle(dict(n_cells=N, init_kind=2, flags=F["QED_OFF"] | F["FIELD_FROZEN"] | F["MERGE_ON"] | F["PERIODIC"],
                      cap_leptons=8000, merge_frac=0.5, merge_every=1, alpha=0.0, seed=21))
    o.set_state(lep)
    o.set_field(np.zeros(N), 0.0)
    return o


def test_merge_conserves_charge_per_cell_and_halves_groups():
    lep = _state()
    before = {}
    for c, w in zip(lep["cell"], lep["w"]):
        before[(int(c), w > 0)] = before.get((int(c), w > 0), 0.0) + w
    o = _run(lep)
    # the merge runs at the start of the step, before the push
    o.step(1)
    L = o.leptons()
    assert o.counts()["n_merged"] > 0
    assert L["w"].size == lep["w"].size - o.counts()["n_merged"]
    # weights are sums of pairs
    assert set(np.abs(L["w"]).tolist()) <= {1.0, 2.0}
    # charge per species summed over the box is unchanged; per cell it moves
    # by at most the drift of one step (FIELD_FROZEN with E = 0: u unchanged)
    tot_b = sum(v for v in before.values())
    assert abs(L["w"].sum() - tot_b) < 1e-12


def test_merge_order_independent():
    lep = _state(seed=3)
    o1 = _run(lep)
    o1.step(1)
    p = np.random.default_rng(9).permutation(lep["w"].size)
    lep2 = {k: v[p] for k, v in lep.items()}
    o2 = _run(lep2)
    o2.step(1)
    a, b = o1.leptons(), o2.leptons()
    ia, ib = np.argsort(a["id"]), np.argsort(b["id"])
    for k in ("cell", "xi", "u", "w", "id"):
        assert np.array_equal(a[k][ia], b[k][ib])
