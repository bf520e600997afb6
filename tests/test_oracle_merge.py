"""The oracle's weight-doubling merge, pinned by a brute-force restatement.

The paper has no merge: it is the cap-keeping step of this build (reading
R14).  What it must do is written out here a second time, in plain Python
loops that share nothing with the oracle but its Philox routine (itself
pinned by the published known-answer vectors):

* leptons are grouped by (cell, charge sign, direction of motion,
  floor(log2 gamma)), photons by (cell, direction, floor(log2 |x|));
* within a group, particles are taken in increasing id order and fused in
  consecutive pairs (an odd one out is left alone);
* of each pair (a, b), a the smaller id, the keeper is b if bit 0 of the
  first word of Philox(counter = (id_a lo, id_a hi, step, MERGE tag << 16),
  key = seed) is set, else a; it takes the summed weight and keeps its own
  position and momentum.

floor(log2 v) is found by walking exact powers of two, not by frexp, and
gamma = sqrt(1 + u^2) is formed with the same two IEEE operations on both
sides, so a bin decision at a power of two is the same comparison.  The
state is ragged (odd group sizes, empty cells, momenta on both sides of
every power of two from 2^-6 to 2^20, |u| < 1 where log2|u| and log2 gamma
part ways), so that a wrong key, a wrong pairing order or a wrong keeper
rule changes the result: the variants below are planted in the brute force
and must disagree with the oracle.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O

F = O.FLAGS
TAG_MERGE = 5
SEED = 0x9E3779B97F4A7C15
STEP = 777


def _floor_log2(v):
    """floor(log2 v) for v > 0 by walking exact powers of two."""
    b = 0
    if v >= 1.0:
        while 2.0 ** (b + 1) <= v:
            b += 1
    else:
        while 2.0 ** b > v:
            b -= 1
    return b


def _gamma(u):
    return math.sqrt(1.0 + u * u)


def lepton_key(c, u, w):
    return (int(c), w > 0, u >= 0, _floor_log2(_gamma(u)))


def photon_key(c, x):
    return (int(c), x >= 0, _floor_log2(abs(x)))


def _keeper_b(id_a, step, seed=SEED):
    r = O.philox([id_a & 0xFFFFFFFF, id_a >> 32, step & 0xFFFFFFFF, TAG_MERGE << 16],
                 [seed & 0xFFFFFFFF, seed >> 32])
    return (r[0] & 1) == 1


def brute_merge(keys, ids, w, step, order="id", keeper=_keeper_b):
    """Survivors {id: weight} of one merge, written out with dicts and loops."""
    groups = {}
    for i, k in enumerate(keys):
        groups.setdefault(k, []).append(i)
    w = [float(v) for v in w]
    alive = [True] * len(w)
    for members in groups.values():
        if order == "id":
            members = sorted(members, key=lambda i: int(ids[i]))
        for j in range(0, len(members) - 1, 2):
            a, b = members[j], members[j + 1]
            keep, drop = (b, a) if keeper(int(ids[a]), step) else (a, b)
            w[keep] += w[drop]
            alive[drop] = False
    return {int(ids[i]): w[i] for i in range(len(w)) if alive[i]}


def _ragged_state(seed=5, nl=7000, npho=5000, N=48):
    rng = np.random.default_rng(seed)
    # cells: a few crowded, some sparse, some empty
    cells = rng.choice(np.arange(N), nl, p=np.r_[np.full(8, 0.06), np.full(N - 16, 0.52 / (N - 16)),
                                                  np.zeros(8)])
    # |u| around every power of two from 2^-6 to 2^20, plus a log-uniform spread
    pw = 2.0 ** rng.integers(-6, 21, nl)
    mag = np.where(rng.random(nl) < 0.5, pw * (1.0 + rng.choice([-1, 1], nl) * 1e-9),
                   np.exp(rng.uniform(-5, 14, nl)))
    u = rng.choice([-1.0, 1.0], nl) * mag
    # gamma exactly at a power of two for a few: u = sqrt(4^k - 1)
    k = rng.integers(1, 12, 200)
    u[:200] = np.sqrt(4.0 ** k - 1.0) * rng.choice([-1, 1], 200)
    w = rng.choice([-1.0, 1.0], nl) * rng.choice([1.0, 2.0, 0.5], nl, p=[0.7, 0.2, 0.1])
    ids = np.unique(rng.integers(1, 1 << 62, nl + npho + 64, dtype=np.int64).astype(np.uint64))
    ids = rng.permutation(ids)[:nl + npho]
    ids[::7] |= np.uint64(1 << 63)           # ids above 2^63 too
    lep = dict(cell=cells.astype(np.int32), xi=rng.random(nl), u=u, w=w, id=ids[:nl])
    pc = rng.integers(0, N, npho)
    pm = np.where(rng.random(npho) < 0.5, 2.0 ** rng.integers(1, 26, npho) * (1.0 + 1e-9 * rng.choice([-1, 1], npho)),
                  np.exp(rng.uniform(0.7, 17, npho)))
    pho = dict(cell=pc.astype(np.int32), xi=rng.random(npho), x=rng.choice([-1.0, 1.0], npho) * pm,
               w=rng.choice([1.0, 2.0], npho), n0=rng.integers(0, STEP, npho), id=ids[nl:])
    return lep, pho, N


def _oracle_merged(lep, pho, N):
    o = O.Oracle(dict(n_cells=N, init_kind=2, flags=F["QED_OFF"] | F["FIELD_FROZEN"] | F["MERGE_ON"] | F["PERIODIC"],
                      cap_leptons=1 << 20, cap_photons=1 << 20, merge_frac=0.5, merge_every=1, alpha=0.0, seed=SEED))
    o.set_state(lep, pho, Es=0.0, step=STEP)
    o.merge_now()
    return o


@pytest.fixture(scope="module")
def merged():
    lep, pho, N = _ragged_state()
    o = _oracle_merged(lep, pho, N)
    return lep, pho, N, o.leptons(), o.photons(), o.counts()


def _as_map(d):
    return {int(i): float(w) for i, w in zip(d["id"], d["w"])}


def test_lepton_merge_equals_brute_force(merged):
    lep, _, _, L, _, c = merged
    keys = [lepton_key(*t) for t in zip(lep["cell"], lep["u"], lep["w"])]
    want = brute_merge(keys, lep["id"], lep["w"], STEP)
    assert _as_map(L) == want
    # survivors keep their own position and momentum
    src = {int(i): (int(c_), x, u) for i, c_, x, u in zip(lep["id"], lep["cell"], lep["xi"], lep["u"])}
    for i, c_, x, u in zip(L["id"], L["cell"], L["xi"], L["u"]):
        assert src[int(i)] == (int(c_), x, u)
    assert c["n_merged"] == lep["id"].size - L["id"].size + (len(pho_ids_merged(merged)))


def pho_ids_merged(merged):
    _, pho, _, _, P, _ = merged
    return set(int(i) for i in pho["id"]) - set(int(i) for i in P["id"])


def test_photon_merge_equals_brute_force(merged):
    _, pho, _, _, P, _ = merged
    keys = [photon_key(c, x) for c, x in zip(pho["cell"], pho["x"])]
    want = brute_merge(keys, pho["id"], pho["w"], STEP)
    assert _as_map(P) == want
    src = {int(i): (int(c), x, xi, n0) for i, c, x, xi, n0 in zip(pho["id"], pho["cell"], pho["x"], pho["xi"], pho["n0"])}
    for i, c, x, xi, n0 in zip(P["id"], P["cell"], P["x"], P["xi"], P["n0"]):
        assert src[int(i)] == (int(c), x, xi, int(n0))


def test_charge_kept_per_cell_and_species(merged):
    lep, pho, N, L, P, _ = merged
    for s in (-1.0, 1.0):
        before = np.bincount(lep["cell"], weights=np.where(np.sign(lep["w"]) == s, lep["w"], 0.0), minlength=N)
        after = np.bincount(L["cell"], weights=np.where(np.sign(L["w"]) == s, L["w"], 0.0), minlength=N)
        assert np.array_equal(before, after)
    assert np.array_equal(np.bincount(pho["cell"], weights=pho["w"], minlength=N),
                          np.bincount(P["cell"], weights=P["w"], minlength=N))
    # the merge did real work in most groups
    assert L["id"].size < 0.75 * lep["id"].size and P["id"].size < 0.75 * pho["id"].size


# Planted mistakes: each would be a plausible misreading of the key or the
# pairing; the state above must expose every one of them.
_LEP_VARIANTS = {
    "direction dropped": lambda c, u, w: (int(c), w > 0, _floor_log2(_gamma(u))),
    "charge sign dropped": lambda c, u, w: (int(c), u >= 0, _floor_log2(_gamma(u))),
    "log2|u| for log2 gamma": lambda c, u, w: (int(c), w > 0, u >= 0, _floor_log2(abs(u))),
    "cell >> 1": lambda c, u, w: (int(c) >> 1, w > 0, u >= 0, _floor_log2(_gamma(u))),
    "round(log2 gamma)": lambda c, u, w: (int(c), w > 0, u >= 0, round(math.log2(_gamma(u)))),
}


@pytest.mark.parametrize("name", sorted(_LEP_VARIANTS))
def test_wrong_lepton_keys_are_detected(merged, name):
    lep, _, _, L, _, _ = merged
    keys = [_LEP_VARIANTS[name](*t) for t in zip(lep["cell"], lep["u"], lep["w"])]
    assert brute_merge(keys, lep["id"], lep["w"], STEP) != _as_map(L)


def test_wrong_pairing_and_keeper_are_detected(merged):
    lep, _, _, L, _, _ = merged
    keys = [lepton_key(*t) for t in zip(lep["cell"], lep["u"], lep["w"])]
    got = _as_map(L)
    assert brute_merge(keys, lep["id"], lep["w"], STEP, order="slot") != got
    assert brute_merge(keys, lep["id"], lep["w"], STEP, keeper=lambda i, s: not _keeper_b(i, s)) != got
    assert brute_merge(keys, lep["id"], lep["w"], STEP + 1) != got


@pytest.mark.parametrize("name", ["direction dropped", "log2 x rounded", "cell >> 1"])
def test_wrong_photon_keys_are_detected(merged, name):
    _, pho, _, _, P, _ = merged
    var = {"direction dropped": lambda c, x: (int(c), _floor_log2(abs(x))),
           "log2 x rounded": lambda c, x: (int(c), x >= 0, round(math.log2(abs(x)))),
           "cell >> 1": lambda c, x: (int(c) >> 1, x >= 0, _floor_log2(abs(x)))}[name]
    keys = [var(c, x) for c, x in zip(pho["cell"], pho["x"])]
    assert brute_merge(keys, pho["id"], pho["w"], STEP) != _as_map(P)


def test_floor_log2_walk():
    for v, b in [(1.0, 0), (1.9999999, 0), (2.0, 1), (3.0, 1), (0.5, -1), (0.49, -2), (2.0 ** 40, 40),
                 (2.0 ** 40 * (1 - 1e-15), 39)]:
        assert _floor_log2(v) == b


# Whole-step properties through the normal step path (merge at the start of
# the step, then the push).
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


def test_merge_in_a_step_halves_and_keeps_total_charge():
    lep = _state()
    o = _run(lep)
    o.step(1)
    L = o.leptons()
    assert o.counts()["n_merged"] > 0
    assert L["w"].size == lep["w"].size - o.counts()["n_merged"]
    assert set(np.abs(L["w"]).tolist()) <= {1.0, 2.0}
    assert abs(L["w"].sum() - lep["w"].sum()) < 1e-12


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
