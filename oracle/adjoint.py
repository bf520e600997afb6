"""FP64 adjoint of the particle loop over a window with the QED events frozen.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): only ``tests/``, the
smoke check and the CPU-baseline leg of the benchmark may import it.

The window map.  From a given state (leptons, photons, E_s, injection
counters) the oracle's step (``oracle.c``) is applied W times with the QED
realisation frozen: the nominal window records its events, and every other
evaluation of the map replays them.  In the frozen map every QED effect is
an exogenous source: a recorded emission is a constant signed recoil offset
on its lepton, a recorded photon birth puts the recorded photon state into
the store, and a recorded conversion turns the (then parameter-independent)
photon into its pair.  The injection count per step does not depend on the
injected weight (``INJ_FIXED``), so the injected charge density
n_inj = inj_rate * inj_weight enters through the weights only.

Loss (time-averaged field energy density over the window):
    L = 1/(W N) sum_{m=1..W} sum_k (E^{n0+m}_{k+1/2})^2 .

Derivatives of the map (Sect. 2.2 field equations, Sect. 4 push), with the
fixed-point rounding of the deposit taken as the identity (a particle of
signed weight w at x = k + xi puts w (1 - xi) on node k and w xi on node
k + 1):
  * Gauss integration: E_{j+1/2} = E_s + w0 sum_{i<=j} rho_i - background,
    so dE_{j+1/2}/dxi = -w0 w [j = k] and dE_{j+1/2}/dw = w0 (1 - xi) [j = k]
    + w0 [j > k];
  * surface field: E_s^{n+1} = E_s^n + w0 (sum of absorbed w + injected
    |w|) + alpha s_co dt;
  * gather E_p = (1 - xi) Eb_k + xi Eb_{k+1}, node field Eb_i = (E_{i-1/2} +
    E_{i+1/2}) / 2 with ghosts E_{-1/2} = E_s, E_{N+1/2} = E_{N-1/2};
  * kick u' = u + sign(w) E_p dt; recoil u'' = u' - x with x frozen
    (du''/du' = 1);
  * drift xi' = xi + cfl u'' / sqrt(1 + u''^2)  (cells);
  * photons and pairs born inside the window are constants of the map.
Absorption and outflow are events of the frozen map: an absorbed lepton
passes its weight to E_s, an outflowing one leaves the box.
"""
from __future__ import annotations

import numpy as np

from .oracle import FLAGS, Oracle, philox

INJ_ID_BASE = 1 << 62
TAG_INJ, TAG_CHILD = 4, 6


def _draw(seed: int, ident: int, step: int, tag: int, sub: int):
    return philox([ident & 0xFFFFFFFF, ident >> 32, step & 0xFFFFFFFF, (tag << 16) | (sub & 0xFFFF)],
                  [seed & 0xFFFFFFFF, seed >> 32])


def child_id(seed: int, parent: int, step: int, j: int) -> int:
    r = _draw(seed, parent, step, TAG_CHILD, j)
    return r[0] | (r[1] << 32)


def _index(ids: np.ndarray):
    order = np.argsort(ids, kind="stable")
    return ids[order], order


def _find(sorted_ids, order, q):
    """Index of each id of q in the array the sorted view came from, -1 if absent."""
    q = np.asarray(q, dtype=np.uint64)
    if sorted_ids.size == 0:
        return np.full(q.shape, -1, np.int64)
    pos = np.minimum(np.searchsorted(sorted_ids, q), sorted_ids.size - 1)
    return np.where(sorted_ids[pos] == q, order[pos], -1)


class Window:
    """The oracle run over W steps from `state` (or from its own initial state),
    recording (or, with `events`, replaying) the QED realisation and keeping
    the state before every step and after the last."""

    def __init__(self, cfg: dict, W: int, state: dict | None = None, events: dict | None = None,
                 keep: bool = True):
        flags = int(cfg.get("flags", 0)) | FLAGS["INJ_FIXED"]
        flags |= FLAGS["REPLAY"] if events is not None else FLAGS["RECORD"]
        self.cfg = dict(cfg, flags=flags)
        o = Oracle(self.cfg)
        if state is not None:
            o.set_state(state["L"], state.get("P"), Es=state["Es"], step=state["step"])
            o.set_injection(state.get("inj_acc", 0.0), state.get("inj_count", 0))
        if events is not None:
            o.set_replay(events)
        self.o, self.W = o, W
        self.N, self.dt, self.w0, self.s_co = o.N, o.dt, o.w0, o.s_co
        self.snaps = []
        loss = 0.0
        for _ in range(W):
            if keep:
                self.snaps.append(self._snap())
            o.step(1)
            E = o.field()
            loss += float(np.dot(E, E))
        if keep:
            self.snaps.append(self._snap())
        self.loss = loss / (W * self.N)
        self.events = o.events() if events is None else events

    def _snap(self) -> dict:
        o = self.o
        c = o.counts()
        return dict(L=o.leptons(), P=o.photons(), Eb=o.node_field(), E=o.field(), Es=o.Es,
                    step=c["step"], n_inj=c["n_injected"])


def export_state(o: Oracle) -> dict:
    """The oracle's state in the form Window takes (injection accumulator
    restarted at zero with the current count)."""
    c = o.counts()
    return dict(L=o.leptons(), P=o.photons(), Es=o.Es, step=c["step"], inj_acc=0.0, inj_count=c["n_injected"])


def adjoint(win: Window) -> dict:
    """Reverse pass over a recorded window: loss, dL/dalpha, dL/d(inj_weight)
    and dL/dn_inj (n_inj = inj_rate * inj_weight at a fixed count schedule)."""
    cfg = win.cfg
    N, dt, w0, s_co, W = win.N, win.dt, win.w0, win.s_co, win.W
    cfl = float(cfg.get("cfl", 0.45))
    seed = int(cfg.get("seed", 0))
    inj_w = float(cfg.get("inj_weight", 1.0))
    norm = 1.0 / (W * N)
    S = win.snaps

    LB = S[W]["L"]
    lam_xi, lam_u, lam_w = np.zeros(LB["id"].size), np.zeros(LB["id"].size), np.zeros(LB["id"].size)
    lamE = 2.0 * norm * S[W]["E"]
    lamEs = 0.0
    d_alpha = 0.0
    d_injw = 0.0

    for j in range(W - 1, -1, -1):
        A, B = S[j], S[j + 1]
        n = A["step"]
        LA, LB = A["L"], B["L"]
        sLB, oLB = _index(LB["id"])

        # (1) field after the step: E(B) from E_s(B) and B's leptons (pairs
        # born in this step are neutral and constants: their lambdas are
        # dropped below)
        lamEs += float(lamE.sum())
        suf = np.zeros(N + 1)
        suf[:N] = np.cumsum(lamE[::-1])[::-1]
        k, xi, w = LB["cell"].astype(np.int64), LB["xi"], LB["w"]
        lam_xi = lam_xi + (-w0 * w * lamE[k])
        lam_w = lam_w + w0 * ((1.0 - xi) * lamE[k] + suf[k + 1])
        d_alpha += lamEs * s_co * dt

        # (2) leptons pushed in step n: A's, then the ones injected at step n
        inj_ids = np.arange(A["n_inj"], B["n_inj"], dtype=np.uint64) + np.uint64(INJ_ID_BASE)
        inj_xi = np.array([(_draw(seed, int(i), n, TAG_INJ, 0)[0] >> 8) / 16777216.0 for i in inj_ids])
        ids = np.concatenate([LA["id"], inj_ids])
        cell = np.concatenate([LA["cell"].astype(np.int64), np.zeros(inj_ids.size, np.int64)])
        xi0 = np.concatenate([LA["xi"], inj_xi])
        wt = np.concatenate([LA["w"], np.full(inj_ids.size, -inj_w)])
        Eb = A["Eb"]
        sg = np.where(wt < 0, -1.0, 1.0)
        ia = _find(sLB, oLB, ids)
        alive = ia >= 0
        ia_c = np.where(alive, ia, 0)
        l_xi1 = np.where(alive, lam_xi[ia_c], 0.0)
        l_u2 = np.where(alive, lam_u[ia_c], 0.0)
        l_w = np.where(alive, lam_w[ia_c], 0.0)
        absorbed = (~alive) & (cell < N // 2)
        l_w = l_w + np.where(absorbed, lamEs * w0, 0.0)
        upp = np.where(alive, LB["u"][ia_c], 0.0)
        g2 = np.sqrt(1.0 + upp * upp)
        l_u1 = l_u2 + l_xi1 * cfl / g2 ** 3
        l_Ep = sg * dt * l_u1
        l_xi = l_xi1 + l_Ep * (Eb[cell + 1] - Eb[cell])
        lamEb = np.zeros(N + 1)
        np.add.at(lamEb, cell, (1.0 - xi0) * l_Ep)
        np.add.at(lamEb, cell + 1, xi0 * l_Ep)
        nA = LA["id"].size
        d_injw += float(np.sum(-l_w[nA:])) + inj_ids.size * lamEs * w0

        # (3) node field -> cell field and surface field of A
        lamE = np.zeros(N)
        lamE[:N - 1] = 0.5 * (lamEb[:N - 1] + lamEb[1:N])
        lamE[N - 1] = 0.5 * lamEb[N - 1] + lamEb[N]
        lamEs += 0.5 * lamEb[0]
        if j >= 1:
            lamE += 2.0 * norm * A["E"]
        lam_xi, lam_u, lam_w = l_xi[:nA], l_u1[:nA], l_w[:nA]

    inj_rate = float(cfg.get("inj_rate", 0.0))
    return dict(loss=win.loss, dL_dalpha=d_alpha, dL_dinjw=d_injw,
                dL_dninj=(d_injw / inj_rate if inj_rate > 0 else 0.0))


def finite_differences(cfg: dict, W: int, state: dict | None, events: dict, h: float = 1e-4) -> dict:
    """Central differences of the frozen map's loss: alpha +- h, and
    n_inj +- h through the injected weight (count schedule fixed)."""
    def loss(**kw):
        return Window(dict(cfg, **kw), W, state, events=events, keep=False).loss
    a = float(cfg.get("alpha", 1.5))
    out = dict(dL_dalpha=(loss(alpha=a + h) - loss(alpha=a - h)) / (2 * h))
    rate = float(cfg.get("inj_rate", 0.0))
    if rate > 0:
        w = float(cfg.get("inj_weight", 1.0))
        # n_inj = rate * w; the step in w is put on the 2^-24 grid of the
        # fixed-point charge, so that every injected particle's quantised
        # charge moves by exactly the same amount
        dw = max(1.0, round(h / rate * 16777216.0)) / 16777216.0
        out["dL_dninj"] = (loss(inj_weight=w + dw) - loss(inj_weight=w - dw)) / (2 * dw * rate)
    return out
