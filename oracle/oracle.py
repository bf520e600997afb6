"""ctypes binding of ``oracle.c`` (the FP64 CPU oracle; test infrastructure only).

The parameter structure below is this side's own definition; the HIP path
defines its own.  Both follow one written interface (field order and flag
bits), not a shared header.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

FLAGS = dict(
    QED_OFF=1, ETA_CO_OFF=2, FIELD_FROZEN=4, RECOIL_OFF=8, PERIODIC=16, MERGE_ON=32,
    TRACK_ALL=64, ANTI_ALIGNED=128, RECORD=256, REPLAY=512, CONV_OFF=1024, EMIT_OFF=2048, INJ_FIXED=4096,
    FILTER=8192, QUANTUM=16384,
)
FILTER_PASSES = 8


def build_oracle(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math: IEEE FP64)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class OracleParams(C.Structure):
    _fields_ = [
        ("n_cells", C.c_int32), ("init_kind", C.c_int32), ("ppc_init", C.c_int32), ("ppc_ref", C.c_int32),
        ("dx", C.c_double), ("cfl", C.c_double), ("alpha", C.c_double), ("b", C.c_double),
        ("r_curv_cm", C.c_double), ("period_s", C.c_double),
        ("lambda_c_scale", C.c_double), ("r_curv_scale", C.c_double), ("h_gap_frac", C.c_double),
        ("inj_rate", C.c_double), ("inj_weight", C.c_double), ("x_thr", C.c_double),
        ("xc_floor", C.c_double), ("u_init", C.c_double), ("merge_frac", C.c_double),
        ("seed", C.c_uint64), ("cap_leptons", C.c_int64), ("cap_photons", C.c_int64),
        ("flags", C.c_uint32), ("nsub_max", C.c_int32), ("merge_every", C.c_int32), ("pad_", C.c_int32),
        ("atm_temp", C.c_double), ("atm_ppc", C.c_int32), ("pad2_", C.c_int32),
    ]


_DEFAULTS = dict(
    n_cells=1024, init_kind=1, ppc_init=16, ppc_ref=16, dx=0.25, cfl=0.45, alpha=1.5, b=0.1,
    r_curv_cm=1e7, period_s=1.0, lambda_c_scale=1.0, r_curv_scale=1.0, h_gap_frac=0.8,
    inj_rate=0.0, inj_weight=1.0, x_thr=2.0, xc_floor=1e-2, u_init=0.0, merge_frac=0.9,
    seed=0, cap_leptons=1 << 40, cap_photons=1 << 40, flags=0, nsub_max=64, merge_every=64,
    atm_temp=0.3, atm_ppc=0,
)


def make_params(cfg: dict) -> OracleParams:
    p = OracleParams()
    for k, v in _DEFAULTS.items():
        setattr(p, k, v)
    for k, v in cfg.items():
        if k in _DEFAULTS:
            setattr(p, k, v)
    return p


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = C.CDLL(build_oracle())
        P = C.POINTER
        lib.orc_create.restype = C.c_void_p
        lib.orc_create.argtypes = [P(OracleParams), P(C.c_int32)]
        lib.orc_free.argtypes = [C.c_void_p]
        lib.orc_step.restype = C.c_int32
        lib.orc_step.argtypes = [C.c_void_p, C.c_int64]
        lib.orc_derived.argtypes = [C.c_void_p, P(C.c_double)]
        lib.orc_counts.argtypes = [C.c_void_p, P(C.c_int64)]
        lib.orc_es.restype = C.c_double
        lib.orc_es.argtypes = [C.c_void_p]
        lib.orc_erad.restype = C.c_double
        lib.orc_erad.argtypes = [C.c_void_p]
        lib.orc_return.argtypes = [C.c_void_p, C.c_void_p]
        lib.orc_filter.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32]
        for f in ("orc_field", "orc_node_field"):
            getattr(lib, f).argtypes = [C.c_void_p, C.c_void_p]
        lib.orc_rho.argtypes = [C.c_void_p, C.c_void_p]
        lib.orc_get_leptons.argtypes = [C.c_void_p] + [C.c_void_p] * 5
        lib.orc_get_protons.argtypes = [C.c_void_p] + [C.c_void_p] * 5
        lib.orc_set_protons.restype = C.c_int32
        lib.orc_set_protons.argtypes = [C.c_void_p, C.c_int64] + [C.c_void_p] * 5
        lib.orc_proton_counts.argtypes = [C.c_void_p, P(C.c_int64)]
        lib.orc_set_atmosphere.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_uint64]
        lib.orc_atm_momentum.restype = C.c_double
        lib.orc_atm_momentum.argtypes = [C.c_uint64, C.c_uint64, C.c_int64, C.c_double]
        lib.orc_get_photons.argtypes = [C.c_void_p] + [C.c_void_p] * 6
        lib.orc_get_events.argtypes = [C.c_void_p] + [C.c_void_p] * 8
        lib.orc_set_state.restype = C.c_int32
        lib.orc_set_state.argtypes = [C.c_void_p, C.c_int64] + [C.c_void_p] * 5 + [C.c_int64] + \
            [C.c_void_p] * 6 + [C.c_double, C.c_int64]
        lib.orc_set_field.argtypes = [C.c_void_p, C.c_void_p, C.c_double]
        lib.orc_set_injection.argtypes = [C.c_void_p, C.c_double, C.c_uint64]
        lib.orc_merge_now.argtypes = [C.c_void_p]
        lib.orc_set_replay.argtypes = [C.c_void_p, C.c_int64] + [C.c_void_p] * 8
        lib.orc_philox.argtypes = [P(C.c_uint32), P(C.c_uint32), P(C.c_uint32)]
        lib.orc_tsyn.restype = C.c_double
        lib.orc_tsyn.argtypes = [C.c_double]
        lib.orc_tbw.restype = C.c_double
        lib.orc_tbw.argtypes = [C.c_double]
        lib.orc_sync_cdf.restype = C.c_double
        lib.orc_sync_cdf.argtypes = [C.c_double]
        lib.orc_sync_inverse_many.argtypes = [C.c_void_p, C.c_void_p, C.c_int64]
        for name in ("orc_qsyn_T", "orc_qsyn_g", "orc_qbw_T"):
            getattr(lib, name).restype = C.c_double
            getattr(lib, name).argtypes = [C.c_double]
        for name in ("orc_qsyn_cdf", "orc_qsyn_inverse", "orc_qbw_cdf", "orc_qbw_inverse"):
            getattr(lib, name).restype = C.c_double
            getattr(lib, name).argtypes = [C.c_double, C.c_double]
        lib.orc_u24.restype = C.c_double
        lib.orc_u24.argtypes = [C.c_uint32]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def philox(ctr, key):
    """Philox4x32-10 of the oracle: 4 counter words, 2 key words -> 4 words."""
    lib = _load()
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib.orc_philox(c, k, o)
    return [int(v) for v in o]


def u24(r: int) -> float:
    return _load().orc_u24(C.c_uint32(r))


def tsyn(chi: float) -> float:
    return _load().orc_tsyn(chi)


def tbw(chi: float) -> float:
    return _load().orc_tbw(chi)


def atm_momentum(seed: int, pid: int, step: int, theta: float) -> float:
    """Momentum u of an atmosphere particle drawn from the one-dimensional
    relativistic thermal distribution exp(-gamma/Theta) (Sect. 6.1)."""
    return _load().orc_atm_momentum(int(seed), int(pid), int(step), float(theta))


def sync_cdf(xi: float) -> float:
    return _load().orc_sync_cdf(xi)


def sync_inverse(r) -> np.ndarray:
    r = np.ascontiguousarray(np.atleast_1d(r), dtype=np.float64)
    out = np.empty_like(r)
    _load().orc_sync_inverse_many(_ptr(r), _ptr(out), r.size)
    return out


# Quantum-corrected spectra (Sect. 3.1 S(gamma, x) and g_Q; Sect. 3.2 pair
# split): rate functions, Gaunt factor, distribution functions and their
# inverses in FP64.
def qsyn_T(chi: float) -> float:
    """Emission rate function from the quantum photon spectrum."""
    return _load().orc_qsyn_T(float(chi))


def qsyn_g(chi: float) -> float:
    """Gaunt factor g_Q = P_syn / P_classical."""
    return _load().orc_qsyn_g(float(chi))


def qsyn_cdf(chi: float, d) -> np.ndarray:
    """Fraction of emitted photons with energy fraction x/gamma below d."""
    lib = _load()
    return np.array([lib.orc_qsyn_cdf(float(chi), float(v)) for v in np.atleast_1d(d)])


def qsyn_inverse(chi, r) -> np.ndarray:
    """Photon energy fraction d with qsyn_cdf(chi, d) = r (chi scalar or per r)."""
    lib = _load()
    r = np.atleast_1d(np.asarray(r, np.float64))
    c = np.broadcast_to(np.asarray(chi, np.float64), r.shape)
    return np.array([lib.orc_qsyn_inverse(float(a), float(b)) for a, b in zip(c, r)])


def qbw_T(chi: float) -> float:
    """Pair creation rate function from the quantum pair spectrum."""
    return _load().orc_qbw_T(float(chi))


def qbw_cdf(chi: float, v) -> np.ndarray:
    """Fraction of pairs whose electron takes less than the energy fraction v."""
    lib = _load()
    return np.array([lib.orc_qbw_cdf(float(chi), float(x)) for x in np.atleast_1d(v)])


def qbw_inverse(chi, r) -> np.ndarray:
    """Electron energy fraction v with qbw_cdf(chi, v) = r."""
    lib = _load()
    r = np.atleast_1d(np.asarray(r, np.float64))
    c = np.broadcast_to(np.asarray(chi, np.float64), r.shape)
    return np.array([lib.orc_qbw_inverse(float(a), float(b)) for a, b in zip(c, r)])


class Oracle:
    """One simulated flux tube, advanced step by step in FP64."""

    def __init__(self, cfg: dict):
        lib = _load()
        self.cfg = dict(cfg)
        self.p = make_params(cfg)
        err = C.c_int32(0)
        h = lib.orc_create(C.byref(self.p), C.byref(err))
        if not h:
            raise ValueError("oracle rejected the parameters (code %d)" % err.value)
        self.h = h
        self.lib = lib
        d = (C.c_double * 8)()
        lib.orc_derived(h, d)
        self.d_cm, self.lam, self.rc, self.dt, self.H, self.w0, self.s_co = list(d)[:7]
        self.N = int(d[7])

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.orc_free(h)
            self.h = None

    def step(self, n: int = 1) -> int:
        return self.lib.orc_step(self.h, n)

    def counts(self) -> dict:
        o = (C.c_int64 * 16)()
        self.lib.orc_counts(self.h, o)
        keys = ["n_lep", "n_pho", "step", "n_emit", "n_pho_born", "n_conv", "n_absorbed", "n_outflow",
                "n_pho_exit", "n_dropped", "n_merged", "err", "n_events", "n_injected", "n_emit_eval",
                "n_conv_eval"]
        return dict(zip(keys, [int(v) for v in o]))

    @property
    def Es(self) -> float:
        return self.lib.orc_es(self.h)

    @property
    def e_rad(self) -> float:
        return self.lib.orc_erad(self.h)

    def return_spectrum(self) -> np.ndarray:
        """Weight absorbed at h = 0 per 1/8 decade of gamma since the last
        call (which clears it), then the total weight and weight x gamma."""
        out = np.zeros(66, np.float64)
        self.lib.orc_return(self.h, _ptr(out))
        return out

    def field(self) -> np.ndarray:
        E = np.empty(self.N, np.float64)
        self.lib.orc_field(self.h, _ptr(E))
        return E

    def node_field(self) -> np.ndarray:
        E = np.empty(self.N + 1, np.float64)
        self.lib.orc_node_field(self.h, _ptr(E))
        return E

    def rho(self) -> np.ndarray:
        r = np.empty(self.N + 1, np.int64)
        self.lib.orc_rho(self.h, _ptr(r))
        return r

    def leptons(self) -> dict:
        n = self.counts()["n_lep"]
        a = dict(cell=np.empty(n, np.int32), xi=np.empty(n), u=np.empty(n), w=np.empty(n),
                 id=np.empty(n, np.uint64))
        self.lib.orc_get_leptons(self.h, *[_ptr(a[k]) for k in ("cell", "xi", "u", "w", "id")])
        return a

    def proton_counts(self) -> dict:
        o = (C.c_int64 * 8)()
        self.lib.orc_proton_counts(self.h, o)
        keys = ["n_pro", "n_pro_absorbed", "n_pro_outflow", "n_atm_e", "n_atm_p", "atm_prev_e", "atm_prev_p",
                "atm_count"]
        return dict(zip(keys, [int(v) for v in o]))

    def protons(self) -> dict:
        n = self.proton_counts()["n_pro"]
        a = dict(cell=np.empty(n, np.int32), xi=np.empty(n), u=np.empty(n), w=np.empty(n),
                 id=np.empty(n, np.uint64))
        self.lib.orc_get_protons(self.h, *[_ptr(a[k]) for k in ("cell", "xi", "u", "w", "id")])
        return a

    def set_protons(self, pro: dict) -> int:
        A = {k: np.ascontiguousarray(pro[k], dtype=dt) for k, dt in (("cell", np.int32), ("xi", np.float64),
                                                                      ("u", np.float64), ("w", np.float64),
                                                                      ("id", np.uint64))}
        self._keep_pro = A
        return self.lib.orc_set_protons(self.h, A["cell"].size, *[_ptr(A[k]) for k in ("cell", "xi", "u", "w", "id")])

    def set_atmosphere(self, prev_e: int, prev_p: int, count: int) -> None:
        self.lib.orc_set_atmosphere(self.h, int(prev_e), int(prev_p), int(count))

    def photons(self) -> dict:
        n = self.counts()["n_pho"]
        a = dict(cell=np.empty(n, np.int32), xi=np.empty(n), x=np.empty(n), w=np.empty(n),
                 n0=np.empty(n, np.int64), id=np.empty(n, np.uint64))
        self.lib.orc_get_photons(self.h, *[_ptr(a[k]) for k in ("cell", "xi", "x", "w", "n0", "id")])
        return a

    _EV = (("kind", np.int32), ("sub", np.int32), ("step", np.int64), ("id", np.uint64), ("x", np.float64),
           ("cell", np.int32), ("xi", np.float64), ("w", np.float64))

    def events(self) -> dict:
        """Recorded QED events: kind 0 emission (x signed), 1 conversion,
        2 tracked-photon birth (id, cell, xi, signed x, w)."""
        n = self.counts()["n_events"]
        a = {k: np.empty(n, dt) for k, dt in self._EV}
        self.lib.orc_get_events(self.h, *[_ptr(a[k]) for k, _ in self._EV])
        return a

    def set_state(self, lep: dict, pho: dict | None = None, Es: float = 0.0, step: int = 0) -> int:
        def arr(d, k, dt):
            return np.ascontiguousarray(d[k], dtype=dt)
        L = {k: arr(lep, k, dt) for k, dt in (("cell", np.int32), ("xi", np.float64), ("u", np.float64),
                                                ("w", np.float64), ("id", np.uint64))}
        if pho is None:
            pho = dict(cell=[], xi=[], x=[], w=[], n0=[], id=[])
        P = {k: arr(pho, k, dt) for k, dt in (("cell", np.int32), ("xi", np.float64), ("x", np.float64),
                                                ("w", np.float64), ("n0", np.int64), ("id", np.uint64))}
        self._keep = (L, P)
        return self.lib.orc_set_state(self.h, L["cell"].size, *[_ptr(L[k]) for k in ("cell", "xi", "u", "w", "id")],
                                      P["cell"].size, *[_ptr(P[k]) for k in ("cell", "xi", "x", "w", "n0", "id")],
                                      float(Es), int(step))

    def set_field(self, E: np.ndarray, Es: float) -> None:
        E = np.ascontiguousarray(E, dtype=np.float64)
        self.lib.orc_set_field(self.h, _ptr(E), float(Es))

    def set_injection(self, acc: float, count: int) -> None:
        self.lib.orc_set_injection(self.h, float(acc), int(count))

    def merge_now(self) -> None:
        """Run the weight-doubling merge of both species on the current
        state (the first part of a step whose merge check is due)."""
        self.lib.orc_merge_now(self.h)

    def set_replay(self, ev: dict) -> None:
        self._rep = {k: np.ascontiguousarray(ev[k], dtype=dt) for k, dt in self._EV}
        self.lib.orc_set_replay(self.h, self._rep["kind"].size, *[_ptr(self._rep[k]) for k, _ in self._EV])


def binomial_filter(x, passes: int = FILTER_PASSES, periodic: bool = False) -> np.ndarray:
    """The oracle's current filter (Sect. 6.1) applied to a copy of x: each
    pass x_i <- (x_{i-1} + 2 x_i + x_{i+1}) / 4, ends wrapped (periodic) or
    repeating the end value."""
    y = np.ascontiguousarray(x, np.float64).copy()
    _load().orc_filter(y.ctypes.data, y.size, int(passes), int(bool(periodic)))
    return y
