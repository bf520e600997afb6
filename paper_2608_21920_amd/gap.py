"""Thin ctypes binding of libgap (argument marshalling only).

Every step of the particle loop runs in the library's HIP kernels; PyTorch
provides device memory (through the allocator callbacks) and the stream.
There is no CPU fallback: constructing a ``Gap`` without the built library
or without a GPU raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgap.so")

QED_OFF, ETA_CO_OFF, FIELD_FROZEN, RECOIL_OFF, PERIODIC, MERGE_ON, TRACK_ALL, ANTI_ALIGNED = \
    1, 2, 4, 8, 16, 32, 64, 128
CONV_OFF, EMIT_OFF, INJ_FIXED, FILTER, QUANTUM = 1024, 2048, 4096, 8192, 16384
FLAGS = dict(QED_OFF=1, ETA_CO_OFF=2, FIELD_FROZEN=4, RECOIL_OFF=8, PERIODIC=16, MERGE_ON=32, TRACK_ALL=64,
             ANTI_ALIGNED=128, CONV_OFF=1024, EMIT_OFF=2048, INJ_FIXED=4096, FILTER=8192, QUANTUM=16384)

ERRORS = {0: "GAP_OK", -1: "GAP_EINVAL", -2: "GAP_ENOMEM", -3: "GAP_ECAP", -4: "GAP_ETILE", -5: "GAP_ENAN",
          -6: "GAP_EDEVICE", -7: "GAP_ESTATE"}

(DIAG_COUNTS, DIAG_FIELD, DIAG_ES, DIAG_RHO, DIAG_LEPTONS, DIAG_PHOTONS, DIAG_NODE_E, DIAG_DERIVED, DIAG_TIMING,
 DIAG_PROFILE, DIAG_PEAK, DIAG_RETURN, DIAG_WATERFALL, DIAG_ESPECTRUM, DIAG_SPECTRA, DIAG_PHASE, DIAG_LAUNCH,
 DIAG_PROTONS) = range(18)
(STATE_PARTICLES, STATE_ES_STEP, STATE_FIELD, STATE_INJECTION, STATE_TIMING, STATE_DRIVE, STATE_LAUNCH,
 STATE_PROFILE_BIN, STATE_WATERFALL, STATE_RAISE, STATE_PROTONS, STATE_ATMOSPHERE) = range(12)
INIT_GAP, INIT_UNIFORM, INIT_EMPTY, INIT_ELECTRON, INIT_ATMOSPHERE = range(5)
# discharge diagnostics: profile groups and the return spectrum's bins
PROFILE_GROUPS = ["e-_up", "e-_down", "e+_up", "e+_down", "x>2_up", "x>2_down"]
RETURN_BINS = 64                      # 1/8 decade of gamma each, gamma in [1, 1e8)
TIMING_KEYS = ["leptons", "photons", "field", "resort", "prologue", "tails", "merge", "conversions"]

COUNT_KEYS = ["n_lep", "n_pho", "step", "n_emit", "n_pho_born", "n_conv", "n_absorbed", "n_outflow",
              "n_pho_exit", "n_dropped", "n_merged", "err", "n_injected", "n_emit_eval", "n_conv_eval",
              "lep_steps", "pho_steps", "rebuckets", "lep_steps_tail", "emit_eval_tail", "pho_steps_tail",
              "conv_eval_tail", "n_pro", "n_pro_absorbed", "n_pro_outflow", "n_atm_e", "n_atm_p"]

from .inputs import LEPTON_DTYPE, PHOTON_DTYPE  # noqa: E402  (record layouts of the C ABI)


class GapError(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        super().__init__("%s%s" % (ERRORS.get(code, str(code)), (": " + what) if what else ""))


class GapParams(C.Structure):
    _fields_ = [
        ("n_cells", C.c_int32), ("init_kind", C.c_int32), ("ppc_init", C.c_int32), ("ppc_ref", C.c_int32),
        ("dx", C.c_double), ("cfl", C.c_double), ("alpha", C.c_double), ("b", C.c_double),
        ("r_curv_cm", C.c_double), ("period_s", C.c_double), ("lambda_c_scale", C.c_double),
        ("r_curv_scale", C.c_double), ("h_gap_frac", C.c_double), ("inj_rate", C.c_double),
        ("inj_weight", C.c_double), ("x_thr", C.c_double), ("xc_floor", C.c_double), ("u_init", C.c_double),
        ("merge_frac", C.c_double), ("seed", C.c_uint64), ("cap_leptons", C.c_int64), ("cap_photons", C.c_int64),
        ("flags", C.c_uint32), ("nsub_max", C.c_int32), ("merge_every", C.c_int32), ("rebucket_every", C.c_int32),
        ("atm_temp", C.c_double), ("atm_ppc", C.c_int32), ("pad_atm", C.c_int32),
    ]


class GapAllocator(C.Structure):
    _fields_ = [("alloc", C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)),
                ("free", C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)),
                ("ctx", C.c_void_p)]


_DEFAULTS = dict(n_cells=1024, init_kind=1, ppc_init=16, ppc_ref=16, dx=0.25, cfl=0.45, alpha=1.5, b=0.1,
                 r_curv_cm=1e7, period_s=1.0, lambda_c_scale=1.0, r_curv_scale=1.0, h_gap_frac=0.8, inj_rate=0.0,
                 inj_weight=1.0, x_thr=2.0, xc_floor=1e-2, u_init=0.0, merge_frac=0.9, seed=0,
                 cap_leptons=1 << 22, cap_photons=1 << 22, flags=0, nsub_max=64, merge_every=64, rebucket_every=0,
                 atm_temp=0.3, atm_ppc=0, pad_atm=0)


def make_params(cfg: dict) -> GapParams:
    p = GapParams()
    for k, v in _DEFAULTS.items():
        setattr(p, k, cfg.get(k, v))
    if cfg.get("merge"):
        p.flags |= MERGE_ON
    return p


_lib = None


def load_library():
    """Load the built library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libgap.so is not built (run __graft_entry__.build())")
    lib = C.CDLL(LIB_PATH)
    P = C.POINTER
    lib.gap_init.restype = C.c_int
    lib.gap_init.argtypes = [P(GapParams), C.c_int32, C.c_void_p, P(GapAllocator), P(C.c_void_p)]
    lib.gap_step.restype = C.c_int
    lib.gap_step.argtypes = [C.c_void_p, C.c_int64]
    lib.gap_step_graph.restype = C.c_int
    lib.gap_step_graph.argtypes = [C.c_void_p, C.c_int64]
    lib.gap_sync.restype = C.c_int
    lib.gap_sync.argtypes = [C.c_void_p]
    lib.gap_diag.restype = C.c_int
    lib.gap_diag.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_size_t, P(C.c_size_t)]
    lib.gap_set_state.restype = C.c_int
    lib.gap_set_state.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_size_t]
    lib.gap_free.restype = None
    lib.gap_free.argtypes = [C.c_void_p]
    lib.gap_strerror.restype = C.c_char_p
    lib.gap_strerror.argtypes = [C.c_int]
    lib.gap_autotune.restype = C.c_int
    lib.gap_autotune.argtypes = [C.c_void_p, C.c_int32, C.c_void_p]
    lib.gap_window_forward.restype = C.c_int
    lib.gap_window_forward.argtypes = [C.c_void_p, C.c_int64, C.c_int32, C.c_void_p]
    lib.gap_window_backward.restype = C.c_int
    lib.gap_window_backward.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    lib.gap_backward.restype = C.c_int
    lib.gap_backward.argtypes = [C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.gap_e_spectrum_noalloc.restype = C.c_int
    lib.gap_e_spectrum_noalloc.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64]
    lib.gap_qed_sample.restype = C.c_int
    lib.gap_qed_sample.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]
    lib.gap_sync_inverse_host.restype = C.c_int
    lib.gap_sync_inverse_host.argtypes = [C.c_void_p, C.c_void_p, C.c_int64]
    _lib = lib
    return lib


def _check(code, what=""):
    if code != 0:
        raise GapError(code, what)


def sync_inverse_host(r) -> np.ndarray:
    """The library's table sampler of the photon spectrum, on the host."""
    lib = load_library()
    r = np.ascontiguousarray(r, dtype=np.float32)
    out = np.empty_like(r)
    _check(lib.gap_sync_inverse_host(r.ctypes.data, out.ctypes.data, r.size), "gap_sync_inverse_host")
    return out


class Gap:
    """A set of flux tubes advanced on the current torch stream of ``device``."""

    def __init__(self, cfgs, device="cuda:0", stream=None, use_torch_alloc=True):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("Gap needs a GPU (no CPU fallback)")
        self.torch = torch
        self.device = torch.device(device)
        lib = load_library()
        self.lib = lib
        if isinstance(cfgs, dict):
            cfgs = [cfgs]
        self.cfgs = [dict(c) for c in cfgs]
        self.n_tubes = len(cfgs)
        arr = (GapParams * self.n_tubes)(*[make_params(c) for c in cfgs])
        self._params = arr
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            self._bufs = {}
            alloc_p = None
            if use_torch_alloc:
                dev = self.device

                def _alloc(nbytes, ctx):
                    t = torch.empty(int(nbytes), dtype=torch.uint8, device=dev)
                    self._bufs[t.data_ptr()] = t
                    return t.data_ptr()

                def _free(ptr, ctx):
                    self._bufs.pop(ptr, None)
                self._cb = GapAllocator(GapAllocator._fields_[0][1](_alloc), GapAllocator._fields_[1][1](_free), None)
                alloc_p = C.byref(self._cb)
            h = C.c_void_p()
            code = lib.gap_init(arr, self.n_tubes, C.c_void_p(self.stream.cuda_stream), alloc_p, C.byref(h))
            _check(code, "gap_init")
            self.h = h

    # -- lifecycle
    def close(self):
        if getattr(self, "h", None):
            self.lib.gap_free(self.h)
            self.h = None
            self._bufs = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- stepping
    def step(self, n=1):
        _check(self.lib.gap_step(self.h, int(n)), "gap_step")

    def step_graph(self, n):
        _check(self.lib.gap_step_graph(self.h, int(n)), "gap_step_graph")

    def sync(self):
        _check(self.lib.gap_sync(self.h), "gap_sync")

    # -- diagnostics
    def _diag(self, kind, tube, nbytes):
        buf = np.empty(max(int(nbytes), 1), np.uint8)
        wr = C.c_size_t(0)
        code = self.lib.gap_diag(self.h, kind, tube, buf.ctypes.data, buf.nbytes, C.byref(wr))
        if code == -1 and wr.value > buf.nbytes:
            buf = np.empty(wr.value, np.uint8)
            code = self.lib.gap_diag(self.h, kind, tube, buf.ctypes.data, buf.nbytes, C.byref(wr))
        _check(code, "gap_diag(%d)" % kind)
        return buf[:wr.value]

    def counts(self, tube=0) -> dict:
        v = self._diag(DIAG_COUNTS, tube, 256).view(np.int64)
        return {k: int(v[i]) for i, k in enumerate(COUNT_KEYS)}

    def n_cells(self, tube=0):
        return int(self.cfgs[tube]["n_cells"])

    def field(self, tube=0) -> np.ndarray:
        return self._diag(DIAG_FIELD, tube, 4 * self.n_cells(tube)).view(np.float32).copy()

    def node_field(self, tube=0) -> np.ndarray:
        return self._diag(DIAG_NODE_E, tube, 4 * (self.n_cells(tube) + 1)).view(np.float32).copy()

    def rho(self, tube=0) -> np.ndarray:
        return self._diag(DIAG_RHO, tube, 8 * (self.n_cells(tube) + 1)).view(np.int64).copy()

    def es(self, tube=0) -> float:
        return float(self._diag(DIAG_ES, tube, 8).view(np.float64)[0])

    def derived(self, tube=0) -> dict:
        v = self._diag(DIAG_DERIVED, tube, 64).view(np.float64)
        return dict(d_cm=v[0], lam=v[1], rc=v[2], dt=v[3], H=v[4], w0=v[5], s_co=v[6], N=int(v[7]))

    def leptons(self, tube=0) -> np.ndarray:
        return self._diag(DIAG_LEPTONS, tube, 0).view(LEPTON_DTYPE).copy()

    def photons(self, tube=0) -> np.ndarray:
        return self._diag(DIAG_PHOTONS, tube, 0).view(PHOTON_DTYPE).copy()

    def protons(self, tube=0) -> np.ndarray:
        """The tube's live protons, records as the leptons' (u = gamma beta)."""
        return self._diag(DIAG_PROTONS, tube, 0).view(LEPTON_DTYPE).copy()

    def set_timing(self, on: bool):
        buf = np.array([1 if on else 0], np.int32)
        _check(self.lib.gap_set_state(self.h, STATE_TIMING, 0, buf.ctypes.data, buf.nbytes), "set_timing")

    def timing(self) -> dict:
        """{kernel group: (launches, total ms)} since timing was enabled or last read."""
        v = self._diag(DIAG_TIMING, 0, 8 * 2 * len(TIMING_KEYS)).view(np.float64)
        return {k: (int(v[2 * i]), float(v[2 * i + 1])) for i, k in enumerate(TIMING_KEYS)}

    # -- state loading (single tube)
    def set_particles(self, lep: np.ndarray, pho: np.ndarray | None = None):
        lep = np.ascontiguousarray(lep, dtype=LEPTON_DTYPE)
        pho = np.zeros(0, PHOTON_DTYPE) if pho is None else np.ascontiguousarray(pho, dtype=PHOTON_DTYPE)
        hdr = np.array([lep.size, pho.size], np.int64)
        buf = np.concatenate([hdr.view(np.uint8), lep.view(np.uint8), pho.view(np.uint8)])
        _check(self.lib.gap_set_state(self.h, STATE_PARTICLES, 0, buf.ctypes.data, buf.nbytes), "set_particles")

    def set_es_step(self, es: float, step: int):
        buf = np.concatenate([np.array([es], np.float64).view(np.uint8), np.array([step], np.int64).view(np.uint8)])
        _check(self.lib.gap_set_state(self.h, STATE_ES_STEP, 0, buf.ctypes.data, buf.nbytes), "set_es_step")

    def set_field(self, E: np.ndarray, es: float):
        buf = np.concatenate([np.ascontiguousarray(E, np.float32).view(np.uint8),
                              np.array([es], np.float64).view(np.uint8)])
        _check(self.lib.gap_set_state(self.h, STATE_FIELD, 0, buf.ctypes.data, buf.nbytes), "set_field")

    def set_protons(self, pro: np.ndarray):
        pro = np.ascontiguousarray(pro, dtype=LEPTON_DTYPE)
        buf = np.concatenate([np.array([pro.size], np.int64).view(np.uint8), pro.view(np.uint8)])
        _check(self.lib.gap_set_state(self.h, STATE_PROTONS, 0, buf.ctypes.data, buf.nbytes), "set_protons")

    def set_atmosphere(self, prev_e: int, prev_p: int, count: int):
        """What the last push left in cell 0, and the atmosphere particles made."""
        buf = np.concatenate([np.array([prev_e, prev_p], np.int32).view(np.uint8),
                              np.array([count], np.uint64).view(np.uint8)])
        _check(self.lib.gap_set_state(self.h, STATE_ATMOSPHERE, 0, buf.ctypes.data, buf.nbytes), "set_atmosphere")

    def set_drive(self, alpha: float, inj_weight: float, tube: int = 0):
        buf = np.array([alpha, inj_weight], np.float64)
        _check(self.lib.gap_set_state(self.h, STATE_DRIVE, int(tube), buf.ctypes.data, buf.nbytes), "set_drive")

    # -- discharge diagnostics
    def set_profile_bin(self, cells: int):
        buf = np.array([cells], np.int32)
        _check(self.lib.gap_set_state(self.h, STATE_PROFILE_BIN, 0, buf.ctypes.data, buf.nbytes), "set_profile_bin")
        self._prof_bin = int(cells)

    def profile(self, tube=0) -> np.ndarray:
        """[nb, 6, 3]: per bin and group (PROFILE_GROUPS) the multiplicity, the
        mean Lorentz factor (photons: mean |x|) and <gamma^-3>."""
        b = getattr(self, "_prof_bin", 64)
        nb = (self.n_cells(tube) + b - 1) // b
        return self._diag(DIAG_PROFILE, tube, 8 * nb * 18).view(np.float64).reshape(nb, 6, 3).copy()

    def peak(self, tube=0) -> dict:
        v = self._diag(DIAG_PEAK, tube, 48).view(np.float64)
        return dict(m_pairs=v[0], h=v[1], g3=v[2], m_photons=v[3], e_min=v[4], e_max=v[5])

    def return_spectrum(self, tube=0) -> np.ndarray:
        """Absorbed weight per 1/8 decade of gamma since the last read, then the
        total weight and the total weight x gamma (reading resets it)."""
        return self._diag(DIAG_RETURN, tube, 8 * (RETURN_BINS + 2)).view(np.float64).copy()

    def set_waterfall(self, every: int, bin_cells: int = 64, capacity: int = 1024):
        """Record the mean of E^2 per bin of `bin_cells` cells after every
        `every`-th step, keeping the last `capacity` records per tube
        (every = 0 stops recording)."""
        buf = np.array([every, bin_cells, capacity], np.int32)
        _check(self.lib.gap_set_state(self.h, STATE_WATERFALL, 0, buf.ctypes.data, buf.nbytes), "set_waterfall")
        self._wf = (int(every), int(bin_cells), int(capacity))

    def waterfall(self, tube=0):
        """(steps [n], E2 [n, nb]) recorded since the last read, oldest first;
        reading empties the record."""
        every, b, cap = getattr(self, "_wf", (0, 64, 1))
        nb = (self.n_cells(tube) + b - 1) // b
        v = self._diag(DIAG_WATERFALL, tube, 16 + 8 * cap * (1 + nb))
        head = v[:16].view(np.int64)
        n, nbr = int(head[0]), int(head[1])
        steps = v[16:16 + 8 * n].view(np.int64).copy()
        e2 = v[16 + 8 * n:16 + 8 * n + 8 * n * nbr].view(np.float64).reshape(n, nbr).copy()
        return steps, e2

    def spectra(self, tube=0) -> np.ndarray:
        """[3, 90]: weight of electrons, positrons (by |u|) and photons (by |x|)
        per 1/8 decade from 1e-2 to 1e9, with underflow and overflow bins."""
        return self._diag(DIAG_SPECTRA, tube, 8 * 3 * 90).view(np.float64).reshape(3, 90).copy()

    def phase_space(self, tube=0) -> np.ndarray:
        """[3, nb, 180]: weight of electrons, positrons (by u) and photons (by x)
        per profile bin and signed momentum column (90 + b for p > 0, 89 - b
        for p <= 0, b the momentum-spectrum bin of |p|)."""
        b = getattr(self, "_prof_bin", 64)
        nb = (self.n_cells(tube) + b - 1) // b
        return self._diag(DIAG_PHASE, tube, 8 * 3 * nb * 180).view(np.float64).reshape(3, nb, 180).copy()

    def e_spectrum(self, tube=0) -> np.ndarray:
        """Power spectrum of E along the gap, zero-padded to M = the next power
        of two >= N: P_k = |X_k|^2 / M for k = 0 .. M/2."""
        M = 1
        while M < self.n_cells(tube):
            M *= 2
        return self._diag(DIAG_ESPECTRUM, tube, 8 * (M // 2 + 1)).view(np.float64).copy()

    def e_spectrum_into(self, power, tube=0):
        """The power spectrum of E into a caller's device tensor (float64,
        at least M/2 + 1 entries), on the handle's stream, allocating
        nothing (gap_e_spectrum_noalloc)."""
        _check(self.lib.gap_e_spectrum_noalloc(self.h, int(tube), C.c_void_p(power.data_ptr()), int(power.numel())),
               "gap_e_spectrum_noalloc")

    def qed_sample(self, kind: int, chi, words) -> np.ndarray:
        """The device's quantum samplers at given points (gap_qed_sample):
        kind 0 the photon energy fraction x/gamma, kind 1 the pair electron's
        energy fraction, at quantum parameter chi for the Philox word."""
        words = np.ascontiguousarray(np.atleast_1d(words), dtype=np.uint32)
        chi = np.ascontiguousarray(np.broadcast_to(np.asarray(chi, np.float64), words.shape))
        out = np.empty(words.shape, np.float64)
        _check(self.lib.gap_qed_sample(self.h, int(kind), chi.ctypes.data, words.ctypes.data, words.size,
                                       out.ctypes.data), "gap_qed_sample")
        return out

    def set_launch(self, grid_leptons: int, grid_photons: int, grid_tails: int, resort_every: int):
        """Launch shapes and re-sort interval (the keys autotune() returns)."""
        buf = np.array([grid_leptons, grid_photons, grid_tails, resort_every], np.int32)
        _check(self.lib.gap_set_state(self.h, STATE_LAUNCH, 0, buf.ctypes.data, buf.nbytes), "set_launch")

    def launch(self) -> dict:
        """The launch shape and re-sort interval in use."""
        v = self._diag(DIAG_LAUNCH, 0, 16).view(np.int32)
        return dict(grid_leptons=int(v[0]), grid_photons=int(v[1]), grid_tails=int(v[2]), resort_every=int(v[3]))

    def autotune(self, trial_steps: int = 32) -> dict:
        """Tune the launch shapes and the re-sort interval on real steps
        (they advance the simulation; results do not depend on the choice)."""
        c = np.zeros(4, np.int32)
        _check(self.lib.gap_autotune(self.h, int(trial_steps), c.ctypes.data), "gap_autotune")
        return dict(grid_leptons=int(c[0]), grid_photons=int(c[1]), grid_tails=int(c[2]), resort_every=int(c[3]))

    # -- differentiable window (frozen QED)
    def window_forward(self, steps: int, ckpt_every: int = 100) -> np.ndarray:
        loss = np.zeros(self.n_tubes, np.float64)
        _check(self.lib.gap_window_forward(self.h, int(steps), int(ckpt_every), loss.ctypes.data),
               "gap_window_forward")
        return loss

    def backward(self):
        da = np.zeros(self.n_tubes, np.float64)
        dn = np.zeros(self.n_tubes, np.float64)
        _check(self.lib.gap_window_backward(self.h, da.ctypes.data, dn.ctypes.data), "gap_window_backward")
        return da, dn

    def window_grad(self, steps: int, ckpt_every: int = 100):
        """Forward and reverse pass in one call: (loss, dL/dalpha, dL/dn_inj)."""
        loss = np.zeros(self.n_tubes, np.float64)
        da = np.zeros(self.n_tubes, np.float64)
        dn = np.zeros(self.n_tubes, np.float64)
        _check(self.lib.gap_backward(self.h, int(steps), int(ckpt_every), loss.ctypes.data, da.ctypes.data,
                                     dn.ctypes.data), "gap_backward")
        return loss, da, dn

    def raise_device_error(self, bits: int):
        """Set device error bits as a kernel would (tests of the error path)."""
        buf = np.array([bits], np.int32)
        _check(self.lib.gap_set_state(self.h, STATE_RAISE, 0, buf.ctypes.data, buf.nbytes), "raise")

    def set_injection(self, acc: float, count: int):
        buf = np.concatenate([np.array([acc], np.float64).view(np.uint8), np.array([count], np.uint64).view(np.uint8)])
        _check(self.lib.gap_set_state(self.h, STATE_INJECTION, 0, buf.ctypes.data, buf.nbytes), "set_injection")


def _window_loss_function():
    import torch

    class GapWindowLoss(torch.autograd.Function):
        """Time-averaged field energy density of a window of steps, as a
        function of the imposed current alpha and the injected charge density
        n_inj (per tube, CPU float64 tensors).  The forward sets the drive of
        every tube (inj_weight = n_inj / inj_rate), runs the window on the GPU
        and returns the per-tube losses; the backward runs the library's
        reverse pass."""

        @staticmethod
        def forward(ctx, alpha, n_inj, gap, steps, ckpt_every):
            a = alpha.detach().cpu().double().numpy().reshape(-1)
            n = n_inj.detach().cpu().double().numpy().reshape(-1)
            for t in range(gap.n_tubes):
                rate = float(gap.cfgs[t].get("inj_rate", 0.0))
                w = n[t] / rate if rate > 0 else float(gap.cfgs[t].get("inj_weight", 1.0))
                gap.set_drive(float(a[t]), w, t)
            loss = gap.window_forward(int(steps), int(ckpt_every))
            ctx.gap = gap
            return torch.as_tensor(loss, dtype=torch.float64)

        @staticmethod
        def backward(ctx, grad):
            da, dn = ctx.gap.backward()
            g = grad.detach().cpu().double()
            return g * torch.as_tensor(da), g * torch.as_tensor(dn), None, None, None

    return GapWindowLoss


def window_loss(alpha, n_inj, gap: Gap, steps: int, ckpt_every: int = 100):
    """Differentiable per-tube window loss (see GapWindowLoss)."""
    return _window_loss_function().apply(alpha, n_inj, gap, steps, ckpt_every)
