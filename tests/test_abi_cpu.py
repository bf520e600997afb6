"""The C ABI without a GPU: the library loads, exports every declared entry
point, rejects invalid parameters before touching the device, and its host
spectrum sampler agrees with the oracle's inverse CDF."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2608_21920_amd import gap as G

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    if not os.path.exists(G.LIB_PATH):
        pytest.skip("libgap.so not built")
    return G.load_library()


def test_exports_every_declared_symbol():
    lib = _lib()
    hdr = open(os.path.join(ROOT, "include", "gap.h")).read()
    names = set(re.findall(r"^\s*(?:int|void|const char\*)\s+(gap_\w+)\s*\(", hdr, re.M))
    assert {"gap_init", "gap_step", "gap_diag", "gap_free", "gap_strerror"} <= names
    for n in names:
        assert hasattr(lib, n), n


def test_params_struct_matches_header():
    # field order and size of the binding's struct equal the header's
    hdr = open(os.path.join(ROOT, "include", "gap.h")).read()
    body = hdr[hdr.index("typedef struct gap_params"):hdr.index("} gap_params;")]
    fields = re.findall(r"^\s*(?:int32_t|uint32_t|int64_t|uint64_t|double)\s+([\w, ]+);", body, re.M)
    names = [n.strip() for f in fields for n in f.split(",")]
    assert names == [f[0] for f in G.GapParams._fields_]
    assert C.sizeof(G.GapParams) == 8 * 4 // 2 + 8 * 15 + 8 + 16 + 16 + 16


def test_strerror():
    lib = _lib()
    assert lib.gap_strerror(0) == b"ok"
    assert b"invalid" in lib.gap_strerror(-1)


@pytest.mark.parametrize("bad", [dict(n_cells=1), dict(cfl=1.0), dict(cfl=0.0), dict(ppc_ref=0), dict(b=0.0),
                                 dict(nsub_max=0), dict(init_kind=7), dict(inj_weight=0.0), dict(cap_leptons=0),
                                 dict(atm_ppc=-1), dict(atm_ppc=4, atm_temp=0.0), dict(atm_ppc=4, flags=16),
                                 dict(init_kind=4, flags=16)])
def test_invalid_params_rejected_on_host(bad):
    lib = _lib()
    cfg = dict(n_cells=64)
    cfg.update(bad)
    p = G.make_params(cfg)
    h = C.c_void_p()
    assert lib.gap_init(C.byref(p), 1, None, None, C.byref(h)) == -1
    assert not h.value


def test_null_arguments():
    lib = _lib()
    h = C.c_void_p()
    assert lib.gap_init(None, 1, None, None, C.byref(h)) == -1
    p = G.make_params(dict(n_cells=64))
    assert lib.gap_init(C.byref(p), 0, None, None, C.byref(h)) == -1
    assert lib.gap_step(None, 1) == -1
    assert lib.gap_sync(None) == -1
    chi, w, out = np.ones(2), np.zeros(2, np.uint32), np.zeros(2)
    assert lib.gap_qed_sample(None, 0, chi.ctypes.data, w.ctypes.data, 2, out.ctypes.data) == -1


def test_host_sampler_matches_oracle_cdf():
    # the library's table inverse of the photon spectrum vs the oracle's CDF
    from oracle import oracle as O
    _lib()
    r = (np.arange(1, 4000) / 4000.0).astype(np.float32)
    xi = G.sync_inverse_host(r)
    c = np.array([O.sync_cdf(float(x)) for x in xi])
    assert np.max(np.abs(c - r.astype(np.float64))) < 2e-6
    assert np.all(np.diff(xi) >= 0)
    # tails
    r2 = np.array([1e-7, 1e-5, 1 - 1e-6, 1 - 2 ** -24], np.float32)
    xi2 = G.sync_inverse_host(r2)
    c2 = np.array([O.sync_cdf(float(x)) for x in xi2])
    rel = np.abs(c2 - r2.astype(np.float64)) / np.minimum(r2, 1 - r2)
    assert np.all(rel < 2e-3), rel
