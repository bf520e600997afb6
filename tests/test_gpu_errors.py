"""Error paths of the C ABI, forced from the host.

A non-finite surface field is a real input: the field update then meets a
non-finite E and the handle reports GAP_ENAN.  The other device conditions
(store overflow, a particle outside its tile window, the field scan's wait
bound) cannot be reached by a valid run of this size without faulting
nothing: they are raised through GAP_STATE_RAISE, which sets the device error
word exactly as the kernels do, so the whole path from the word to the code
returned is exercised.  No kernel is made to fail on purpose."""
import math

import numpy as np
import pytest

from paper_2608_21920_amd import Gap, workloads
from paper_2608_21920_amd import gap as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _small():
    return dict(workloads.TINY, n_cells=256, ppc_init=4)


def test_non_finite_surface_field_reports_enan(torch_gpu):
    print("case: E_s = nan through GAP_STATE_ES_STEP", flush=True)
    g = Gap(_small())
    g.step(3)
    with pytest.raises(G.GapError) as ei:
        g.set_es_step(math.nan, 3)
    assert ei.value.code == -5
    # sticky: reported again, and no further step is enqueued
    assert g.lib.gap_sync(g.h) == -5
    assert g.lib.gap_step(g.h, 5) == -5
    assert g.lib.gap_step_graph(g.h, 5) == -5
    assert g.counts()["step"] == 3
    g.close()


@pytest.mark.parametrize("bits,code", [(1, -3), (2, -4), (4, -5), (8, -6), (2 | 1, -4), (4 | 1, -5)])
def test_device_error_word_maps_to_codes(torch_gpu, bits, code):
    print("case: device error bits %d" % bits, flush=True)
    g = Gap(_small())
    g.step(2)
    g.raise_device_error(bits)
    assert g.lib.gap_sync(g.h) == code
    # reported by every later call that synchronises, and it stops the run
    assert g.lib.gap_step(g.h, 1) == code
    w = np.zeros(4, np.float64)
    assert g.lib.gap_window_forward(g.h, 4, 2, w.ctypes.data) == code
    if code == -6:
        # the scan's wait bound reads as a device error: reads refuse too
        with pytest.raises(G.GapError):
            g.counts()
    else:
        c = g.counts()
        assert c["err"] == code and c["step"] == 2
    g.close()


def test_raise_refuses_unknown_bits(torch_gpu):
    g = Gap(_small())
    with pytest.raises(G.GapError) as ei:
        g.raise_device_error(16)
    assert ei.value.code == -1
    assert g.lib.gap_sync(g.h) == 0
    g.close()


def test_backward_without_window_is_estate(torch_gpu):
    g = Gap(dict(_small(), flags=G.INJ_FIXED))
    da, dn = np.zeros(1), np.zeros(1)
    assert g.lib.gap_window_backward(g.h, da.ctypes.data, dn.ctypes.data) == -7
    g.close()
