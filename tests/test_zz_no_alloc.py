"""The allocation-free entry point (gap_e_spectrum_noalloc) against the
allocating one (GAP_DIAG_ESPECTRUM): the same transform, its ping-pong
buffers in the library's static workspace instead of handle memory.  Two
calls in a row, the second on a smaller tube, each equal to gap_diag's
spectrum of the same field bit for bit (same kernels, same order); then the
refusals (a tube beyond the workspace, a short output buffer)."""
import numpy as np
import pytest

from paper_2608_21920_amd import Gap, workloads
from paper_2608_21920_amd import gap as G

pytestmark = pytest.mark.gpu


def test_noalloc_spectrum_equals_diag_spectrum():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("case: no-alloc spectrum, tubes of 70000 and 1000 cells", flush=True)
    cfgs = [dict(workloads.TINY, n_cells=70000, ppc_init=2, seed=3), dict(workloads.TINY, n_cells=1000, seed=4)]
    g = Gap(cfgs)
    g.step(30)
    g.sync()
    out = torch.full((70000,), -1.0, dtype=torch.float64, device="cuda")
    for t, M in ((0, 131072), (1, 1024)):
        g.e_spectrum_into(out, tube=t)
        g.sync()
        got = out[:M // 2 + 1].cpu().numpy()
        want = g.e_spectrum(t)
        assert want.shape == got.shape
        assert np.array_equal(got, want), t
        assert np.all(np.isfinite(got)) and got.max() > 0
        # Parseval over the padded transform: sum over all M modes = sum E^2
        E = g.field(t).astype(np.float64)
        full = got[0] + got[-1] + 2.0 * got[1:-1].sum()
        assert abs(full - float((E * E).sum())) <= 1e-9 * float((E * E).sum())
    # refusals: a buffer one short, a null buffer
    with pytest.raises(G.GapError):
        g.e_spectrum_into(out[:512], tube=1)
    assert g.lib.gap_e_spectrum_noalloc(g.h, 1, None, 600) == -1
    g.close()


def test_noalloc_spectrum_refuses_tubes_beyond_the_workspace():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("case: no-alloc spectrum refusal, 300000 cells", flush=True)
    g = Gap(dict(workloads.BASE, n_cells=300000, init_kind=2, b=0.1, r_curv_cm=1e7, alpha=0.0,
                 cap_leptons=1 << 16, cap_photons=1 << 16))
    out = torch.zeros(1 << 19, dtype=torch.float64, device="cuda")
    with pytest.raises(G.GapError) as ei:
        g.e_spectrum_into(out, tube=0)
    assert ei.value.code == -1
    g.close()
