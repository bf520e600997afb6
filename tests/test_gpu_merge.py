"""Weight-doubling merge on the GPU vs the oracle on an identical state.

The merge is not part of the paper (it keeps the stores under their cap);
its result on a given state is deterministic, so the comparison is exact:
same surviving ids, same weights, same positions and momenta."""
import numpy as np
import pytest

from paper_2608_21920_amd import Gap, workloads
from paper_2608_21920_amd import gap as G
from paper_2608_21920_amd.inputs import random_state
from oracle.oracle import Oracle

from gpu_util import by_id, gpu_leptons_as_oracle, gpu_photons_as_oracle

pytestmark = pytest.mark.gpu


def _state(seed, n, N):
    return random_state(seed, n, n // 2, N)


@pytest.mark.parametrize("n,N", [(20000, 64), (3000, 700)])
def test_merge_matches_oracle_on_identical_state(n, N):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("case: merge n=%d N=%d" % (n, N), flush=True)
    cfg = dict(workloads.BASE, n_cells=N, init_kind=2, b=0.1, r_curv_cm=1e7, alpha=0.0,
               flags=G.QED_OFF | G.FIELD_FROZEN | G.PERIODIC | G.MERGE_ON, cap_leptons=int(1.2 * n),
               cap_photons=int(0.6 * n), merge_frac=0.5, merge_every=1, seed=13)
    L, P = _state(1, n, N)
    g = Gap(cfg)
    g.set_particles(L, P)
    g.set_field(np.zeros(N, np.float32), 0.0)
    o = Oracle(cfg)
    o.set_state(gpu_leptons_as_oracle(L), gpu_photons_as_oracle(P))
    o.set_field(np.zeros(N), 0.0)
    g.step(1)
    o.step(1)
    cg, co = g.counts(), o.counts()
    assert cg["err"] == 0
    assert cg["n_merged"] == co["n_merged"] > 0
    A, B = by_id(gpu_leptons_as_oracle(g.leptons())), by_id(o.leptons())
    assert np.array_equal(A["id"], B["id"])
    assert np.array_equal(A["w"], B["w"])
    assert np.array_equal(A["cell"], B["cell"])
    assert np.allclose(A["xi"], B["xi"], atol=1e-6)
    C, D = by_id(gpu_photons_as_oracle(g.photons())), by_id(o.photons())
    assert np.array_equal(C["id"], D["id"])
    assert np.array_equal(C["w"], D["w"])
    g.close()


def test_merge_at_scale_matches_oracle():
    """The merge at the production grid's size: 2.4e6 leptons and 1.2e6
    photons on 65536 cells (hundreds of radix-sort blocks per pass, every
    kind of group from empty to crowded), exact against the oracle."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    N, nl, npho = 65536, 2_400_000, 1_200_000
    print("case: merge at scale nl=%d np=%d N=%d" % (nl, npho, N), flush=True)
    cfg = dict(workloads.BASE, n_cells=N, init_kind=2, b=0.1, r_curv_cm=1e7, alpha=0.0,
               flags=G.QED_OFF | G.FIELD_FROZEN | G.PERIODIC | G.MERGE_ON, cap_leptons=3_000_000,
               cap_photons=1_500_000, merge_frac=0.5, merge_every=1, seed=29)
    L, P = random_state(4, nl, npho, N, u_range=(-4.0, 12.0), x_range=(0.7, 14.0), weights=(-1.0, 1.0, 2.0, -0.5))
    g = Gap(cfg)
    g.set_particles(L, P)
    g.set_field(np.zeros(N, np.float32), 0.0)
    o = Oracle(cfg)
    o.set_state(gpu_leptons_as_oracle(L), gpu_photons_as_oracle(P))
    o.set_field(np.zeros(N), 0.0)
    g.step(1)
    o.step(1)
    cg, co = g.counts(), o.counts()
    assert cg["err"] == 0
    assert cg["n_merged"] == co["n_merged"] > 0.2 * (nl + npho)
    A, B = by_id(gpu_leptons_as_oracle(g.leptons())), by_id(o.leptons())
    assert np.array_equal(A["id"], B["id"])
    assert np.array_equal(A["w"], B["w"])
    assert np.array_equal(A["u"], B["u"])
    # positions after the step's drift: cells exact except at a wrap near-tie
    assert np.mean(A["cell"] != B["cell"]) < 1e-5
    C, D = by_id(gpu_photons_as_oracle(g.photons())), by_id(o.photons())
    assert np.array_equal(C["id"], D["id"])
    assert np.array_equal(C["w"], D["w"])
    assert np.array_equal(C["x"], D["x"])
    g.close()
