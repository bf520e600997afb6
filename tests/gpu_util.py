"""Helpers shared by the GPU tests (conversions between the two state layouts)."""
import numpy as np

TWO24 = float(1 << 24)


from paper_2608_21920_amd.inputs import leptons_as_oracle as gpu_leptons_as_oracle  # noqa: E402,F401
from paper_2608_21920_amd.inputs import photons_as_oracle as gpu_photons_as_oracle  # noqa: E402,F401


def by_id(d):
    o = np.argsort(d["id"], kind="stable")
    return {k: np.asarray(v)[o] for k, v in d.items()}


def rel_field_err(Eg, Eo):
    Eo = np.asarray(Eo, np.float64)
    return float(np.max(np.abs(np.asarray(Eg, np.float64) - Eo)) / max(np.max(np.abs(Eo)), 1e-300))
