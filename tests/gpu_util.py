"""Helpers shared by the GPU tests (conversions between the two state layouts)."""
import numpy as np

TWO24 = float(1 << 24)


def gpu_leptons_as_oracle(rec):
    """GPU lepton records -> oracle state arrays (exact: frac/2^24 and f32 -> f64)."""
    return dict(cell=rec["cell"].astype(np.int32), xi=rec["frac"].astype(np.float64) / TWO24,
                u=rec["u"].astype(np.float64), w=rec["w"].astype(np.float64), id=rec["id"].astype(np.uint64))


def gpu_photons_as_oracle(rec):
    return dict(cell=rec["cell"].astype(np.int32), xi=rec["frac"].astype(np.float64) / TWO24,
                x=rec["x"].astype(np.float64), w=rec["w"].astype(np.float64), n0=rec["n0"].astype(np.int64),
                id=rec["id"].astype(np.uint64))


def by_id(d):
    o = np.argsort(d["id"], kind="stable")
    return {k: np.asarray(v)[o] for k, v in d.items()}


def rel_field_err(Eg, Eo):
    Eo = np.asarray(Eo, np.float64)
    return float(np.max(np.abs(np.asarray(Eg, np.float64) - Eo)) / max(np.max(np.abs(Eo)), 1e-300))
