"""Seeded synthetic particle states shared by the GPU path and the oracle.

Plain data only: numpy draws in the library's record layout (cell, 24-bit
fraction, momentum or photon energy, weight, id) and the conversion of those
records to the oracle's arrays (fraction / 2^24, float32 -> float64).  Nothing
here computes any step of the method.
"""
from __future__ import annotations

import numpy as np

LEPTON_DTYPE = np.dtype([("cell", "<i4"), ("frac", "<u4"), ("u", "<f4"), ("w", "<f4"), ("id", "<u8")])
PHOTON_DTYPE = np.dtype([("cell", "<i4"), ("frac", "<u4"), ("x", "<f4"), ("w", "<f4"), ("n0", "<i4"),
                         ("pad", "<i4"), ("id", "<u8")])
TWO24 = float(1 << 24)


def random_state(seed: int, n_lep: int, n_pho: int, n_cells: int, u_range=(0.0, 10.0), x_range=(1.0, 8.0),
                 weights=(-1.0, 1.0, 2.0), cell_range=None):
    """Leptons with log-uniform |u| (e^u_range), random sign and weights drawn
    from `weights`; photons with log-uniform |x| (e^x_range), random direction,
    unit weight, birth step 0.  Distinct ids."""
    rng = np.random.default_rng(seed)
    lo, hi = cell_range if cell_range is not None else (0, n_cells)
    L = np.zeros(n_lep, LEPTON_DTYPE)
    L["cell"] = rng.integers(lo, hi, n_lep)
    L["frac"] = rng.integers(0, 1 << 24, n_lep)
    L["u"] = (rng.choice([-1, 1], n_lep) * np.exp(rng.uniform(*u_range, n_lep))).astype(np.float32)
    L["w"] = rng.choice(np.asarray(weights, np.float64), n_lep)
    L["id"] = rng.permutation(n_lep).astype(np.uint64) * np.uint64(2654435761) + np.uint64(7)
    P = np.zeros(n_pho, PHOTON_DTYPE)
    P["cell"] = rng.integers(lo, hi, n_pho)
    P["frac"] = rng.integers(0, 1 << 24, n_pho)
    P["x"] = (rng.choice([-1, 1], n_pho) * np.exp(rng.uniform(*x_range, n_pho))).astype(np.float32)
    P["w"] = 1.0
    P["n0"] = 0
    P["id"] = rng.permutation(n_pho).astype(np.uint64) * np.uint64(40503) + np.uint64(11)
    return L, P


def discharge_sample(seed: int, n_cells: int, h_gap_frac: float, n_lep: int, n_pho: int, step: int):
    """A discharge-like mix for timing: leptons spread over the QED zone with
    Lorentz factors log-uniform in [1, 1e8] (both charges, both directions),
    photons spread over the zone with energies log-uniform in [2, 1e8] and
    birth steps up to 2000 steps back."""
    rng = np.random.default_rng(seed)
    top = max(1, int(h_gap_frac * n_cells))
    L = np.zeros(n_lep, LEPTON_DTYPE)
    L["cell"] = rng.integers(0, top, n_lep)
    L["frac"] = rng.integers(0, 1 << 24, n_lep)
    L["u"] = (rng.choice([-1, 1], n_lep) * np.exp(rng.uniform(0.0, np.log(1e8), n_lep))).astype(np.float32)
    L["w"] = rng.choice([-1.0, 1.0], n_lep)
    L["id"] = rng.permutation(n_lep).astype(np.uint64) * np.uint64(2654435761) + np.uint64(7)
    P = np.zeros(n_pho, PHOTON_DTYPE)
    P["cell"] = rng.integers(0, top, n_pho)
    P["frac"] = rng.integers(0, 1 << 24, n_pho)
    P["x"] = (rng.choice([-1, 1], n_pho) * np.exp(rng.uniform(np.log(2.0), np.log(1e8), n_pho))).astype(np.float32)
    P["w"] = 1.0
    P["n0"] = step - rng.integers(0, 2000, n_pho)
    P["id"] = rng.permutation(n_pho).astype(np.uint64) * np.uint64(40503) + np.uint64(11)
    return L, P


def leptons_as_oracle(rec) -> dict:
    """Record array -> the oracle's lepton arrays (exact conversions)."""
    return dict(cell=rec["cell"].astype(np.int32), xi=rec["frac"].astype(np.float64) / TWO24,
                u=rec["u"].astype(np.float64), w=rec["w"].astype(np.float64), id=rec["id"].astype(np.uint64))


def photons_as_oracle(rec) -> dict:
    return dict(cell=rec["cell"].astype(np.int32), xi=rec["frac"].astype(np.float64) / TWO24,
                x=rec["x"].astype(np.float64), w=rec["w"].astype(np.float64), n0=rec["n0"].astype(np.int64),
                id=rec["id"].astype(np.uint64))
