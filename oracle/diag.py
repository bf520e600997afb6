"""Discharge diagnostics of a particle state, written out as plain
definitions in FP64 (test infrastructure only; parity unpinned beyond the
checks in tests/test_oracle_diag.py).

These are the quantities the paper reads off its kinetic simulations
(Sect. 5):
 * multiplicity m = n / n_co (its definition with the screening time,
   Sect. 3).  A macro-particle of weight w stands for w dx / ppc_ref
   particles per unit area (the plasma at n_co has ppc_ref particles of unit
   weight per cell), so a bin of B cells has m = sum |w| / (B ppc_ref);
 * the mean Lorentz factor per species and direction (Fig. 3, row 6);
 * the plasma-inertia measure <gamma^-3> = n^-1 sum gamma^-3 over the pairs
   (its definition with eq. omega_osc, Sect. 3; Fig. 3, row 7);
 * the multiplicity of electrons, positrons and photons with x > 2, split
   by direction (Fig. 3, row 5);
 * the peak pair multiplicity in the gap zone and <gamma^-3> at its
   location, and the extremes of E (Fig. 5);
 * one row of the space-time diagram of E^2 (Fig. 4): the mean of E^2 over
   each bin of cells, the last bin ragged;
 * momentum spectra (Fig. 3, row 1): the weight of electrons and positrons
   per 1/8 decade of |u| = gamma beta and of photons per 1/8 decade of |x|,
   from 1e-2 to 1e9, with an underflow and an overflow bin; a value goes to
   the last edge 10^(-2 + b/8) its square reaches (compared in FP64 against
   10^(2 (-2 + b/8)));
 * phase space (Fig. 3, rows 1-4): the same weights per bin of B cells and
   per signed momentum bin, 180 columns running from large negative to large
   positive p (u or x): column 90 + b for p > 0, 89 - b for p <= 0, b the
   momentum-spectrum bin of |p|;
 * the power spectrum of E along the gap (the full-scale configuration's
   field diagnostic): the field zero-padded to M = the next power of two
   >= N cells, P_k = |sum_j E_j exp(-2 pi i j k / M)|^2 / M for
   k = 0 .. M/2 (Parseval: sum over all M of P_k = sum_j E_j^2).

Groups, in order: electrons moving up (u > 0), down; positrons up, down;
photons with |x| > 2 moving up (x > 0), down.  A lepton's species is the
sign of its weight (electrons carry w < 0).
"""
from __future__ import annotations

import numpy as np

GROUPS = ("e-_up", "e-_down", "e+_up", "e+_down", "x>2_up", "x>2_down")


def profile_sums(lep: dict, pho: dict, n_cells: int, bin_cells: int) -> np.ndarray:
    """[nb, 6, 3]: per bin and group, sum |w|, sum |w| gamma (photons: sum
    w |x|) and sum |w| gamma^-3 (photons: 0)."""
    nb = (n_cells + bin_cells - 1) // bin_cells
    acc = np.zeros((nb, 6, 3))
    cell = np.clip(np.asarray(lep["cell"], np.int64), 0, n_cells - 1)
    w = np.asarray(lep["w"], np.float64)
    u = np.asarray(lep["u"], np.float64)
    live = w != 0.0
    b = cell[live] // bin_cells
    grp = np.where(w[live] < 0.0, 0, 2) + np.where(u[live] > 0.0, 0, 1)
    aw = np.abs(w[live])
    g = np.sqrt(1.0 + u[live] * u[live])
    np.add.at(acc, (b, grp, 0), aw)
    np.add.at(acc, (b, grp, 1), aw * g)
    np.add.at(acc, (b, grp, 2), aw / (g * g * g))
    if pho is not None and len(pho["x"]):
        x = np.asarray(pho["x"], np.float64)
        pw = np.asarray(pho["w"], np.float64)
        sel = (x != 0.0) & (np.abs(x) > 2.0)
        pc = np.clip(np.asarray(pho["cell"], np.int64), 0, n_cells - 1)[sel] // bin_cells
        pg = 4 + np.where(x[sel] > 0.0, 0, 1)
        np.add.at(acc, (pc, pg, 0), pw[sel])
        np.add.at(acc, (pc, pg, 1), pw[sel] * np.abs(x[sel]))
    return acc


def profile(sums: np.ndarray, bin_cells: int, ppc_ref: int) -> np.ndarray:
    """[nb, 6, 3]: multiplicity, mean Lorentz factor (photons: mean |x|) and
    <gamma^-3> (0 for photons and for empty groups)."""
    out = np.zeros_like(sums)
    w = sums[:, :, 0]
    out[:, :, 0] = w / (bin_cells * ppc_ref)
    nz = w > 0.0
    out[:, :, 1][nz] = sums[:, :, 1][nz] / w[nz]
    out[:, :, 2][nz] = sums[:, :, 2][nz] / w[nz]
    return out


def peak(sums: np.ndarray, E: np.ndarray, bin_cells: int, dx: float, H: float, ppc_ref: int) -> dict:
    """The largest pair multiplicity over the bins whose centre lies below H
    (the first of equal values), the height of that bin's centre, <gamma^-3>
    of the pairs there, the photon multiplicity there, and min/max of E."""
    nb = sums.shape[0]
    centre = (np.arange(nb) + 0.5) * bin_cells * dx
    pair_w = sums[:, :4, 0].sum(axis=1)
    zone = np.nonzero(centre < H)[0]
    if zone.size == 0:
        return dict(m_pairs=0.0, h=-1.0, g3=0.0, m_photons=0.0,
                    e_min=float(np.min(E)) if len(E) else 0.0, e_max=float(np.max(E)) if len(E) else 0.0)
    b = int(zone[np.argmax(pair_w[zone])])
    w = pair_w[b]
    g3 = sums[b, :4, 2].sum() / w if w > 0.0 else 0.0
    return dict(m_pairs=w / (bin_cells * ppc_ref), h=float(centre[b]), g3=float(g3),
                m_photons=float((sums[b, 4, 0] + sums[b, 5, 0]) / (bin_cells * ppc_ref)),
                e_min=float(np.min(E)), e_max=float(np.max(E)))


def waterfall_row(E: np.ndarray, bin_cells: int) -> np.ndarray:
    """[nb]: the mean of E^2 over each bin of `bin_cells` cells of the field at
    cell centres (the last bin holds the remaining cells)."""
    E = np.asarray(E, np.float64)
    nb = (E.size + bin_cells - 1) // bin_cells
    out = np.zeros(nb)
    for b in range(nb):
        seg = E[b * bin_cells:(b + 1) * bin_cells]
        out[b] = np.sum(seg * seg) / seg.size
    return out


def e_power_spectrum(E: np.ndarray) -> np.ndarray:
    """[M/2 + 1]: P_k = |X_k|^2 / M of the field zero-padded to M = 2^ceil(log2 N)
    (numpy's FFT in FP64 as the transform)."""
    E = np.asarray(E, np.float64)
    M = 1
    while M < E.size:
        M *= 2
    x = np.zeros(M)
    x[:E.size] = E
    X = np.fft.fft(x)
    return (X.real ** 2 + X.imag ** 2)[:M // 2 + 1] / M


SPEC_EDGES = 89                          # edges 10^(-2 + b/8), b = 0 .. 88
SPEC_NB = SPEC_EDGES + 1                 # underflow, 88 bins, overflow


def spectrum_edges_sq() -> np.ndarray:
    """Squares of the spectrum's bin edges, 10^(2 (-2 + b/8))."""
    return np.array([10.0 ** (2.0 * (-2.0 + b / 8.0)) for b in range(SPEC_EDGES)])


def spectra(lep: dict, pho: dict) -> np.ndarray:
    """[3, SPEC_NB]: weight of electrons (by |u|), positrons (by |u|) and
    photons (by |x|) per bin; bin = number of edges whose square is <= the
    value's square (0: below 1e-2, SPEC_NB - 1: at or above 1e9)."""
    thr = spectrum_edges_sq()
    out = np.zeros((3, SPEC_NB))
    w = np.asarray(lep["w"], np.float64)
    u = np.asarray(lep["u"], np.float64)
    live = w != 0.0
    b = np.searchsorted(thr, u[live] * u[live], side="right")
    sp = np.where(w[live] < 0.0, 0, 1)
    np.add.at(out, (sp, b), np.abs(w[live]))
    if pho is not None and len(pho["x"]):
        x = np.asarray(pho["x"], np.float64)
        pw = np.asarray(pho["w"], np.float64)
        a = x != 0.0
        np.add.at(out, (2, np.searchsorted(thr, x[a] * x[a], side="right")), pw[a])
    return out


PHASE_NP = 2 * SPEC_NB                   # signed momentum columns


def phase_space(lep: dict, pho: dict, n_cells: int, bin_cells: int) -> np.ndarray:
    """[3, nb, 180]: weight of electrons, positrons (by u) and photons (by x)
    per bin of `bin_cells` cells and signed momentum column."""
    thr = spectrum_edges_sq()
    nb = (n_cells + bin_cells - 1) // bin_cells
    out = np.zeros((3, nb, PHASE_NP))

    def col(p):
        b = np.searchsorted(thr, p * p, side="right")
        return np.where(p > 0.0, SPEC_NB + b, SPEC_NB - 1 - b)

    w = np.asarray(lep["w"], np.float64)
    u = np.asarray(lep["u"], np.float64)
    live = w != 0.0
    cell = np.clip(np.asarray(lep["cell"], np.int64), 0, n_cells - 1)[live]
    np.add.at(out, (np.where(w[live] < 0.0, 0, 1), cell // bin_cells, col(u[live])), np.abs(w[live]))
    if pho is not None and len(pho["x"]):
        x = np.asarray(pho["x"], np.float64)
        a = x != 0.0
        pc = np.clip(np.asarray(pho["cell"], np.int64), 0, n_cells - 1)[a]
        np.add.at(out, (2, pc // bin_cells, col(x[a])), np.asarray(pho["w"], np.float64)[a])
    return out
