"""The plain FFT method on the CPU, FP64: a second host baseline.

TEST INFRASTRUCTURE ONLY, like the rest of `oracle/`: the benchmark times it
beside the direct oracle, and a test pins it to the direct oracle.  It is
the correlation theorem of Eq. 9 applied as the paper applies it on CPUs:
the receptor grids zero-padded to the FFT edge and transformed once, each
configuration's ligand channels spread densely (Eq. 8's ligand grids, the
oracle's trilinear spreading), transformed with real-to-complex 3D FFTs
(`scipy.fft`, pocketfft, all host threads), multiplied by the receptor
spectra as R * conj(L), summed over ELE / LJr / LJa and inverse-transformed
into the interaction energy at every translation.  In occupancy mode the
Eq. 10 overlap is the same correlation of the two occupancy grids, and a
translation clashes when it reaches one half (the overlap is an integer
count).  The valid translations of the ligand box are then reduced to the
per-configuration partials of Eq. 2 by the oracle's own reducer.
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft as sfft

from . import kT, ligand_weights, occ_dense, occ_thresholds, partial, place_cfg, spread_dense, valid_shape


def _workers() -> int:
    return int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or len(os.sched_getaffinity(0))


def receptor_spectra(w, grids, occ):
    """rfftn of the three energy grids (and the occupancy grid), each
    zero-padded from n_rec^3 to n_fft^3; arrays are [z][y][x]."""
    n, N = w.n_rec, w.n_fft
    pad = np.zeros((N, N, N))
    out = []
    for ch in range(3):
        pad[:n, :n, :n] = grids[ch]
        out.append(sfft.rfftn(pad, workers=_workers()))
    if occ is not None:
        pad[:] = 0.0
        pad[:n, :n, :n] = occ
        out.append(sfft.rfftn(pad, workers=_workers()))
    return out


def config_partial(w, spectra, lig_idx: int, cfg: int, return_fields: bool = False):
    """Partials (m, s, n_valid, n_finite, psi_min, argmin) of one
    configuration by the FFT correlation; optionally the raw energies and
    clash mask on the valid translations."""
    L = w.ligands[lig_idx]
    N = w.n_fft
    u, box = place_cfg(w, lig_idx, cfg)
    gam = ligand_weights(L)
    Vz, Vy, Vx = valid_shape(w, box)
    acc = None
    for ch in range(3):
        lf = sfft.rfftn(spread_dense(N, u, gam[:, ch]), workers=_workers())
        term = spectra[ch] * np.conj(lf)
        acc = term if acc is None else acc + term
    psi = sfft.irfftn(acc, s=(N, N, N), workers=_workers())[:Vz, :Vy, :Vx]
    clash = None
    if w.clash_mode == "occ":
        ol = sfft.rfftn(occ_dense(N, u, occ_thresholds(L, w.occ_f, w.h)).astype(np.float64), workers=_workers())
        ov = sfft.irfftn(spectra[3] * np.conj(ol), s=(N, N, N), workers=_workers())[:Vz, :Vy, :Vx]
        clash = (ov >= 0.5).astype(np.uint8)
    p = partial(psi, clash, 1.0 / kT(w.T))
    if return_fields:
        return p, psi, clash
    return p


def scan(w, spectra, lig_idx: int = 0, cfgs=None) -> np.ndarray:
    """Per-configuration partials [n][6] for one ligand and one snapshot."""
    L = w.ligands[lig_idx]
    sel = np.arange(L.n_cfg) if cfgs is None else np.asarray(cfgs)
    return np.stack([config_partial(w, spectra, lig_idx, int(c)) for c in sel]) if len(sel) else np.zeros((0, 6))
