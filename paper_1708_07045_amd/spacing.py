"""Accuracy of grid-based interaction energies against direct atom-pair sums
as the grid spacing varies (results section on FFT-based interaction energy
accuracy; the paper compares 0.125, 0.25, 0.5 and 0.8 A and reports the
Pearson correlation and RMS error).  Driver over library calls only.

Poses are drawn by sampling importance resampling from a finished scan
(fftdg_sample_poses), i.e. low-energy clash-free poses like those the BPMF is
made of.  For every spacing the receptor grids of the same box are built on
the GPU (fftdg_grids_build, FP64) and the poses' energies are interpolated
from them (fftdg_grid_energies); the reference is the direct pair sum
(fftdg_pair_energies) with the grids' exclusion rule, so the difference is
the discretisation error alone.
"""
from __future__ import annotations

import numpy as np

from . import _lib as fd


def pose_coordinates(ctx, batch, cfg, t, w) -> np.ndarray:
    """World coordinates [K][n_atoms][3] of poses (configuration, translation)
    from the library's placement (lattice of 2^-16 grid units)."""
    out = []
    origin = np.asarray(w.origin, np.float64)
    for c, tt in zip(cfg, t):
        U, _ = ctx.place(batch, int(c))
        out.append(origin[None, :] + w.h * (U.astype(np.float64) / 65536.0 + np.asarray(tt, np.float64)[None, :]))
    return np.stack(out)


def study(w, ctx, batch, partials, n_poses=200, spacings=(0.125, 0.25, 0.5, 0.8), seed=91, snap=0):
    """Per spacing: Pearson R and RMS error (kcal/mol) of the total
    interaction energy against the direct sum, over n_poses resampled poses
    of ligand 0 (snapshot `snap`)."""
    from workload import synth
    L = w.ligands[0]
    cfg, t, psi = ctx.sample_poses(batch, partials, 0, snap, w.T, synth.uniforms(seed, 2 * n_poses))
    X = pose_coordinates(ctx, batch, cfg, t, w)
    edge = w.n_rec * w.h
    centre = np.asarray(w.origin, np.float64) + 0.5 * (w.n_rec - 1) * w.h
    r = w.receptor
    tools0 = fd.GridTools(2, 1.0, centre)
    direct = tools0.pair_energies(r.xyz[snap], r.q, r.sigma, r.eps, X, L.q, L.sigma, L.eps, exclusion=True)
    dtot = direct.sum(axis=1)
    rows = []
    for h in spacings:
        n = int(round(edge / h))
        tools = fd.GridTools(n, h, centre - 0.5 * (n - 1) * h, "f64", w.clash_mode, w.ljr_cap, w.occ_f)
        grids, _ = tools.build(r.xyz[snap], r.q, r.sigma, r.eps)
        e = tools.grid_energies(grids, X, L.q, L.sigma, L.eps)
        etot = e.sum(axis=1)
        rows.append({"spacing_A": h, "n_rec": n, "pearson_r": float(np.corrcoef(etot, dtot)[0, 1]),
                     "rmse_kcal_mol": float(np.sqrt(np.mean((etot - dtot) ** 2))),
                     "max_abs_err_kcal_mol": float(np.max(np.abs(etot - dtot))),
                     "rmse_by_term_kcal_mol": [float(np.sqrt(np.mean((e[:, k] - direct[:, k]) ** 2))) for k in range(3)]})
        del grids
    return {"poses": int(n_poses), "distinct_configurations": int(len(set(cfg.tolist()))),
            "direct_energy_range_kcal_mol": [float(dtot.min()), float(dtot.max())],
            "by_spacing": rows}
