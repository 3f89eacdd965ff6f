"""FP64 references for the grid-spacing accuracy study (test
infrastructure only; independent of the GPU kernels).

  - pair_energies: the direct atom-pair interaction energies of Eqs. 4-6
    (ELE 332.05 q_i q_j / r, LJr sqrt(eps_i eps_j)(sigma_i sigma_j)^6 / r^12,
    LJa -2 sqrt(eps_i eps_j)(sigma_i sigma_j)^3 / r^6), optionally dropping
    every pair closer than 2^(-1/6) sigma_j of the receptor atom (the
    exclusion of the receptor grids, Eq. 7, in occupancy mode);
  - grid_energies: the same interaction from receptor grids by trilinear
    interpolation at each ligand atom (Eqs. 3 and 8 at one position), grid
    corners outside the grid taken as zero.
"""
from __future__ import annotations

import numpy as np

ELE = 332.05


def pair_energies(rxyz, rq, rs, re, poses, q, s, e, exclusion=True) -> np.ndarray:
    """poses [P][n][3] -> [P][3] (ELE, LJr, LJa), kcal/mol."""
    rxyz = np.asarray(rxyz, np.float64)
    rq, rs, re = (np.asarray(a, np.float64) for a in (rq, rs, re))
    q, s, e = (np.asarray(a, np.float64) for a in (q, s, e))
    poses = np.asarray(poses, np.float64)
    out = np.zeros((poses.shape[0], 3))
    rex = 2.0 ** (-1.0 / 6.0) * rs
    for p in range(poses.shape[0]):
        d = np.linalg.norm(poses[p][:, None, :] - rxyz[None, :, :], axis=-1)   # [n][Nr]
        keep = d >= rex[None, :] if exclusion else np.ones_like(d, bool)
        dk = np.where(keep, d, 1.0)
        out[p, 0] = np.sum(np.where(keep, ELE * q[:, None] * rq[None, :] / dk, 0.0))
        eij = np.sqrt(e[:, None] * re[None, :])
        sij = s[:, None] * rs[None, :]
        out[p, 1] = np.sum(np.where(keep, eij * sij ** 6 / dk ** 12, 0.0))
        out[p, 2] = np.sum(np.where(keep, -2.0 * eij * sij ** 3 / dk ** 6, 0.0))
    return out


def grid_energies(grids, h, origin, poses, q, s, e) -> np.ndarray:
    """grids [3][n][n][n] ([z][y][x]); poses [P][n_atoms][3] -> [P][3]."""
    g = np.asarray(grids, np.float64)
    n = g.shape[1]
    q, s, e = (np.asarray(a, np.float64) for a in (q, s, e))
    gam = np.stack([q, np.sqrt(e) * s ** 6, -2.0 * np.sqrt(e) * s ** 3], axis=1)   # [n_atoms][3]
    poses = np.asarray(poses, np.float64)
    out = np.zeros((poses.shape[0], 3))
    for p in range(poses.shape[0]):
        u = (poses[p] - np.asarray(origin, np.float64)[None, :]) / h          # (x, y, z) grid units
        i0 = np.floor(u).astype(np.int64)
        f = u - i0
        v = np.zeros((u.shape[0], 3))
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    c = i0 + np.array([dx, dy, dz])
                    w = ((f[:, 0] if dx else 1 - f[:, 0]) * (f[:, 1] if dy else 1 - f[:, 1])
                         * (f[:, 2] if dz else 1 - f[:, 2]))
                    ok = np.all((c >= 0) & (c < n), axis=1)
                    cc = np.where(ok[:, None], c, 0)
                    for ch in range(3):
                        val = g[ch][cc[:, 2], cc[:, 1], cc[:, 0]]
                        v[:, ch] += np.where(ok, w * val, 0.0)
        out[p] = np.sum(gam * v, axis=0)
    return out


def grid_values(rxyz, rq, rs, re, points, chunk: int = 4096) -> np.ndarray:
    """Receptor grid values of Eq. 7 in occupancy mode (every term zero within
    2^(-1/6) sigma_j) at arbitrary points [K][3]: [K][3] (ELE, LJr, LJa) with
    ELE = 332.05 sum q_j / r, LJr = sum sqrt(eps_j) sigma_j^6 / r^12,
    LJa = sum sqrt(eps_j) sigma_j^3 / r^6."""
    rxyz = np.asarray(rxyz, np.float64)
    rq, rs, re = (np.asarray(a, np.float64) for a in (rq, rs, re))
    pts = np.asarray(points, np.float64)
    rex = 2.0 ** (-1.0 / 6.0) * rs
    se = np.sqrt(re)
    out = np.zeros((pts.shape[0], 3))
    for a in range(0, pts.shape[0], chunk):
        d = np.linalg.norm(pts[a:a + chunk, None, :] - rxyz[None, :, :], axis=-1)
        keep = d >= rex[None, :]
        dk = np.where(keep, d, 1.0)
        out[a:a + chunk, 0] = np.sum(np.where(keep, ELE * rq[None, :] / dk, 0.0), axis=1)
        out[a:a + chunk, 1] = np.sum(np.where(keep, se * rs ** 6 / dk ** 12, 0.0), axis=1)
        out[a:a + chunk, 2] = np.sum(np.where(keep, se * rs ** 3 / dk ** 6, 0.0), axis=1)
    return out


def occupancy_values(rxyz, rs, occ_f: float, points, chunk: int = 4096) -> np.ndarray:
    """Eq. 10 receptor occupancy at arbitrary points: 1 where some receptor atom
    lies closer than occ_f 2^(-1/6) sigma_j."""
    rxyz = np.asarray(rxyz, np.float64)
    rad = occ_f * 2.0 ** (-1.0 / 6.0) * np.asarray(rs, np.float64)
    pts = np.asarray(points, np.float64)
    out = np.zeros(pts.shape[0], np.uint8)
    for a in range(0, pts.shape[0], chunk):
        d = np.linalg.norm(pts[a:a + chunk, None, :] - rxyz[None, :, :], axis=-1)
        out[a:a + chunk] = np.any(d < rad[None, :], axis=1)
    return out


def occupancy_grid(rxyz, rs, occ_f: float, n_rec: int, h: float, origin) -> np.ndarray:
    """Eq. 10 receptor occupancy on the whole grid [z][y][x] by rasterising
    each atom's ball (nodes closer than occ_f 2^(-1/6) sigma_j)."""
    rxyz = np.asarray(rxyz, np.float64)
    rad = occ_f * 2.0 ** (-1.0 / 6.0) * np.asarray(rs, np.float64)
    org = np.asarray(origin, np.float64)
    occ = np.zeros((n_rec, n_rec, n_rec), np.uint8)
    for j in range(rxyz.shape[0]):
        lo = np.maximum(np.floor((rxyz[j] - rad[j] - org) / h).astype(int), 0)
        hi = np.minimum(np.ceil((rxyz[j] + rad[j] - org) / h).astype(int), n_rec - 1)
        if np.any(hi < lo):
            continue
        xs, ys, zs = (np.arange(lo[d], hi[d] + 1) for d in range(3))
        X, Y, Z = np.meshgrid(xs, ys, zs, indexing="ij")
        p = org[None, :] + h * np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
        inside = np.linalg.norm(p - rxyz[j], axis=1) < rad[j]
        occ[Z.ravel()[inside], Y.ravel()[inside], X.ravel()[inside]] = 1
    return occ
