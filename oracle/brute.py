"""Pure-Python second witness for the oracle on tiny inputs (test only).

Restates the method from the paper in a different form than `oracle.c`:
  - rotation by the quaternion sandwich product q (0, v) q* instead of a
    rotation matrix ("Ligand Sampling": random rotation about the centroid);
  - the ligand grid G_L is built explicitly by trilinear spreading into a
    dictionary and the energy is the correlation sum of Eq. 8,
    Psi(t) = sum_n G_R(n + t) G_L(n), instead of interpolating G_R at atoms;
  - the clash test counts the overlap of the two occupancy grids of Eq. 10,
    sum_n O_R(n + t) O_L(n), instead of stopping at the first hit;
  - Eq. 7 grids are summed atom by atom with Python floats.
Only for grids of edge <= ~10 (cost grows as the sixth power of the edge).
"""
from __future__ import annotations

import math


def quat_rotate(q, v):
    w, x, y, z = q
    n = math.sqrt(w * w + x * x + y * y + z * z)
    w, x, y, z = w / n, x / n, y / n, z / n

    def mul(a, b):
        a0, a1, a2, a3 = a
        b0, b1, b2, b3 = b
        return (a0 * b0 - a1 * b1 - a2 * b2 - a3 * b3,
                a0 * b1 + a1 * b0 + a2 * b3 - a3 * b2,
                a0 * b2 - a1 * b3 + a2 * b0 + a3 * b1,
                a0 * b3 + a1 * b2 - a2 * b1 + a3 * b0)

    r = mul(mul((w, x, y, z), (0.0, v[0], v[1], v[2])), (w, -x, -y, -z))
    return [r[1], r[2], r[3]]


def place(conf, quat, h):
    n = len(conf)
    c = [sum(p[d] for p in conf) / n for d in range(3)]
    rot = [quat_rotate(quat, [p[d] - c[d] for d in range(3)]) for p in conf]
    mn = [min(p[d] for p in rot) for d in range(3)]
    u = [[round(((p[d] - mn[d]) / h + 2.0) * 65536.0) / 65536.0 for d in range(3)] for p in rot]
    box = [math.ceil(max(p[d] for p in u)) + 2 for d in range(3)]
    return u, box


def receptor_grids(xyz, q, sigma, eps, n_rec, h, origin, mode, cap, occ_f):
    """Eq. 7 (ELE, LJr, LJa) and Eq. 10 as nested lists [ch][z][y][x]."""
    k = 2.0 ** (-1.0 / 6.0)
    G = [[[[0.0] * n_rec for _ in range(n_rec)] for _ in range(n_rec)] for _ in range(3)]
    O = [[[0] * n_rec for _ in range(n_rec)] for _ in range(n_rec)]
    for z in range(n_rec):
        for y in range(n_rec):
            for x in range(n_rec):
                p = (origin[0] + h * x, origin[1] + h * y, origin[2] + h * z)
                for j in range(len(q)):
                    r = math.dist(p, xyz[j])
                    if r < occ_f * k * sigma[j]:
                        O[z][y][x] = 1
                    lj_r = math.sqrt(eps[j]) * sigma[j] ** 6 / r ** 12 if r > 0 else math.inf
                    if r >= k * sigma[j]:
                        G[0][z][y][x] += 332.05 * q[j] / r
                        G[1][z][y][x] += lj_r
                        G[2][z][y][x] += math.sqrt(eps[j]) * sigma[j] ** 3 / r ** 6
                    elif mode == "cap":
                        G[1][z][y][x] += lj_r
                if mode == "cap":
                    G[1][z][y][x] = min(G[1][z][y][x], cap)
    return G, O


def ligand_grid(u, weights, n_fft):
    """Trilinear spreading of one channel: {(x,y,z) mod n_fft: value}."""
    g = {}
    for ui, wi in zip(u, weights):
        a = [math.floor(c) for c in ui]
        f = [ui[d] - a[d] for d in range(3)]
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    wt = ((f[0] if dx else 1 - f[0]) * (f[1] if dy else 1 - f[1]) *
                          (f[2] if dz else 1 - f[2]))
                    key = ((a[0] + dx) % n_fft, (a[1] + dy) % n_fft, (a[2] + dz) % n_fft)
                    g[key] = g.get(key, 0.0) + wi * wt
    return g


def ligand_occ(u, rho, n_fft):
    """Eq. 10 for the ligand on the periodic grid, exact lattice test."""
    pts = set()
    for ui, r in zip(u, rho):
        U = [round(c * 65536) for c in ui]
        thr = math.ceil(r * r * 4294967296.0)
        lo = [math.floor(ui[d] - r) - 1 for d in range(3)]
        hi = [math.ceil(ui[d] + r) + 1 for d in range(3)]
        for z in range(lo[2], hi[2] + 1):
            for y in range(lo[1], hi[1] + 1):
                for x in range(lo[0], hi[0] + 1):
                    D = (x * 65536 - U[0]) ** 2 + (y * 65536 - U[1]) ** 2 + (z * 65536 - U[2]) ** 2
                    if D < thr:
                        pts.add((x % n_fft, y % n_fft, z % n_fft))
    return pts


def rec_value(G, n_rec, x, y, z):
    if x < n_rec and y < n_rec and z < n_rec:
        return G[z][y][x]
    return 0.0


def energies(G, n_rec, n_fft, u, gamma, box):
    """Psi(t) for box-valid t, as dict {(tx,ty,tz): value}, by Eq. 8."""
    grids = [ligand_grid(u, [g[ch] for g in gamma], n_fft) for ch in range(3)]
    out = {}
    for tz in range(n_rec - box[2]):
        for ty in range(n_rec - box[1]):
            for tx in range(n_rec - box[0]):
                s = 0.0
                for ch in range(3):
                    for (x, y, z), v in grids[ch].items():
                        s += v * rec_value(G[ch], n_rec, (x + tx) % n_fft, (y + ty) % n_fft,
                                           (z + tz) % n_fft)
                out[(tx, ty, tz)] = s
    return out


def overlaps(O, n_rec, n_fft, pts, box):
    out = {}
    for tz in range(n_rec - box[2]):
        for ty in range(n_rec - box[1]):
            for tx in range(n_rec - box[0]):
                out[(tx, ty, tz)] = sum(
                    int(rec_value(O, n_rec, (x + tx) % n_fft, (y + ty) % n_fft, (z + tz) % n_fft))
                    for (x, y, z) in pts)
    return out
