"""Seeded synthetic inputs for the FFT translational BPMF scan.

This module only draws random numbers and lays out arrays: receptor atoms,
ligand atoms and rigid conformers, rotation quaternions, snapshot jitter and
snapshot weights.  It contains none of the method's arithmetic (no grids, no
energies, no placement); both the FP64 oracle and the GPU library consume what
it produces.

The workloads stand in for the paper's T4 lysozyme L99A receptor, its 141
ligands and their parallel-tempering conformers (Methodology, "Ligand
Sampling"), none of which are available.  They keep the paper's shapes:
16 A-class grids at 0.5 / 0.25 A spacing (FFT-based BPMF estimation section),
conformers randomly rotated about their centroid, receptor snapshots with
normalised weights (Eq. 13).

Recipe (all parameters per atom, receptor and ligand alike):
    tiny case (config 1):  q ~ N(0, 0.4) e,  eps ~ U(0.05, 0.2) kcal/mol;
    cavity cases (configs 2-5, an apolar T4L-L99A-like pocket and apolar
    ligands):              q ~ N(0, 0.1) e,  eps ~ U(0.025, 0.1) kcal/mol;
    sigma ~ U(3, 4) A everywhere;
then charges are made locally neutral: receptor atoms are grouped with
their nearest of n/4 random group centres and each group's mean charge is
subtracted; a ligand's mean charge is subtracted.  (Independent charges
give vacuum potentials of ~10^3 kcal/mol/e inside the cavity, far from
any real receptor.)  The cavity cases' scale was set against the spread the
paper reports for BPMFs over ligand configurations (results section,
convergence figure: bootstrap standard deviations of 0.04-0.3 kcal/mol at
about 1000 configurations): with the config-1 parameters the cavity cases
have a single configuration carrying > 99.9 % of the Boltzmann weight and
bootstrap deviations of several kcal/mol, far outside that range; with the
cavity parameters the median over the 141 ligands is ~0.25 kcal/mol.
Ligand geometry: compact self-avoiding random tree (each new atom bonds,
1.5 A away, to a random earlier atom with fewer than three bonds, chosen
with weight exp(-d/1.5 A) by distance d from the centroid; non-bonded
separation >= 2.5 A), the branched shape of drug-like ligands; each extra
conformer is the previous one after three pivot moves (the atoms on one side
of a random bond rotated rigidly about the bond's inner atom), a move being
kept only if it stays self-avoiding and within 1.1x the first conformer's
radius of gyration (gas-phase conformers stay compact).
Rotations: Shoemake's uniform unit quaternions.
Root seed 170807045 split with numpy SeedSequence.spawn.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

ROOT_SEED = 170807045

# stream indices of SeedSequence(ROOT_SEED).spawn(...)
_STREAM_RECEPTOR, _STREAM_LIGANDS, _STREAM_ROTATIONS, _STREAM_JITTER, \
    _STREAM_SPLIT, _STREAM_IS, _STREAM_MLP, _STREAM_MISC = range(8)


def streams(seed: int = ROOT_SEED, n: int = 8):
    """Independent numpy Generators (PCG64) for the named input streams."""
    ss = np.random.SeedSequence(seed)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(n)]


@dataclass
class Receptor:
    xyz: np.ndarray      # f64 [n_snap][n_atoms][3], Angstrom
    q: np.ndarray        # f64 [n_atoms], e
    sigma: np.ndarray    # f64 [n_atoms], Angstrom (r_min form)
    eps: np.ndarray      # f64 [n_atoms], kcal/mol
    weights: np.ndarray  # f64 [n_snap], sums to 1

    @property
    def n_snap(self) -> int:
        return self.xyz.shape[0]


@dataclass
class Ligand:
    q: np.ndarray          # f64 [n_atoms]
    sigma: np.ndarray      # f64 [n_atoms]
    eps: np.ndarray        # f64 [n_atoms]
    conformers: np.ndarray  # f64 [n_conf][n_atoms][3], Angstrom
    cfg_conf: np.ndarray   # i32 [n_cfg] conformer index of each configuration
    cfg_quat: np.ndarray   # f64 [n_cfg][4] unit quaternion (w, x, y, z)

    @property
    def n_atoms(self) -> int:
        return self.q.shape[0]

    @property
    def n_cfg(self) -> int:
        return self.cfg_conf.shape[0]


@dataclass
class Workload:
    name: str
    n_rec: int            # receptor grid edge (points)
    n_fft: int            # FFT edge (points), >= n_rec
    h: float              # grid spacing, Angstrom
    origin: np.ndarray    # f64 [3], position of grid point (0,0,0), Angstrom
    clash_mode: str       # "occ" or "cap"
    ljr_cap: float        # kcal/mol per unit ligand weight (cap mode)
    occ_f: float          # occupancy radius scale f (rho = f 2^-1/6 sigma)
    T: float              # Kelvin
    precision: str        # "f32" or "f64"
    receptor: Receptor
    ligands: List[Ligand] = field(default_factory=list)

    @property
    def n_cfg_total(self) -> int:
        return int(sum(l.n_cfg for l in self.ligands))


# (charge sd in e, eps range in kcal/mol) of the two parameter sets
TINY_PARAMS = (0.4, (0.05, 0.2))
CAVITY_PARAMS = (0.1, (0.025, 0.1))


def atom_params(rng: np.random.Generator, n: int, params=TINY_PARAMS):
    q_sd, (e_lo, e_hi) = params
    q = rng.normal(0.0, q_sd, n)
    sigma = rng.uniform(3.0, 4.0, n)
    eps = rng.uniform(e_lo, e_hi, n)
    return q, sigma, eps


def neutralize_groups(rng: np.random.Generator, xyz: np.ndarray, q: np.ndarray,
                      group: int = 4) -> np.ndarray:
    """Subtract the mean charge of each spatial group (atoms assigned to the
    nearest of n/group random centres)."""
    n = q.shape[0]
    k = max(1, n // group)
    centres = xyz[rng.choice(n, k, replace=False)]
    lab = np.empty(n, np.int64)
    for s in range(0, n, 512):
        d = np.linalg.norm(xyz[s:s + 512, None, :] - centres[None], axis=-1)
        lab[s:s + 512] = np.argmin(d, axis=1)
    out = q.copy()
    for g in range(k):
        m = lab == g
        if np.any(m):
            out[m] -= out[m].mean()
    return out


def uniform_quaternions(rng: np.random.Generator, n: int) -> np.ndarray:
    """Shoemake (Graphics Gems III, 1992): uniform random unit quaternions."""
    u1, u2, u3 = rng.random(n), rng.random(n), rng.random(n)
    a, b = np.sqrt(1.0 - u1), np.sqrt(u1)
    q = np.stack([a * np.sin(2 * np.pi * u2), a * np.cos(2 * np.pi * u2),
                  b * np.sin(2 * np.pi * u3), b * np.cos(2 * np.pi * u3)], axis=1)
    return q  # (w, x, y, z); already unit norm up to rounding


def _random_unit(rng):
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def random_tree(rng, n: int, bond: float = 1.5, min_sep: float = 2.5,
                max_bonds: int = 3):
    """Compact self-avoiding random tree: atom i bonds to a random earlier
    atom with fewer than max_bonds bonds.  Returns (xyz [n][3], parent [n])."""
    while True:
        xyz = np.zeros((n, 3))
        parent = np.full(n, -1, np.int64)
        deg = np.zeros(n, np.int64)
        ok = True
        for i in range(1, n):
            placed = False
            for _ in range(400):
                cands = np.flatnonzero(deg[:i] < max_bonds)
                # compact growth: prefer attachment atoms near the centroid
                dc = np.linalg.norm(xyz[cands] - xyz[:i].mean(axis=0), axis=1)
                pr = np.exp(-(dc - dc.min()) / 1.5)
                a = int(rng.choice(cands, p=pr / pr.sum()))
                cand = xyz[a] + bond * _random_unit(rng)
                others = np.ones(i, bool)
                others[a] = False
                if np.all(np.linalg.norm(xyz[:i][others] - cand, axis=1) >= min_sep):
                    xyz[i], parent[i] = cand, a
                    deg[a] += 1
                    deg[i] += 1
                    placed = True
                    break
            if not placed:
                ok = False
                break
        if ok:
            return xyz, parent


def _rg(xyz: np.ndarray) -> float:
    return float(np.sqrt(np.mean(np.sum((xyz - xyz.mean(axis=0)) ** 2, axis=1))))


def _subtree(parent: np.ndarray, root: int) -> np.ndarray:
    n = parent.shape[0]
    inside = np.zeros(n, bool)
    inside[root] = True
    for i in range(n):  # parents precede children
        if parent[i] >= 0 and inside[parent[i]]:
            inside[i] = True
    return inside


def _quat_matrix_for_inputs(q):
    # rotation used only to reshape synthetic conformers (input generation)
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _self_avoiding(xyz: np.ndarray, parent: np.ndarray, min_sep: float) -> bool:
    n = xyz.shape[0]
    d = np.linalg.norm(xyz[:, None, :] - xyz[None, :, :], axis=-1)
    bonded = np.zeros((n, n), bool)
    for i in range(n):
        if parent[i] >= 0:
            bonded[i, parent[i]] = bonded[parent[i], i] = True
    iu = np.triu_indices(n, k=1)
    return bool(np.all((d[iu] >= min_sep) | bonded[iu]))


def pivot_conformers(rng, base: np.ndarray, parent: np.ndarray, n_conf: int,
                     moves: int = 3, min_sep: float = 2.5) -> np.ndarray:
    """Conformer k+1 = conformer k after `moves` accepted pivot moves: the
    subtree below a random bond is rotated rigidly about the bond's parent
    atom."""
    n = base.shape[0]
    out = [base.copy()]
    cur = base.copy()
    rg0 = _rg(base)
    for _ in range(1, n_conf):
        done = 0
        tries = 0
        while done < moves and tries < 1000 and n >= 3:
            tries += 1
            child = int(rng.integers(1, n))
            piv = int(parent[child])
            sub = _subtree(parent, child)
            R = _quat_matrix_for_inputs(uniform_quaternions(rng, 1)[0])
            cand = cur.copy()
            cand[sub] = (cur[sub] - cur[piv]) @ R.T + cur[piv]
            if _self_avoiding(cand, parent, min_sep) and _rg(cand) <= 1.1 * rg0:
                cur = cand
                done += 1
        out.append(cur.copy())
    return np.stack(out)


def make_ligand(rng_lig, rng_rot, n_atoms: int, n_conf: int, n_rot_per_conf: int,
                params=TINY_PARAMS) -> Ligand:
    q, sigma, eps = atom_params(rng_lig, n_atoms, params)
    q = q - q.mean()
    base, parent = random_tree(rng_lig, n_atoms)
    confs = pivot_conformers(rng_lig, base, parent, n_conf)
    cfg_conf = np.repeat(np.arange(n_conf, dtype=np.int32), n_rot_per_conf)
    cfg_quat = uniform_quaternions(rng_rot, n_conf * n_rot_per_conf)
    return Ligand(q, sigma, eps, confs, cfg_conf, cfg_quat)


def _ball_atoms(rng, n, r_max):
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    r = r_max * rng.random(n) ** (1.0 / 3.0)
    return v * r[:, None]


def _shell_atoms(rng, n, r_in, r_out):
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    r = (r_in ** 3 + (r_out ** 3 - r_in ** 3) * rng.random(n)) ** (1.0 / 3.0)
    return v * r[:, None]


def _grid_origin(center, n_rec, h):
    return np.asarray(center, dtype=np.float64) - 0.5 * (n_rec - 1) * h


def config1(seed: int = ROOT_SEED) -> Workload:
    """Tiny plain case: 300 receptor atoms uniform in a ball of radius 8 A
    centred in a 32^3 grid at 0.5 A; capped LJ repulsion; one 12-atom rigid
    ligand under 100 uniform rotations; FP64; 300 K."""
    rs = streams(seed)
    n_rec, h = 32, 0.5
    xyz = _ball_atoms(rs[_STREAM_RECEPTOR], 300, 8.0)
    q, s, e = atom_params(rs[_STREAM_RECEPTOR], 300)
    q = neutralize_groups(rs[_STREAM_RECEPTOR], xyz, q)
    rec = Receptor(xyz[None], q, s, e, np.ones(1))
    lig = make_ligand(rs[_STREAM_LIGANDS], rs[_STREAM_ROTATIONS], 12, 1, 100)
    return Workload("c1: 300-atom ball, 32^3 @ 0.5 A, cap, 12-atom ligand x 100 rotations, f64",
                    n_rec, 32, h, _grid_origin(np.zeros(3), n_rec, h), "cap", 10.0, 0.5,
                    300.0, "f64", rec, [lig])


def cavity_receptor(rng, n_atoms=2600, r_in=10.0, r_out=19.3, params=CAVITY_PARAMS):
    xyz = _shell_atoms(rng, n_atoms, r_in, r_out)
    q, s, e = atom_params(rng, n_atoms, params)
    q = neutralize_groups(rng, xyz, q)
    return xyz, q, s, e


def config2(seed: int = ROOT_SEED, n_rot: int = 1000, n_conf: int = 8, params=CAVITY_PARAMS) -> Workload:
    """T4L-sized plain case: 2600 atoms in a shell around a 10 A cavity,
    96^3 grid at 0.25 A zero-padded to a 128^3 FFT, occupancy clash mode;
    one 25-atom ligand, 8 rigid conformers x 1000 rotations; FP32.
    params=TINY_PARAMS gives the same geometry with the larger charges and
    well depths of the tiny case (the precision stress)."""
    rs = streams(seed)
    n_rec, h = 96, 0.25
    xyz, q, s, e = cavity_receptor(rs[_STREAM_RECEPTOR], params=params)
    rec = Receptor(xyz[None], q, s, e, np.ones(1))
    lig = make_ligand(rs[_STREAM_LIGANDS], rs[_STREAM_ROTATIONS], 25, n_conf, n_rot, params)
    tag = "" if params == CAVITY_PARAMS else f", q sd {params[0]} e, eps U{params[1]}"
    return Workload("c2: 2600-atom cavity, 96^3 @ 0.25 A -> 128^3 FFT, occ, 25-atom ligand x 8 conf x 1000 rot, f32"
                    + tag, n_rec, 128, h, _grid_origin(np.zeros(3), n_rec, h), "occ", 10.0, 0.5,
                    300.0, "f32", rec, [lig])


def config3(seed: int = ROOT_SEED, n_ligands: int = 141, n_snap: int = 10,
            jitter: float = 0.3, cfg_scale: float = 1.0) -> Workload:
    """Batched case: the config-2 receptor jittered N(0, 0.3 A) into 10
    snapshots (uniform weights); 141 ligands with 8-40 atoms and 200-2000
    configurations (8 conformers x rotations)."""
    rs = streams(seed)
    n_rec, h = 96, 0.25
    xyz, q, s, e = cavity_receptor(rs[_STREAM_RECEPTOR])
    jit = rs[_STREAM_JITTER]
    snaps = np.stack([xyz + jit.normal(0.0, jitter, xyz.shape) for _ in range(n_snap)])
    rec = Receptor(snaps, q, s, e, np.full(n_snap, 1.0 / n_snap))
    rl, rr, rm = rs[_STREAM_LIGANDS], rs[_STREAM_ROTATIONS], rs[_STREAM_MISC]
    ligs = []
    for _ in range(n_ligands):
        na = int(rm.integers(8, 41))
        ncfg = int(rm.integers(200, 2001))
        ncfg = max(8, int(round(ncfg * cfg_scale / 8.0)) * 8)
        ligs.append(make_ligand(rl, rr, na, 8, ncfg // 8, CAVITY_PARAMS))
    return Workload("c3: 141 ligands (8-40 atoms, 200-2000 cfgs) x 10 snapshots, 128^3 FFT, occ, f32",
                    n_rec, 128, h, _grid_origin(np.zeros(3), n_rec, h), "occ", 10.0, 0.5,
                    300.0, "f32", rec, ligs)


def config6(seed: int = ROOT_SEED, n_rot: int = 1000, n_conf: int = 8) -> Workload:
    """Whole-surface case: the config-2 receptor and ligand on a 62 A grid at
    0.25 A (248 points) zero-padded to a 256^3 FFT, covering the entire
    receptor surface (the paper's larger grid); occupancy mode, FP32."""
    w = config2(seed, n_rot, n_conf)
    n_rec, h = 248, 0.25
    return Workload("c6: 2600-atom cavity receptor, 248^3 @ 0.25 A (62 A) -> 256^3 FFT, occ, "
                    f"25-atom ligand x {n_conf} conf x {n_rot} rot, f32",
                    n_rec, 256, h, _grid_origin(np.zeros(3), n_rec, h), "occ", 10.0, 0.5,
                    300.0, "f32", w.receptor, w.ligands)


def tiny(seed: int = 1, n_rec: int = 8, n_fft: Optional[int] = None, h: float = 1.0,
         n_rec_atoms: int = 6, n_lig_atoms: int = 2, n_cfg: int = 3,
         clash_mode: str = "occ", occ_f: float = 0.5, precision: str = "f64",
         n_snap: int = 1, r_ball: Optional[float] = None) -> Workload:
    """Very small random case for brute-force checks."""
    rs = streams(seed)
    n_fft = n_fft or n_rec
    r_ball = r_ball if r_ball is not None else 0.5 * (n_rec - 1) * h
    xyz = _ball_atoms(rs[_STREAM_RECEPTOR], n_rec_atoms, r_ball)
    q, s, e = atom_params(rs[_STREAM_RECEPTOR], n_rec_atoms)
    if n_rec_atoms >= 8:
        q = neutralize_groups(rs[_STREAM_RECEPTOR], xyz, q)
    snaps = np.stack([xyz + rs[_STREAM_JITTER].normal(0, 0.3, xyz.shape) if k else xyz
                      for k in range(n_snap)])
    rec = Receptor(snaps, q, s, e, np.full(n_snap, 1.0 / n_snap))
    lig = make_ligand(rs[_STREAM_LIGANDS], rs[_STREAM_ROTATIONS], n_lig_atoms, 1, n_cfg)
    return Workload("tiny", n_rec, n_fft, h, _grid_origin(np.zeros(3), n_rec, h),
                    clash_mode, 10.0, occ_f, 300.0, precision, rec, [lig])


def subset(w: Workload, n_cfg: int, lig: int = 0, stride: int = 1) -> Workload:
    """Same workload restricted to the first n_cfg (every stride-th)
    configurations of one ligand."""
    L = w.ligands[lig]
    sel = np.arange(0, L.n_cfg, stride)[:n_cfg]
    L2 = Ligand(L.q, L.sigma, L.eps, L.conformers, L.cfg_conf[sel].copy(), L.cfg_quat[sel].copy())
    return Workload(w.name + f" [subset {len(sel)} cfgs]", w.n_rec, w.n_fft, w.h, w.origin,
                    w.clash_mode, w.ljr_cap, w.occ_f, w.T, w.precision, w.receptor, [L2])


def uniforms(seed: int, n: int) -> np.ndarray:
    """Uniform(0,1) draws handed to samplers as inputs (f64)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([ROOT_SEED, seed]))).random(n)
