"""FP64 CPU oracle for the FFT translational BPMF scan.

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's CPU
baseline may use it; the product package never imports it, and it imports
nothing from the product package.  It shares no code with the GPU path; the
only common module is `workload.synth`, which draws inputs.

`oracle.c` holds the per-translation definitions (Eq. 7 grids, placement,
the direct trilinear form of Eq. 8, the clash test of Eq. 10, partial sums of
Eq. 2); `estimators.py` holds the averages of Eqs. 2, 12 and 13 and the
importance-sampling estimators; `mlp.py` the FP64 network.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (FP64, OpenMP)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_SO)
        d, i, p = ctypes.c_double, ctypes.c_int, ctypes.c_void_p
        L.orc_receptor_grids.argtypes = [i, p, p, p, p, i, d, p, i, d, d, p, p]
        L.orc_receptor_grids.restype = None
        L.orc_ligand_weights.argtypes = [i, p, p, p, p]
        L.orc_ligand_weights.restype = None
        L.orc_occ_threshold.argtypes = [d, d, d]
        L.orc_occ_threshold.restype = d
        L.orc_place.argtypes = [i, p, p, d, p, p]
        L.orc_place.restype = i
        L.orc_direct_energy.argtypes = [i, i, p, i, p, p, p, p, p]
        L.orc_direct_energy.restype = None
        L.orc_clash.argtypes = [i, i, p, i, p, p, p, p]
        L.orc_clash.restype = i
        L.orc_partial.argtypes = [ctypes.c_longlong, p, p, d, p]
        L.orc_partial.restype = None
        L.orc_scan.argtypes = [i, i, p, p, d, i, p, p, p, i, p, p, d, i, p, p]
        L.orc_scan.restype = i
        L.orc_spread_dense.argtypes = [i, i, p, p, p]
        L.orc_spread_dense.restype = None
        L.orc_occ_dense.argtypes = [i, i, p, p, p]
        L.orc_occ_dense.restype = i
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


R_KCAL = 1.987204259e-3   # kcal mol^-1 K^-1
C_STANDARD = 6.02214076e-4  # 1 M in molecules per A^3


def kT(T: float) -> float:
    return R_KCAL * T


# ---------------------------------------------------------------- grids
def receptor_grids(w, snap: int = 0):
    """Eq. 7 grids [3][n_rec^3] (ELE, LJr, LJa) and Eq. 10 occupancy
    [n_rec^3] (None in cap mode) for one receptor snapshot, FP64."""
    r = w.receptor
    n = w.n_rec
    g = np.zeros((3, n, n, n))
    occ = np.zeros((n, n, n), np.uint8) if w.clash_mode == "occ" else None
    mode = 0 if w.clash_mode == "occ" else 1
    xyz = _f64(r.xyz[snap])
    q, s, e, o = _f64(r.q), _f64(r.sigma), _f64(r.eps), _f64(w.origin)
    lib().orc_receptor_grids(xyz.shape[0], _p(xyz), _p(q), _p(s), _p(e), n, w.h, _p(o), mode,
                             w.ljr_cap, w.occ_f, _p(g), _p(occ) if occ is not None else None)
    return g, occ


def ligand_weights(lig) -> np.ndarray:
    q, s, e = _f64(lig.q), _f64(lig.sigma), _f64(lig.eps)
    g = np.zeros((q.shape[0], 3))
    lib().orc_ligand_weights(q.shape[0], _p(q), _p(s), _p(e), _p(g))
    return g


def occ_thresholds(lig, occ_f: float, h: float) -> np.ndarray:
    return np.array([lib().orc_occ_threshold(float(s), occ_f, h) for s in lig.sigma])


# ---------------------------------------------------------------- placement
def place(conf_xyz: np.ndarray, quat: np.ndarray, h: float):
    """Placed lattice coordinates u [n][3] (grid units) and box [3]."""
    x = _f64(conf_xyz)
    qq = _f64(quat)
    u = np.zeros_like(x)
    box = np.zeros(3, np.int32)
    rc = lib().orc_place(x.shape[0], _p(x), _p(qq), h, _p(u), _p(box))
    if rc != 0:
        raise ValueError("zero quaternion")
    return u, box


def place_cfg(w, lig_idx: int, cfg: int):
    L = w.ligands[lig_idx]
    return place(L.conformers[L.cfg_conf[cfg]], L.cfg_quat[cfg], w.h)


def valid_shape(w, box):
    return tuple(int(max(w.n_rec - b, 0)) for b in box[::-1])  # (Vz, Vy, Vx)


# ---------------------------------------------------------------- energies
def direct_energy(w, grids, u, gamma, box, mask=None) -> np.ndarray:
    """Raw Psi at every box-valid translation, array [Vz][Vy][Vx]."""
    Vz, Vy, Vx = valid_shape(w, box)
    psi = np.zeros((Vz, Vy, Vx))
    if psi.size == 0:
        return psi
    g = _f64(grids)
    uu, gm = _f64(u), _f64(gamma)
    b = np.ascontiguousarray(box, np.int32)
    m = None if mask is None else np.ascontiguousarray(mask, np.uint8)
    lib().orc_direct_energy(w.n_rec, w.n_fft, _p(g), uu.shape[0], _p(uu), _p(gm), _p(b),
                            _p(m) if m is not None else None, _p(psi))
    return psi


def clash(w, occ, u, thr, box) -> np.ndarray:
    Vz, Vy, Vx = valid_shape(w, box)
    out = np.zeros((Vz, Vy, Vx), np.uint8)
    if out.size == 0:
        return out
    o = np.ascontiguousarray(occ, np.uint8)
    uu, tt = _f64(u), _f64(thr)
    b = np.ascontiguousarray(box, np.int32)
    rc = lib().orc_clash(w.n_rec, w.n_fft, _p(o), uu.shape[0], _p(uu), _p(tt), _p(b), _p(out))
    if rc < 0:
        raise MemoryError
    return out


def partial(psi, clash_mask, beta):
    """(m, s, n_valid, n_finite, psi_min, argmin) over one configuration."""
    ps = _f64(psi).ravel()
    cm = None if clash_mask is None else np.ascontiguousarray(clash_mask, np.uint8).ravel()
    out = np.zeros(6)
    lib().orc_partial(ps.shape[0], _p(ps), _p(cm) if cm is not None else None, beta, _p(out))
    return out


def config_eval(w, grids, occ, lig_idx, cfg):
    """Everything for one configuration: u, box, raw psi, clash mask, partial."""
    L = w.ligands[lig_idx]
    u, box = place_cfg(w, lig_idx, cfg)
    gamma = ligand_weights(L)
    psi = direct_energy(w, grids, u, gamma, box)
    cl = None
    if w.clash_mode == "occ":
        cl = clash(w, occ, u, occ_thresholds(L, w.occ_f, w.h), box)
    beta = 1.0 / kT(w.T)
    return dict(u=u, box=box, psi=psi, clash=cl, partial=partial(psi, cl, beta))


def scan(w, grids, occ, lig_idx: int = 0, cfgs=None, raw_everywhere: bool = False):
    """Per-configuration partials [n][6] and boxes [n][3] for one ligand
    against one snapshot (OpenMP over configurations)."""
    L = w.ligands[lig_idx]
    sel = np.arange(L.n_cfg) if cfgs is None else np.asarray(cfgs)
    conf = _f64(L.conformers)
    gamma = ligand_weights(L)
    thr = occ_thresholds(L, w.occ_f, w.h)
    cc = np.ascontiguousarray(L.cfg_conf[sel], np.int32)
    qq = _f64(L.cfg_quat[sel])
    out = np.zeros((sel.shape[0], 6))
    boxes = np.zeros((sel.shape[0], 3), np.int32)
    g = _f64(grids)
    o = None if occ is None else np.ascontiguousarray(occ, np.uint8)
    rc = lib().orc_scan(w.n_rec, w.n_fft, _p(g), _p(o) if o is not None else None, w.h,
                        L.n_atoms, _p(conf), _p(gamma), _p(thr), sel.shape[0], _p(cc), _p(qq),
                        1.0 / kT(w.T), int(raw_everywhere), _p(out), _p(boxes))
    if rc != 0:
        raise RuntimeError("oracle scan failed")
    return out, boxes


def spread_dense(n_fft, u, weights):
    out = np.zeros((n_fft, n_fft, n_fft))
    uu, ww = _f64(u), _f64(weights)
    lib().orc_spread_dense(n_fft, uu.shape[0], _p(uu), _p(ww), _p(out))
    return out


def occ_dense(n_fft, u, thr):
    out = np.zeros((n_fft, n_fft, n_fft), np.uint8)
    uu, tt = _f64(u), _f64(thr)
    rc = lib().orc_occ_dense(n_fft, uu.shape[0], _p(uu), _p(tt), _p(out))
    if rc < 0:
        raise MemoryError
    return out
