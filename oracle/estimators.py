"""FP64 estimators of the oracle (test infrastructure only).

Each function is the plain formula from the paper, in double precision:
  - sample-mean BPMF, Eq. 2, pooled over every (configuration, translation)
    sample including the infinite (clash) ones;
  - binding-site volume V_site of the standard-binding-free-energy section
    (average box-valid region, counted in grid points times h^3);
  - standard binding free energy, Eqs. 12-13, with the sign reading
    -kT ln(V_site C0) (Omega / 8 pi^2 = V_site);
  - the importance-sampled form of Eq. 2 over configurations;
  - not in the paper: the learned proposal's stratified sampling plan
    (exact top stratum + defensive-mixture draws, weighted forms of Eq. 2)
    and the per-configuration scan descriptors it takes as inputs.
Partials are rows (m, s, n_valid, n_finite, psi_min, argmin) with
x = -beta Psi, m = max x and s = sum exp(x - m) over one configuration.
"""
from __future__ import annotations

import math

import numpy as np

R_KCAL = 1.987204259e-3
C_STANDARD = 6.02214076e-4  # 1 mol/L in A^-3


def kT(T: float) -> float:
    return R_KCAL * T


def log_z(partials: np.ndarray) -> np.ndarray:
    """ln Z_c = m_c + ln s_c per configuration (-inf if nothing finite)."""
    p = np.asarray(partials, dtype=np.float64)
    out = np.full(p.shape[0], -np.inf)
    ok = p[:, 3] > 0
    out[ok] = p[ok, 0] + np.log(p[ok, 1])
    return out


def lse(x: np.ndarray) -> float:
    """max-shifted log-sum-exp in FP64; -inf for an empty or all -inf set."""
    x = np.asarray(x, dtype=np.float64)
    if x.size == 0:
        return -math.inf
    m = np.max(x)
    if m == -math.inf:
        return -math.inf
    return float(m + math.log(np.sum(np.exp(x - m))))


def bpmf(partials: np.ndarray, T: float) -> float:
    """Eq. 2 pooled over all configurations of one ligand and one snapshot:
    B = -kT [ ln sum_c Z_c - ln sum_c n_c ];  +inf if nothing is finite."""
    p = np.asarray(partials, dtype=np.float64)
    n = float(np.sum(p[:, 2]))
    lz = lse(log_z(p))
    if lz == -math.inf or n <= 0:
        return math.inf
    return -kT(T) * (lz - math.log(n))


def bpmf_naive(psi_all: np.ndarray, T: float) -> float:
    """Eq. 2 literally: -kT ln (1/N) sum exp(-beta Psi) (no shift)."""
    beta = 1.0 / kT(T)
    psi_all = np.asarray(psi_all, dtype=np.float64)
    return -kT(T) * math.log(np.mean(np.exp(-beta * psi_all)))


def v_site(boxes: np.ndarray, n_rec: int, h: float) -> float:
    """V_site = h^3 * mean over configurations of the number of box-valid
    translations, prod_d (n_rec - box_d)."""
    b = np.asarray(boxes, dtype=np.int64)
    v = np.clip(n_rec - b, 0, None)
    return float(h ** 3 * np.mean(np.prod(v, axis=1)))


def dg_standard(B: np.ndarray, W: np.ndarray, vsite: float, T: float) -> float:
    """Eq. 13 with the reading -kT ln(V_site C0):
    dG = -kT ln sum_s W_s exp(-beta B_s) - kT ln(V_site C0)."""
    B = np.asarray(B, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    W = W / np.sum(W)
    beta = 1.0 / kT(T)
    fin = np.isfinite(B) & (W > 0)
    if not np.any(fin):
        return math.inf
    x = np.log(W[fin]) - beta * B[fin]
    return -kT(T) * lse(x) - kT(T) * math.log(vsite * C_STANDARD)


def bpmf_is(logz_cfg: np.ndarray, n_total: float, idx: np.ndarray, q: np.ndarray,
            T: float) -> float:
    """Importance-sampled Eq. 2 over configurations:
    Z_hat = (1/K) sum_k Z_{c_k} / q_{c_k};  B_hat = -kT ln(Z_hat / n_total)."""
    lz = np.asarray(logz_cfg, dtype=np.float64)[idx]
    lq = np.log(np.asarray(q, dtype=np.float64)[idx])
    K = len(idx)
    val = lse(lz - lq) - math.log(K)
    if val == -math.inf:
        return math.inf
    return -kT(T) * (val - math.log(n_total))


def proposal(yhat: np.ndarray, alpha: float, tau: float) -> np.ndarray:
    """Defensive mixture q = (1 - alpha) softmax(yhat / tau) + alpha / P."""
    y = np.asarray(yhat, dtype=np.float64) / tau
    y = y - np.max(y)
    e = np.exp(y)
    P = y.shape[0]
    return (1.0 - alpha) * e / np.sum(e) + alpha / P


def inverse_cdf_sample(q: np.ndarray, uniforms: np.ndarray) -> np.ndarray:
    """Index k with cdf[k-1] <= u < cdf[k], cdf the running sum of q taken
    left to right (FP64)."""
    cdf = np.cumsum(np.asarray(q, dtype=np.float64))
    u = np.asarray(uniforms, dtype=np.float64) * cdf[-1]
    return np.minimum(np.searchsorted(cdf, u, side="right"), len(q) - 1)


def bpmf_weighted(logz_cfg: np.ndarray, n_total: float, weight: np.ndarray, T: float) -> float:
    """Eq. 2 with per-configuration weights w_c >= 0 on the numerator:
    B = -kT [ ln sum_{w_c > 0} w_c Z_c - ln n_total ]; +inf if the sum is 0."""
    lz = np.asarray(logz_cfg, dtype=np.float64)
    w = np.asarray(weight, dtype=np.float64)
    ok = (w > 0) & np.isfinite(lz)
    val = lse(np.log(w[ok]) + lz[ok]) if np.any(ok) else -math.inf
    if val == -math.inf or n_total <= 0:
        return math.inf
    return -kT(T) * (val - math.log(n_total))


def stratified_plan(yhat: np.ndarray, cfg_off: np.ndarray, top_frac: float, draw_frac: float,
                    alpha: float, tau: float, uniforms: np.ndarray):
    """Stratified importance sampling over each ligand's configurations
    (not in the paper; the proposal's sampling plan).  Per ligand of P
    configurations: the ceil(top_frac P) largest yhat (ties to the lower
    index) form an exact stratum (weight 1); the remaining R, in index order,
    are sampled K = ceil(draw_frac P) times from the defensive mixture over
    them (`proposal`, `inverse_cdf_sample`), each drawn one weighted
    multiplicity / (K q).  Uniforms are consumed ligand by ligand.  Returns
    (select uint8: 1 exact stratum, 2 drawn, 0 not scanned; weight float64)
    over all configurations."""
    y = np.asarray(yhat, dtype=np.float64)
    u = np.asarray(uniforms, dtype=np.float64)
    sel = np.zeros(y.size, np.uint8)
    wt = np.zeros(y.size)
    used = 0
    for l in range(len(cfg_off) - 1):
        a, b = int(cfg_off[l]), int(cfg_off[l + 1])
        P = b - a
        if P == 0:
            continue
        nt = min(P, math.ceil(top_frac * P))
        order = sorted(range(P), key=lambda j: (-y[a + j], j))
        top = np.zeros(P, bool)
        top[order[:nt]] = True
        sel[a:b][top] = 1
        wt[a:b][top] = 1.0
        rest = np.flatnonzero(~top)
        K = math.ceil(draw_frac * P) if rest.size else 0
        if K == 0:
            continue
        q = proposal(y[a + rest], alpha, tau)
        draws = inverse_cdf_sample(q, u[used:used + K])
        used += K
        mult = np.bincount(draws, minlength=rest.size)
        hit = mult > 0
        sel[a + rest[hit]] = 2
        wt[a + rest[hit]] = mult[hit] / (K * q[hit])
    return sel, wt


def scan_features(parts_by_snap, W: np.ndarray, cfg_off: np.ndarray) -> np.ndarray:
    """Per-configuration scan descriptors (the proposal network's inputs
    taken from a finished scan): x_c = ln sum_s W_s Z_{c,s} (W normalised),
    psi_c = min_s psi_min, f_c = sum_s n_finite / sum_s n_valid; returned as
    (max(x_c - max_l x, -25) / 5, min(psi_c - min_l psi, 50) / 10, f_c), max_l
    and min_l over the ligand's configurations; (-5, 5, 0) when nothing is
    finite.  parts_by_snap: [n_snap][n_cfg][6] partial rows."""
    p = np.asarray(parts_by_snap, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    W = W / W.sum()
    S, C = p.shape[0], p.shape[1]
    x = np.full(C, -math.inf)
    for c in range(C):
        terms = [math.log(W[s]) + log_z(p[s, c:c + 1])[0] for s in range(S) if W[s] > 0]
        x[c] = lse(np.array(terms)) if terms else -math.inf
    psi = p[:, :, 4].min(axis=0)
    nv = p[:, :, 2].sum(axis=0)
    f = np.where(nv > 0, p[:, :, 3].sum(axis=0) / np.where(nv > 0, nv, 1), 0.0)
    out = np.zeros((C, 3))
    for l in range(len(cfg_off) - 1):
        a, b = int(cfg_off[l]), int(cfg_off[l + 1])
        if b == a:
            continue
        X, PM = np.max(x[a:b]), np.min(psi[a:b])
        for c in range(a, b):
            out[c, 0] = max(x[c] - X, -25.0) / 5.0 if np.isfinite(x[c]) else -5.0
            out[c, 1] = min(psi[c] - PM, 50.0) / 10.0 if np.isfinite(psi[c]) else 5.0
            out[c, 2] = f[c]
    return out


def sample_poses(partials: np.ndarray, energies, T: float, uniforms: np.ndarray):
    """Sampling importance resampling of poses (solvation section: K poses
    drawn from the scanned bound state with weight exp(-Psi/kT)), in two
    inverse-CDF steps with the uniforms u[2k], u[2k+1]:
      configuration: running sum over configurations in index order of
        Z_c = exp(m_c - max m) s_c (configurations with nothing finite weigh 0);
      translation: running sum over the configuration's clash-free
        translations in linear (tz, ty, tx) order of exp(-(Psi - min Psi)/kT).
    A draw takes the first running sum exceeding u times the total.
    partials: rows of one ligand and snapshot; energies(c) -> (psi [Vz][Vy][Vx],
    clash mask or None).  Returns (cfg [K], t [K][3] as (tx, ty, tz), psi [K])."""
    p = np.asarray(partials, dtype=np.float64)
    u = np.asarray(uniforms, dtype=np.float64)
    K = u.size // 2
    fin = p[:, 3] > 0
    if not np.any(fin):
        raise ValueError("no clash-free translation to draw")
    M = np.max(p[fin, 0])
    z = np.where(fin, np.exp(np.where(fin, p[:, 0], M) - M) * p[:, 1], 0.0)
    cdf = np.cumsum(z)
    cfg = np.minimum(np.searchsorted(cdf, u[0::2][:K] * cdf[-1], side="right"), len(z) - 1)
    t = np.zeros((K, 3), np.int64)
    psi_k = np.zeros(K)
    beta = 1.0 / kT(T)
    for c in np.unique(cfg):
        psi, clash = energies(int(c))
        Vz, Vy, Vx = psi.shape
        f = psi.ravel()
        ok = np.ones(f.size, bool) if clash is None else ~np.asarray(clash, bool).ravel()
        w = np.where(ok, np.exp(-beta * (f - np.min(f[ok]))), 0.0)
        cw = np.cumsum(w)
        ks = np.flatnonzero(cfg == c)
        lin = np.minimum(np.searchsorted(cw, u[2 * ks + 1] * cw[-1], side="right"), f.size - 1)
        t[ks, 0] = lin % Vx
        t[ks, 1] = (lin // Vx) % Vy
        t[ks, 2] = lin // (Vx * Vy)
        psi_k[ks] = f[lin]
    return cfg, t, psi_k
