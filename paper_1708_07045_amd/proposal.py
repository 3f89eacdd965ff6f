"""Learned importance sampling over ligand configurations (driver).

Not part of the paper.  Eq. 2 pools every configuration of a ligand; when a
few configurations carry most of the Boltzmann weight, a subset chosen with a
proposal close to those weights estimates the same sum with fewer scans.
Z_{c,s} = sum_t exp(-Psi/kT) is configuration c's weight in snapshot s.

Pipeline, each step a library call (this module only arranges them):
  1. a coarse-spacing context (twice the spacing, half the grid edge) scans
     every configuration: about 1/12 of the cost of the fine scan;
  2. per-configuration inputs: fftdg_config_features (rotation, conformer,
     size, extent) and fftdg_scan_features of the coarse scan;
  3. the network (fftdg_mlp, BF16 MFMA) predicts each configuration's
     relative log weight ln sum_s W_s Z_{c,s} - max (in units of 5 nats, the
     scale of the scan descriptors); it is trained with the library's Adam
     step on exhaustive fine scans of training ligands, the targets being
     fftdg_scan_features of those scans.  In the residual form the coarse
     scan's own relative log weight is added to the output (a skip
     connection with no parameters): the network learns fine - coarse and,
     with its output layer started at zero, starts from the coarse ranking;
  4. fftdg_is_plan: the top fraction by prediction is scanned exactly, the
     rest sampled from a defensive mixture with 1/q weights;
  5. fftdg_scan with cfg_select, fftdg_reduce with cfg_weight: unbiased
     B_s and dG;
  6. fallback: a ligand whose predicted weights put more than `max_share`
     of the total outside the exact stratum is scanned exhaustively.  The
     rule depends on the predictions only, fixed before any draw, so each
     ligand's estimate of sum_c Z_c stays unbiased; the share the sampled
     stratum actually carries is reported as a diagnostic.
"""
from __future__ import annotations

from typing import Optional

import numpy as np

from . import _lib as fd

KCAL_R = 1.987204259e-3
N_IN_FULL = fd.N_FEATURES + fd.N_SCAN_FEATURES


def coarse_desc(w, factor: int = 2) -> dict:
    """Grid of a coarse context covering the same box: spacing x factor,
    edges / factor."""
    n_rec = w.n_rec // factor
    h = w.h * factor
    centre = np.asarray(w.origin, np.float64) + 0.5 * (w.n_rec - 1) * w.h
    return dict(n_rec=n_rec, n_fft=w.n_fft // factor, h=h, origin=centre - 0.5 * (n_rec - 1) * h)


def make_context(w, grid: Optional[dict] = None, device: int = 0, snapshots=None,
                 clash_mode: Optional[str] = None):
    """Context with receptor grids of every snapshot (or of the listed ones,
    equally weighted; or, with snapshots == "mean", of one receptor at the
    snapshots' mean atom coordinates) built and set.  clash_mode overrides
    the workload's (a coarse pre-scan may cap the repulsion instead of
    excluding overlaps: one inverse channel instead of two)."""
    import torch
    g = dict(n_rec=w.n_rec, n_fft=w.n_fft, h=w.h, origin=w.origin)
    if grid:
        g.update(grid)
    mode = clash_mode or w.clash_mode
    ctx = fd.FFTDG(g["n_rec"], g["n_fft"], g["h"], g["origin"], w.precision, mode, w.ljr_cap, w.occ_f,
                   device)
    if isinstance(snapshots, str) and snapshots == "mean":
        structures = [np.mean(np.asarray(w.receptor.xyz, np.float64), axis=0)]
        wts = np.ones(1)
    else:
        snaps = list(range(w.receptor.n_snap)) if snapshots is None else list(snapshots)
        structures = [w.receptor.xyz[s] for s in snaps]
        wts = w.receptor.weights if snapshots is None else np.full(len(snaps), 1.0 / len(snaps))
    gl, ol = [], []
    for xyz in structures:
        gg, oo = ctx.receptor_grids(xyz, w.receptor.q, w.receptor.sigma, w.receptor.eps)
        gl.append(gg)
        ol.append(oo)
    grids = torch.stack(gl).contiguous()
    occ = torch.stack(ol).contiguous() if mode == "occ" else None
    ctx.set_receptors(grids, occ, wts)
    ctx._grids = (grids, occ)
    return ctx


def inputs(ctx_fine, ctx_coarse, batch, part_coarse, with_scan: bool = True):
    """Device float matrix [n_cfg][N_FEATURES (+ N_SCAN_FEATURES)]."""
    import torch
    F = ctx_fine.features(batch)
    n_in = N_IN_FULL if with_scan else fd.N_FEATURES
    X = torch.zeros((batch.n_cfg, n_in), dtype=torch.float32, device=ctx_fine.device)
    X[:, :fd.N_FEATURES] = torch.as_tensor(F, device=ctx_fine.device)
    if with_scan:
        ctx_coarse.scan_features(batch, part_coarse, X, fd.N_FEATURES)
    return X


def targets(ctx_fine, batch, part_fine):
    """(t [n_cfg] relative log weight / 5 on the device, loss weights): the
    first scan descriptor of an exhaustive fine scan; configurations within
    5 nats of their ligand's best weigh 10x."""
    import torch
    D = torch.zeros((batch.n_cfg, fd.N_SCAN_FEATURES), dtype=torch.float32, device=ctx_fine.device)
    ctx_fine.scan_features(batch, part_fine, D, 0)
    t = D[:, 0].contiguous()
    w = np.where(t.cpu().numpy() > -1.0, 10.0, 1.0).astype(np.float32)
    return t, torch.as_tensor(w, device=ctx_fine.device)


def targets_snapmax(P_fine, cfg_off, device=None):
    """(t [n_cfg], loss weights) for the per-snapshot criterion: t_c =
    max_s (ln Z_{c,s} - max_{c' of the ligand} ln Z_{c',s}), floored at -25
    and divided by 5 (the descriptor units), from exhaustive fine partials
    [n_snap][n_cfg] (host FP64).  A configuration that dominates any one
    snapshot scores 0 even when that snapshot's total is small, which the
    snapshot-summed descriptor hides.  Configurations within 5 nats of the
    top in some snapshot weigh 10x."""
    import torch
    fin = P_fine["n_finite"] > 0
    lz = np.where(fin, P_fine["m"] + np.log(np.where(fin, P_fine["s"], 1.0)), -np.inf)
    off = np.asarray(cfg_off, np.int64)
    t = np.full(lz.shape[1], -5.0)
    for l in range(off.size - 1):
        a, b = off[l], off[l + 1]
        if b == a:
            continue
        seg = lz[:, a:b]
        m = np.max(seg, axis=1, keepdims=True)
        rel = np.where(np.isfinite(m), seg - np.where(np.isfinite(m), m, 0.0), -np.inf)
        t[a:b] = np.maximum(np.max(rel, axis=0), -25.0) / 5.0
    w = np.where(t > -1.0, 10.0, 1.0).astype(np.float32)
    dev = device if device is not None else "cpu"
    return torch.as_tensor(t.astype(np.float32), device=dev), torch.as_tensor(w, device=dev)


def coarse_score(ctx_coarse, batch, part_coarse) -> np.ndarray:
    """The coarse scan's prediction of the fine target, host float [n_cfg]
    in units of 5 nats: max over the coarse context's receptors of the
    configuration's relative log weight (targets_snapmax of the coarse
    partials).  With one coarse receptor it equals the first scan
    descriptor."""
    P = ctx_coarse.partials_numpy(part_coarse, ctx_coarse.n_snap, batch.n_cfg)
    t, _ = targets_snapmax(P, batch.cfg_off)
    return t.numpy()


def init_params(n_in: int, width: int, seed: int = 0, zero_output: bool = False) -> np.ndarray:
    """Flat FP32 parameters (fftdg_mlp layout), each weight and bias
    uniform in +-1/sqrt(fan_in); zero_output starts the output layer at zero
    (the residual form then starts from its skip input)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([170807045, 5, seed])))
    out = []
    for li, (rows, cols) in enumerate(((width, n_in), (width, width), (width, width), (1, width))):
        a = 0.0 if (zero_output and li == 3) else 1.0 / np.sqrt(cols)
        out.append(rng.uniform(-a, a, rows * cols))
        out.append(rng.uniform(-a, a, rows))
    return np.concatenate(out).astype(np.float32)


def make_network(n_in: int, width: int = 256, residual: bool = False, max_batch: int = 512):
    """The proposal network; residual: the output adds the coarse scan's
    relative log weight (input column N_FEATURES, same units as the target)
    and the output layer starts at zero."""
    net = fd.Network(n_in, width, max_batch)
    net.set_params(init_params(n_in, width, zero_output=residual))
    if residual:
        net.set_skip(fd.N_FEATURES, 1.0)
    return net


def train(net, X, t, w, rows: np.ndarray, epochs: int = 20, batch: int = 512, lr: float = 1e-3,
          seed: int = 0, log=None, checkpoint=None):
    """Adam with the library's kernels over the given rows (device tensors
    X, t, w); the learning rate decays linearly to lr/10.  checkpoint(epoch)
    is called before the first epoch (0) and after each one.  Returns the
    last batch loss of each epoch."""
    import torch
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([170807045, 7, seed])))
    rows = np.asarray(rows, np.int32)
    n_steps = epochs * max(1, rows.size // batch)
    step, hist = 0, []
    if checkpoint:
        checkpoint(0)
    for ep in range(epochs):
        idx = torch.as_tensor(rows[rng.permutation(rows.size)], device=X.device)
        last = None
        nb = max(1, rows.size // batch)
        for k in range(nb):
            f = 1.0 - 0.9 * step / max(1, n_steps - 1)
            last = net.train_step(X, t, w, idx[k * batch:(k + 1) * batch], lr * f, want_loss=(k == nb - 1))
            step += 1
        hist.append(last)
        if log:
            log(f"epoch {ep + 1}/{epochs}: batch loss {last:.4f}")
        if checkpoint:
            checkpoint(ep + 1)
    return hist


def predict(net, X):
    """Network prediction (device float [n]), in units of 5 nats."""
    return net.forward(X)


def predicted_remainder(batch, yhat, top_frac: float) -> np.ndarray:
    """Per ligand: the share of the predicted weight sum_c exp(5 yhat_c)
    outside the ceil(top_frac P) largest predictions (a function of the
    predictions alone)."""
    y = 5.0 * np.asarray(yhat, np.float64)
    out = np.zeros(batch.n_lig)
    for l in range(batch.n_lig):
        a, b = batch.cfg_off[l], batch.cfg_off[l + 1]
        v = np.sort(y[a:b])[::-1]
        nt = min(v.size, int(np.ceil(top_frac * v.size)))
        e = np.exp(v - v[0])
        out[l] = e[nt:].sum() / e.sum()
    return out


def is_estimate(ctx, batch, yhat, top_frac: float, draw_frac: float, alpha: float, tau: float, uniforms,
                T: float, max_share: float = 0.5):
    """Importance-sampled B [n_lig][n_snap] and per-ligand results from one
    plan, with the exhaustive fallback per ligand decided before any draw:
    a ligand goes to the exhaustive scan when its predictions put more than
    max_share of their weight outside the exact stratum.

    yhat is in units of 5 nats, so the mixture's temperature is tau / 5 in
    those units (tau in nats).  Returns dict(B, res, n_scanned (per ligand:
    every configuration scanned for it), fallback (per ligand, bool),
    share (per ligand: the largest fraction of a snapshot's estimate that
    came from sampled configurations, a diagnostic))."""
    yh = np.asarray(yhat.cpu().numpy() if hasattr(yhat, "cpu") else yhat, np.float64)
    fallback = predicted_remainder(batch, yh, top_frac) > max_share
    sel, wt, _ = ctx.is_plan(batch, yhat, top_frac, draw_frac, alpha, tau / 5.0, uniforms)
    for l in np.flatnonzero(fallback):  # those ligands are scanned whole instead
        a, b = batch.cfg_off[l], batch.cfg_off[l + 1]
        sel[a:b] = 1
        wt[a:b] = 1.0
    bsel = batch.with_select(sel)
    part = ctx.scan(bsel, T)
    B, res = ctx.reduce(bsel, part, T, cfg_weight=wt)
    P = ctx.partials_numpy(part, ctx.n_snap, batch.n_cfg)
    fin = P["n_finite"] > 0
    lz = np.where(fin, P["m"] + np.log(np.where(fin, P["s"], 1.0)), -np.inf)
    nl = batch.n_lig
    share = np.zeros(nl)
    n_scanned = np.zeros(nl, np.int64)
    for l in range(nl):
        a, b = batch.cfg_off[l], batch.cfg_off[l + 1]
        n_scanned[l] = np.count_nonzero(sel[a:b])
        z = lz[:, a:b] + np.log(np.where(wt[a:b] > 0, wt[a:b], 1.0))[None, :]
        z = np.where((wt[a:b] > 0)[None, :], z, -np.inf)
        m = np.max(z, axis=1, keepdims=True)
        ok = np.isfinite(m[:, 0])
        if not np.any(ok):
            continue
        e = np.exp(z[ok] - m[ok])
        share[l] = np.max(e[:, sel[a:b] == 2].sum(axis=1) / e.sum(axis=1))
    return dict(B=B, res=res, n_scanned=n_scanned, fallback=fallback, share=share)


# --------------------------------------------------------------------------
# Measurement: configurations needed for +-0.1 kcal/mol (replicate protocol)
# --------------------------------------------------------------------------

BUDGETS = (0.01, 0.02, 0.03, 0.05, 0.07, 0.1, 0.15, 0.2, 0.3, 0.5)
PLAIN_K = (25, 50, 100, 200, 400, 800, 1600, 3200)


def _err_rms(Zs, Zw, kT):
    """RMS over replicates of kT ln(Z_hat / Z) per snapshot: Zs [S][P]
    (exhaustive, scaled), Zw [R][S] replicate estimates of sum_c Zs."""
    with np.errstate(divide="ignore"):
        e = -kT * (np.log(Zw) - np.log(Zs.sum(axis=1))[None, :])
    e = np.where(np.isfinite(e), e, 1e3)
    return np.sqrt(np.mean(e ** 2, axis=0))


def kstar_plain(Zs, kT, rng, reps: int = 200, tol: float = 0.1):
    """Distinct configurations a uniform with-replacement sample needs for
    RMS <= tol in every snapshot (the exhaustive scan, P, if none does)."""
    P = Zs.shape[1]
    for K in PLAIN_K:
        idx = rng.integers(0, P, (reps, K))
        Zw = Zs[:, idx].mean(axis=2).T * P
        if np.max(_err_rms(Zs, Zw, kT)) <= tol:
            return min(float(P), float(np.mean([np.unique(r).size for r in idx])))
    return float(P)


def kstar_is(sub_batch, Zs, yhat, alpha, tau, kT, seed0, reps: int = 200, tol: float = 0.1,
             exact_share: float = 0.5):
    """Same for the stratified plan (exact_share of the budget the exact top,
    the rest draws) over the budget fractions BUDGETS; returns (distinct
    configurations, budget fraction) or (P, None)."""
    P = Zs.shape[1]
    for bf in BUDGETS:
        top = bf * exact_share
        draw = bf - top
        K = int(np.ceil(draw * P))
        Wr = np.zeros((reps, P))
        ns = np.zeros(reps)
        for r in range(reps):
            u = np.random.Generator(np.random.PCG64(np.random.SeedSequence([170807045, seed0, r]))).random(K + 1)
            sel, wt, n = fd.is_plan(sub_batch, yhat, top, draw, alpha, tau / 5.0, u)
            Wr[r] = wt
            ns[r] = n
        Zw = Wr @ Zs.T
        if np.max(_err_rms(Zs, Zw, kT)) <= tol:
            return float(np.mean(ns)), bf
    return float(P), None


def pool_fraction_scorer(w, batch, P_fine, ligs, alpha: float, plans, kT: float, reps: int = 50, seed0: int = 1000):
    """Function y -> (mean over `ligs` of the fraction of the pool the
    stratified plan needs (kstar_is), best plan of `plans`) for predictions y
    over all configurations of `batch`; a plan is (mixture temperature tau,
    exact share of the budget), a bare tau meaning (tau, 0.5).  Used to choose
    the plan and the training epochs on ligands not fitted."""
    Z = {int(l): ligand_weights(P_fine, batch.cfg_off, l) for l in ligs}
    plans = [tuple(p) if isinstance(p, (tuple, list)) else (float(p), 0.5) for p in plans]

    def score(y):
        best = None
        for tau, share in plans:
            ks = []
            for l in ligs:
                yl = y[batch.cfg_off[l]:batch.cfg_off[l + 1]]
                k, _ = kstar_is(sub_batch(w, l), Z[int(l)], yl, alpha, tau, kT, seed0 + int(l), reps=reps,
                                exact_share=share)
                ks.append(k / Z[int(l)].shape[1])
            m = float(np.mean(ks))
            if best is None or m < best[0]:
                best = (m, (tau, share))
        return best

    return score


def fit_selected(net, X, t, wt, rows, score, epochs: int, check_at=(0, 2, 5, 10, 20, 40, 80), log=None, name=""):
    """Train `net` on `rows` for `epochs` and keep the parameters of the
    checkpoint (epoch in check_at, or the last) that `score` rates best;
    epoch 0 is the starting network (for the residual form, the coarse
    score itself).  Returns dict(score, tau (the plan score chose), epoch,
    params, loss) and leaves the kept parameters set."""
    at = {e for e in check_at if e <= epochs} | {epochs}
    keep = {}

    def checkpoint(ep):
        if ep not in at:
            return
        sc, tau = score(net.forward(X).cpu().numpy())
        if log:
            log(f"{name} epoch {ep}: score {sc:.4f} at plan {tau}")
        if "score" not in keep or sc < keep["score"]:
            keep.update(score=sc, tau=tau, epoch=ep, params=net.get_params())

    hist = train(net, X, t, wt, rows, epochs=epochs, checkpoint=checkpoint)
    net.set_params(keep["params"])
    keep["loss"] = hist[-1] if hist else None
    return keep


def ligand_weights(P_fine, cfg_off, l):
    """Exhaustive Z_{c,s} of ligand l scaled by the per-snapshot maximum
    (host FP64) from fine partials [S][n_cfg]."""
    a, b = cfg_off[l], cfg_off[l + 1]
    p = P_fine[:, a:b]
    fin = p["n_finite"] > 0
    lz = np.where(fin, p["m"] + np.log(np.where(fin, p["s"], 1.0)), -np.inf)
    m = np.max(lz, axis=1, keepdims=True)
    m = np.where(np.isfinite(m), m, 0.0)
    return np.exp(lz - m)


def sub_batch(w, l):
    return fd.Batch([w.ligands[l]])


def split_ligands(n: int, n_train: int, seed: int = 170807045):
    perm = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 11]))).permutation(n)
    return np.sort(perm[:n_train]), np.sort(perm[n_train:])


def rows_of(cfg_off, ligs):
    return np.concatenate([np.arange(cfg_off[l], cfg_off[l + 1]) for l in ligs]).astype(np.int32)


__all__ = ["coarse_desc", "make_context", "inputs", "targets", "train", "predict", "is_estimate", "kstar_plain",
           "make_network", "predicted_remainder", "targets_snapmax", "coarse_score", "pool_fraction_scorer", "fit_selected",
           "kstar_is", "ligand_weights", "sub_batch", "split_ligands", "rows_of", "BUDGETS", "PLAIN_K",
           "N_IN_FULL", "init_params"]
