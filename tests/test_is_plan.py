"""The stratified importance-sampling plan: the oracle's form pinned by the
mathematics it must satisfy (reduction to the plain and to the
unstratified estimator, exact unbiasedness over the uniforms), and the
library's host implementation (fftdg_is_plan, no GPU needed) against it."""
import math

import numpy as np
import pytest

from oracle import estimators as est
from workload import synth

T = 300.0


def _ligand_logz(P, seed):
    rng = np.random.default_rng(seed)
    lz = rng.normal(0.0, 3.0, P)
    lz[rng.random(P) < 0.1] = -np.inf      # configurations with nothing finite
    return lz


def test_top_fraction_one_is_the_plain_estimate():
    P = 37
    lz = _ligand_logz(P, 1)
    y = np.random.default_rng(2).normal(size=P)
    sel, wt = est.stratified_plan(y, np.array([0, P]), 1.0, 0.3, 0.1, 1.0, synth.uniforms(3, 100))
    assert sel.all() and np.all(wt == 1.0)
    n = 1234.0
    parts = np.c_[lz, np.ones(P), np.full(P, n / P), np.isfinite(lz).astype(float), np.zeros(P), np.zeros(P)]
    parts[~np.isfinite(lz), 0] = 0.0
    assert est.bpmf_weighted(lz, n, wt, T) == pytest.approx(est.bpmf(parts, T), abs=1e-12)


def test_top_fraction_zero_is_the_unstratified_estimate():
    P, K = 50, 20
    lz = _ligand_logz(P, 4)
    y = np.random.default_rng(5).normal(size=P) * 2
    u = synth.uniforms(6, K)
    sel, wt = est.stratified_plan(y, np.array([0, P]), 0.0, K / P, 0.2, 0.7, u)
    q = est.proposal(y, 0.2, 0.7)
    idx = est.inverse_cdf_sample(q, u)
    assert set(np.flatnonzero(sel)) == set(idx.tolist())
    assert est.bpmf_weighted(lz, 999.0, wt, T) == pytest.approx(est.bpmf_is(lz, 999.0, idx, q, T), abs=1e-10)


@pytest.mark.parametrize("K,M", [(1, 40000), (2, 200)])
def test_stratified_estimate_is_unbiased_over_the_uniforms(K, M):
    """E_u[Z_hat] = Z: the midpoint rule over a grid of the K uniforms
    integrates the piecewise-constant estimate; the error is bounded by the
    cells that straddle a CDF boundary."""
    P = 6
    lz = np.array([0.3, -1.0, 2.0, -0.5, 1.1, -2.2])
    Z = np.exp(lz)
    y = np.array([0.1, 0.9, 1.5, -0.3, 0.0, 0.4])   # imperfect prediction
    off = np.array([0, P])
    grid = (np.arange(M) + 0.5) / M
    acc = 0.0
    if K == 1:
        for u in grid:
            _, wt = est.stratified_plan(y, off, 2 / P, K / P, 0.25, 0.8, np.array([u]))
            acc += np.sum(wt * Z)
        mean = acc / M
    else:
        for u1 in grid:
            for u2 in grid:
                _, wt = est.stratified_plan(y, off, 2 / P, K / P, 0.25, 0.8, np.array([u1, u2]))
                acc += np.sum(wt * Z)
        mean = acc / M ** 2
    assert mean == pytest.approx(Z.sum(), rel=(4 * K + 2) / M * 10)


def test_stratified_estimate_unbiased_monte_carlo():
    P = 120
    lz = _ligand_logz(P, 7)
    Z = np.where(np.isfinite(lz), np.exp(lz), 0.0)
    y = np.where(np.isfinite(lz), lz, -10) + np.random.default_rng(8).normal(0, 1.5, P)
    off = np.array([0, P])
    vals = []
    for r in range(1500):
        _, wt = est.stratified_plan(y, off, 0.05, 0.1, 0.1, 1.0, synth.uniforms(1000 + r, 12))
        vals.append(np.sum(wt * Z))
    vals = np.array(vals)
    z = (vals.mean() - Z.sum()) / (vals.std(ddof=1) / math.sqrt(vals.size))
    assert abs(z) < 4.0, z


def _batch_of(sizes, seed=9):
    import paper_1708_07045_amd as fd
    rng = np.random.default_rng(seed)
    ligs = []
    for P in sizes:
        L = synth.make_ligand(rng, rng, 5, 1, P)
        ligs.append(L)
    return fd.Batch(ligs)


@pytest.mark.parametrize("top,draw,alpha,tau", [(0.05, 0.1, 0.1, 1.0), (0.0, 0.3, 0.0, 0.5), (1.0, 0.2, 0.1, 1.0),
                                                (0.3, 0.0, 0.1, 1.0), (0.1, 0.5, 1.0, 2.0)])
def test_library_plan_matches_oracle(top, draw, alpha, tau):
    import paper_1708_07045_amd as fd
    b = _batch_of([1, 17, 300, 64, 2])
    rng = np.random.default_rng(10)
    y = (rng.normal(size=b.n_cfg) * 3).astype(np.float32)
    y[5:9] = y[4]                                  # ties go to the lower index
    u = synth.uniforms(11, 1000)
    sel, wt, n = fd.is_plan(b, y, top, draw, alpha, tau, u)
    sel_o, wt_o = est.stratified_plan(y.astype(np.float64), b.cfg_off, top, draw, alpha, tau, u)
    np.testing.assert_array_equal(sel, sel_o)
    np.testing.assert_allclose(wt, wt_o, rtol=1e-12, atol=0)
    assert n == int(np.count_nonzero(sel))
    assert set(np.unique(sel)) <= {0, 1, 2}


def test_library_plan_rejects_bad_arguments():
    import paper_1708_07045_amd as fd
    b = _batch_of([10, 10])
    y = np.zeros(b.n_cfg, np.float32)
    u = synth.uniforms(12, 100)
    for kw in [dict(top_frac=1.5), dict(draw_frac=-0.1), dict(alpha=2.0), dict(tau=0.0)]:
        args = dict(top_frac=0.1, draw_frac=0.1, alpha=0.1, tau=1.0)
        args.update(kw)
        with pytest.raises(fd.FFTDGError):
            fd.is_plan(b, y, uniforms=u, **args)
    with pytest.raises(fd.FFTDGError):
        fd.is_plan(b, y, 0.1, 0.5, 0.1, 1.0, u[:3])           # too few uniforms
    bad = y.copy()
    bad[3] = np.nan
    with pytest.raises(fd.FFTDGError):
        fd.is_plan(b, bad, 0.1, 0.1, 0.1, 1.0, u)
    with pytest.raises(fd.FFTDGError):
        fd.is_plan(b, y, 0.1, 0.1, 0.1, 1.0, np.full(100, 1.0))  # uniforms must be < 1


def test_scan_features_follow_eq2_and_eq13():
    """Column 0 is ln sum_s W_s Z_{c,s} relative to the ligand's maximum:
    recovered independently from the per-configuration BPMFs (Eq. 2) and
    their combination over snapshots (Eq. 13)."""
    rng = np.random.default_rng(13)
    S, C = 3, 9
    parts = np.zeros((S, C, 6))
    parts[:, :, 0] = rng.normal(0, 4, (S, C))
    parts[:, :, 1] = rng.uniform(1, 50, (S, C))
    parts[:, :, 2] = 500
    parts[:, :, 3] = rng.integers(1, 500, (S, C))
    parts[:, :, 4] = rng.normal(-5, 2, (S, C))
    parts[:, 2, 3] = 0                       # config 2: nothing finite anywhere
    parts[:, 2, 4] = np.inf
    parts[1, 5, 3] = 0                       # config 5: nothing finite in snapshot 1
    W = np.array([0.5, 0.3, 0.2])
    off = np.array([0, 4, 9])
    f = est.scan_features(parts, W, off)
    kTv = est.kT(T)
    x = np.full(C, -np.inf)
    for c in range(C):
        B = np.array([est.bpmf(parts[s, c:c + 1], T) for s in range(S)])
        if np.all(~np.isfinite(B)):
            continue
        vs = 1.0  # any V_site: it cancels
        dg = est.dg_standard(B, W, vs, T)
        x[c] = math.log(500) - (dg + kTv * math.log(vs * est.C_STANDARD)) / kTv
    for a, b in zip(off[:-1], off[1:]):
        X = np.max(x[a:b])
        for c in range(a, b):
            want = max(x[c] - X, -25) / 5 if np.isfinite(x[c]) else -5.0
            assert f[c, 0] == pytest.approx(want, abs=1e-12)
    assert f[2, 1] == 5.0 and f[2, 2] == 0.0
    assert f[5, 2] == pytest.approx(parts[:, 5, 3].sum() / 1500)
    for a, b in zip(off[:-1], off[1:]):
        assert min(f[a:b, 1]) == 0.0


class _B:
    """Stand-in for a batch: only the ligand offsets are read."""

    def __init__(self, cfg_off):
        self.cfg_off = np.asarray(cfg_off, np.int32)
        self.n_lig = self.cfg_off.size - 1


def test_predicted_remainder_closed_forms():
    """Share of sum_c exp(5 y_c) outside the ceil(top_frac P) largest."""
    from paper_1708_07045_amd import proposal as prop
    y = np.array([0.0, -np.log(3.0) / 5, -np.log(6.0) / 5, 0.0, 0.0])   # weights 1, 1/3, 1/6 | 1, 1
    r = prop.predicted_remainder(_B([0, 3, 5]), y, 0.34)          # ligand 0 keeps 2, ligand 1 keeps 1
    assert r[0] == pytest.approx((1 / 6) / (1 + 1 / 3 + 1 / 6), rel=1e-12)
    assert r[1] == pytest.approx(0.5, rel=1e-12)
    assert np.all(prop.predicted_remainder(_B([0, 3, 5]), y, 1.0) == 0.0)
    assert np.all(prop.predicted_remainder(_B([0, 3, 5]), y, 0.0) == 1.0)
    # order and shift invariance within a ligand
    r2 = prop.predicted_remainder(_B([0, 3, 5]), np.r_[y[[2, 0, 1]] + 7.0, y[3:]], 0.34)
    np.testing.assert_allclose(r2, r, rtol=1e-12)


def test_snapshot_max_targets_closed_forms():
    """t_c = max_s (ln Z_{c,s} - max_{c'} ln Z_{c',s}) floored at -25, / 5;
    a configuration that dominates a small snapshot still scores 0."""
    from paper_1708_07045_amd import proposal as prop
    pd = np.dtype([("m", "<f8"), ("s", "<f8"), ("n_finite", "<i8")])
    P = np.zeros((2, 4), pd)
    # ligand 0: configurations 0..2; ligand 1: configuration 3 (nothing finite)
    lz = np.array([[10.0, 4.0, 9.0, 0.0], [-50.0, -40.0, -80.0, 0.0]])
    P["m"] = lz - 1.0
    P["s"] = np.e
    P["n_finite"] = 1
    P["n_finite"][:, 3] = 0
    t, w = prop.targets_snapmax(P, [0, 3, 4])
    t = t.numpy()
    np.testing.assert_allclose(t[:3], [0.0, 0.0, -1.0 / 5.0], atol=1e-6)
    # snapshot 0 alone: configuration 1 sits 6 nats down; snapshot 1 makes it the top
    assert t[3] == -5.0
    np.testing.assert_array_equal(w.numpy(), [10.0, 10.0, 10.0, 1.0])
    P["m"][0, 2] = -100.0            # now 110 nats below in snapshot 0 and 40 below in 1: floored
    t, _ = prop.targets_snapmax(P, [0, 3, 4])
    assert t.numpy()[2] == pytest.approx(-25.0 / 5.0)
