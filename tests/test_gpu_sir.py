"""Pose resampling (sampling importance resampling) through the C-ABI
against the oracle's draws from the same uniforms.  The two sides compute
the Boltzmann weights in different precisions (FP32 energies on the GPU,
FP64 in the oracle), so a draw may differ only where its uniform lies
within rounding of a boundary of the oracle's running sums; every other
draw must be identical, and the drawn pose's energy must match."""
import math

import numpy as np
import pytest

import oracle
from oracle import estimators as est
from workload import synth

pytestmark = pytest.mark.gpu


def _near_boundary(cdf, x, rel):
    return np.min(np.abs(cdf - x)) <= rel * cdf[-1]


def _compare(w, precision, K=300, seed=61, select=None):
    import paper_1708_07045_amd as fd
    from paper_1708_07045_amd import proposal as prop
    print(f"pose resampling: {w.name[:3]} {precision} K={K}", flush=True)
    ctx = fd.FFTDG.from_workload(w, precision=precision)
    g, o = ctx.receptor_grids(w.receptor.xyz[0], w.receptor.q, w.receptor.sigma, w.receptor.eps)
    ctx.set_receptors(g[None].contiguous(), o[None].contiguous() if o is not None else None, w.receptor.weights)
    b = fd.Batch(w.ligands, select)
    part = ctx.scan(b, w.T)
    u = synth.uniforms(seed, 2 * K)
    cfg, t, psi = ctx.sample_poses(b, part, 0, 0, w.T, u)
    go, oo = oracle.receptor_grids(w)
    parts, _ = oracle.scan(w, go, oo)
    if select is not None:
        parts[np.asarray(select) == 0, 3] = 0      # unscanned: never drawn
    cache = {}

    def energies(c):
        if c not in cache:
            r = oracle.config_eval(w, go, oo, 0, c)
            cache[c] = (r["psi"], r["clash"])
        return cache[c]
    cfg_o, t_o, psi_o = est.sample_poses(parts, energies, w.T, u)
    fin = parts[:, 3] > 0
    z = np.where(fin, np.exp(np.where(fin, parts[:, 0], 0) - np.max(parts[fin, 0])) * parts[:, 1], 0.0)
    cdf_c = np.cumsum(z)
    tol = 1e-4 if precision == "f32" else 1e-9
    same_c = cfg == cfg_o
    for k in np.flatnonzero(~same_c):
        assert _near_boundary(cdf_c, u[2 * k] * cdf_c[-1], tol), k
    assert same_c.mean() >= 0.97
    same_t = same_c & np.all(t == t_o, axis=1)
    for k in np.flatnonzero(same_c & ~same_t):
        ps, cl = energies(int(cfg[k]))
        f = ps.ravel()
        ok = np.ones(f.size, bool) if cl is None else ~np.asarray(cl, bool).ravel()
        cw = np.cumsum(np.where(ok, np.exp(-(f - f[ok].min()) / est.kT(w.T)), 0.0))
        assert _near_boundary(cw, u[2 * k + 1] * cw[-1], tol), k
    assert same_t.mean() >= 0.95
    # every drawn pose is a clash-free valid translation of a drawn
    # configuration, and its energy matches the oracle's there
    for k in range(K):
        ps, cl = energies(int(cfg[k]))
        tx, ty, tz = t[k]
        assert 0 <= tz < ps.shape[0] and 0 <= ty < ps.shape[1] and 0 <= tx < ps.shape[2]
        assert cl is None or not cl[tz, ty, tx]
        scale = np.max(np.abs(ps))
        assert abs(psi[k] - ps[tz, ty, tx]) <= (1e-5 if precision == "f32" else 1e-10) * scale
    if select is not None:
        assert np.all(np.asarray(select)[cfg] != 0)
    return cfg, t


def test_pose_resampling_c2_fp32():
    w = synth.subset(synth.config2(), 40, stride=197)
    _compare(w, "f32")


def test_pose_resampling_selected_subset():
    w = synth.subset(synth.config2(), 30, stride=251)
    sel = np.zeros(30, np.uint8)
    sel[::2] = 1
    _compare(w, "f32", K=120, seed=62, select=sel)


def test_pose_resampling_c1_fp64_cap():
    w = synth.subset(synth.config1(), 25)
    _compare(w, "f64", K=200, seed=63)


def test_pose_resampling_all_clash_is_an_error():
    import paper_1708_07045_amd as fd
    w = synth.config2(n_rot=3, n_conf=1)
    ctx = fd.FFTDG.from_workload(w)
    g, o = ctx.receptor_grids(w.receptor.xyz[0], w.receptor.q, w.receptor.sigma, w.receptor.eps)
    o.fill_(1)
    ctx.set_receptors(g[None].contiguous(), o[None].contiguous())
    b = fd.Batch(w.ligands)
    part = ctx.scan(b, w.T)
    with pytest.raises(fd.FFTDGError) as e:
        ctx.sample_poses(b, part, 0, 0, w.T, synth.uniforms(1, 10))
    assert e.value.code == -2
