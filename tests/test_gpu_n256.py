"""The 256-point FFT path (row and column passes over planes in device
memory) against the FP64 oracle: raw energies and clash masks, and scan
partials and BPMFs, on a 25 A receptor box zero-padded into a 256^3 FFT
(the whole-surface grid of the paper is 62 A at 0.25 A, 248 points)."""
import numpy as np
import pytest

import oracle
from oracle import estimators as est
from workload import synth

pytestmark = pytest.mark.gpu

TOL_F32 = 1e-5


def _w(n_rot=3, n_conf=2):
    w = synth.config2(n_rot=n_rot, n_conf=n_conf)
    w.n_rec, w.n_fft = 100, 256
    w.origin = -0.5 * (100 - 1) * w.h * np.ones(3)
    return w


def _ctx(w, **tuning):
    import torch
    import paper_1708_07045_amd as fd
    ctx = fd.FFTDG.from_workload(w)
    if tuning:
        ctx.set_tuning(**tuning)
    g, o = ctx.receptor_grids(w.receptor.xyz[0], w.receptor.q, w.receptor.sigma, w.receptor.eps)
    ctx.set_receptors(g[None].contiguous(), o[None].contiguous(), w.receptor.weights)
    torch.cuda.synchronize()
    return ctx


@pytest.mark.parametrize("edirect", [0, 2])
def test_energy_n256(edirect):
    import paper_1708_07045_amd as fd
    w = _w()
    ctx = _ctx(w, energy_xy_direct=edirect)
    b = fd.Batch(w.ligands)
    go, oo = oracle.receptor_grids(w)
    for c in (0, 3, 5):
        print(f"n256 energy edirect={edirect} cfg {c}", flush=True)
        psi, clash = ctx.energy_grid(0, b, c, w.T)
        r = oracle.config_eval(w, go, oo, 0, c)
        assert psi.shape == r["psi"].shape
        a, ref = psi.cpu().numpy().astype(np.float64), r["psi"]
        assert np.linalg.norm(a - ref) <= TOL_F32 * np.linalg.norm(ref)
        assert np.max(np.abs(a - ref)) <= TOL_F32 * np.max(np.abs(ref))
        np.testing.assert_array_equal(clash.cpu().numpy(), r["clash"])


@pytest.mark.parametrize("edirect,chunk", [(2, 256), (0, 256), (2, 5)])
def test_scan_n256(edirect, chunk):
    import paper_1708_07045_amd as fd
    w = _w(n_rot=6, n_conf=2)
    ctx = _ctx(w, energy_xy_direct=edirect, configs_per_chunk=chunk)
    b = fd.Batch(w.ligands)
    print(f"n256 scan edirect={edirect} chunk={chunk} n_cfg={b.n_cfg}", flush=True)
    part = ctx.scan(b, w.T)
    P = ctx.partials_numpy(part, 1, b.n_cfg)[0]
    B, res = ctx.reduce(b, part, w.T)
    go, oo = oracle.receptor_grids(w)
    parts, boxes = oracle.scan(w, go, oo)
    np.testing.assert_array_equal(P["n_valid"], parts[:, 2].astype(np.int64))
    np.testing.assert_array_equal(P["n_finite"], parts[:, 3].astype(np.int64))
    Bo = est.bpmf(parts, w.T)
    assert abs(B[0, 0] - Bo) < 0.01, (B[0, 0], Bo)


def test_n256_rejects_energy_mode_1():
    import paper_1708_07045_amd as fd
    w = _w()
    ctx = fd.FFTDG.from_workload(w)
    with pytest.raises(fd.FFTDGError):
        ctx.set_tuning(energy_xy_direct=1)
