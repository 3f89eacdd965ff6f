"""fftdg_reduce_static (the reduce with the library's static device scratch,
for callers that cannot allocate) against fftdg_reduce on the same partials:
bit-identical B and per-ligand results on two calls in a row, the second
with a smaller batch and importance weights; a batch beyond the scratch
limit is refused on the host before anything runs."""
import ctypes

import numpy as np
import pytest

from workload import synth

pytestmark = pytest.mark.gpu


def _context(w):
    import torch
    import paper_1708_07045_amd as fd
    ctx = fd.FFTDG.from_workload(w)
    gs, os_ = [], []
    for s in range(w.receptor.n_snap):
        g, o = ctx.receptor_grids(w.receptor.xyz[s], w.receptor.q, w.receptor.sigma, w.receptor.eps)
        gs.append(g)
        os_.append(o)
    grids = torch.stack(gs).contiguous()
    occ = torch.stack(os_).contiguous() if w.clash_mode == "occ" else None
    ctx.set_receptors(grids, occ, w.receptor.weights)
    torch.cuda.synchronize()
    return ctx, grids, occ


def _same(a, b):
    Ba, ra = a
    Bb, rb = b
    np.testing.assert_array_equal(Ba, Bb)
    for f in ra.dtype.names:
        np.testing.assert_array_equal(ra[f], rb[f])


def test_reduce_static_matches_reduce_on_two_calls():
    import torch
    import paper_1708_07045_amd as fd
    w = synth.config3(n_ligands=5, n_snap=3, cfg_scale=0.02)
    print("no-alloc reduce: 5 ligands x 3 snapshots, then 2 ligands with weights", flush=True)
    ctx, grids, occ = _context(w)
    b1 = fd.Batch(w.ligands)
    p1 = ctx.scan(b1, w.T)
    ref1 = ctx.reduce(b1, p1, w.T)
    got1 = ctx.reduce_static(b1, p1, w.T)
    assert np.all(np.isfinite(ref1[0]))
    _same(got1, ref1)
    # second call: fewer ligands, importance weights (some zero), static first
    b2 = fd.Batch(w.ligands[:2])
    p2 = ctx.scan(b2, w.T)
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([170807045, 77])))
    wt = rng.uniform(0.0, 3.0, b2.n_cfg)
    wt[::4] = 0.0
    wt_dev = torch.as_tensor(wt, dtype=torch.float64, device=ctx.device)
    got2 = ctx.reduce_static(b2, p2, w.T, cfg_weight=wt_dev)
    ref2 = ctx.reduce(b2, p2, w.T, cfg_weight=wt_dev)
    _same(got2, ref2)
    assert not np.array_equal(got2[0], got1[0][:2])  # the weights changed the result
    # a batch beyond the static scratch: refused before any launch, context usable after
    n_big = 100000
    off = np.zeros(n_big + 1, np.int32)
    big = fd._lib.BatchC()
    big.n_lig = n_big
    big.cfg_off = off.ctypes.data
    B = np.zeros((n_big, ctx.n_snap))
    res = np.zeros(n_big, fd._lib.RESULT_DTYPE)
    rc = ctx.L.fftdg_reduce_static(ctx.h_ctx, ctypes.byref(big), p1.data_ptr(), None, float(w.T),
                                   B.ctypes.data, res.ctypes.data)
    assert rc == fd._lib.E_INVALID
    assert "static scratch" in ctx.L.fftdg_last_error(ctx.h_ctx).decode()
    _same(ctx.reduce_static(b1, p1, w.T), ref1)
