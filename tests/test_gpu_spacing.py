"""Grid tools without an FFT context, through the C-ABI, against the FP64
oracle: grids of any edge, trilinear pose energies, direct pair energies;
and the spacing study's trend (finer grids, smaller error)."""
import numpy as np
import pytest

import oracle
from oracle import pairs
from workload import synth

pytestmark = pytest.mark.gpu


def _tiny():
    return synth.tiny(seed=4, n_rec=37, h=0.3, n_rec_atoms=120, n_lig_atoms=9, n_cfg=2, clash_mode="occ",
                      precision="f64")


def test_grids_build_any_edge_matches_oracle():
    import paper_1708_07045_amd as fd
    print("grid tools: build 37^3 f64 occ", flush=True)
    w = _tiny()
    r = w.receptor
    tools = fd.GridTools(w.n_rec, w.h, w.origin, "f64", "occ", w.ljr_cap, w.occ_f)
    g, o = tools.build(r.xyz[0], r.q, r.sigma, r.eps)
    go, oo = oracle.receptor_grids(w)
    gg = g.cpu().numpy()
    for ch in range(3):
        np.testing.assert_allclose(gg[ch], go[ch], rtol=1e-12, atol=1e-12)
    np.testing.assert_array_equal(o.cpu().numpy(), oo)


def test_pose_energies_match_oracle():
    import paper_1708_07045_amd as fd
    print("grid tools: pose energies", flush=True)
    w = _tiny()
    r = w.receptor
    L = w.ligands[0]
    rng = np.random.default_rng(5)
    centre = w.origin + 0.5 * (w.n_rec - 1) * w.h
    base = L.conformers[0] - L.conformers[0].mean(axis=0)
    poses = np.stack([base + centre + rng.uniform(-3, 3, 3) for _ in range(17)])
    tools = fd.GridTools(w.n_rec, w.h, w.origin, "f64", "occ", w.ljr_cap, w.occ_f)
    g, _ = tools.build(r.xyz[0], r.q, r.sigma, r.eps)
    eg = tools.grid_energies(g, poses, L.q, L.sigma, L.eps)
    go, _ = oracle.receptor_grids(w)
    ego = pairs.grid_energies(go, w.h, w.origin, poses, L.q, L.sigma, L.eps)
    np.testing.assert_allclose(eg, ego, rtol=1e-10, atol=1e-10)
    for excl in (True, False):
        ed = tools.pair_energies(r.xyz[0], r.q, r.sigma, r.eps, poses, L.q, L.sigma, L.eps, exclusion=excl)
        edo = pairs.pair_energies(r.xyz[0], r.q, r.sigma, r.eps, poses, L.q, L.sigma, L.eps, exclusion=excl)
        np.testing.assert_allclose(ed, edo, rtol=1e-12, atol=1e-12)


def test_spacing_study_trend():
    import paper_1708_07045_amd as fd
    from paper_1708_07045_amd import spacing
    print("spacing study: c2 subset, 60 poses", flush=True)
    w = synth.subset(synth.config2(), 40, stride=199)
    ctx = fd.FFTDG.from_workload(w)
    g, o = ctx.receptor_grids(w.receptor.xyz[0], w.receptor.q, w.receptor.sigma, w.receptor.eps)
    ctx.set_receptors(g[None].contiguous(), o[None].contiguous(), w.receptor.weights)
    b = fd.Batch(w.ligands)
    part = ctx.scan(b, w.T)
    res = spacing.study(w, ctx, b, part, n_poses=60, spacings=(0.125, 0.25, 0.5, 0.8))
    rows = res["by_spacing"]
    print(rows, flush=True)
    # finer grids, smaller error: RMSE rises and R falls with the spacing
    rm = [r["rmse_kcal_mol"] for r in rows]
    pr = [r["pearson_r"] for r in rows]
    assert all(a < b for a, b in zip(rm, rm[1:])), rm
    assert all(a > b for a, b in zip(pr, pr[1:])), pr
    assert pr[0] > 0.9
    # the scan's energies at the resampled poses are the 0.25 A grid
    # energies of the same poses (the FFT computes the trilinear sum)
    assert rows[1]["n_rec"] == 96
