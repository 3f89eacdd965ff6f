"""Precision study at full size: the 8000-configuration T4L-sized workload
scanned in FP32 on the GPU (FP32 transforms, products, energies and
max-shifted log-sum-exp; FP64 accumulation over configurations and the dG
logarithm) against the FP64 oracle's results stored by
tests/golden/make_c2_oracle.py, in occupancy mode and in capped-repulsion
mode, with the cavity atom parameters and (stress) with the tiny case's
larger charges and well depths, whose energies span a wider range.  Errors
are printed per result."""
import json
import math
import os

import numpy as np
import pytest

from workload import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# Capped-repulsion mode with the stress parameters: the clamped repulsion of
# overlapping poses reaches ~10^5 kcal/mol, and FP32 transform round-off is
# normwise (about 1e-7 of the field's norm per pass), so the error on the
# low-energy translations that carry the Boltzmann weight scales with those
# values: measured 0.015 kcal/mol on B = -225 kcal/mol (7e-5 relative).
# That case is held to 0.05 kcal/mol; occupancy mode (the paper's) meets
# 0.01 with both parameter sets.
TOL = {("occ", "cavity"): 0.01, ("cap", "cavity"): 0.01, ("occ", "stress"): 0.01, ("cap", "stress"): 0.05}


@pytest.mark.parametrize("params", ["cavity", "stress"])
@pytest.mark.parametrize("mode", ["occ", "cap"])
@pytest.mark.parametrize("fused,energy_xy_direct", [(1, 0), (2, 0), (0, 0), (0, 2)])
def test_full_c2_fp32_against_fp64_oracle(params, mode, fused, energy_xy_direct):
    tol = TOL[(mode, params)]
    import torch
    import paper_1708_07045_amd as fd
    gold = "c2_oracle.json" if params == "cavity" else "c2_stress_oracle.json"
    ref = json.load(open(os.path.join(GOLDEN, gold)))[mode]
    print(f"precision study: c2 {params} {mode} fused={fused} energy_xy_direct={energy_xy_direct}", flush=True)
    w = synth.config2(params=synth.CAVITY_PARAMS if params == "cavity" else synth.TINY_PARAMS)
    w.clash_mode = mode
    ctx = fd.FFTDG.from_workload(w)
    ctx.set_tuning(energy_xy_direct=energy_xy_direct, configs_per_chunk=512, fused=fused)
    g, o = ctx.receptor_grids(w.receptor.xyz[0], w.receptor.q, w.receptor.sigma, w.receptor.eps)
    ctx.set_receptors(g[None].contiguous(), o[None].contiguous() if o is not None else None, w.receptor.weights)
    b = fd.Batch(w.ligands)
    part = ctx.scan(b, w.T)
    B, res = ctx.reduce(b, part, w.T)
    P = ctx.partials_numpy(part, 1, b.n_cfg)[0]
    dB = abs(B[0, 0] - ref["B"])
    ddg = abs(res["dG"][0] - ref["dG"])
    fin = P["n_finite"] > 0
    lz = np.where(fin, P["m"] + np.log(np.where(fin, P["s"], 1.0)), -np.inf)[::100]
    lz_ref = np.array([-np.inf if v is None else v for v in ref["log_z_every_100th"]])
    kT = 1.987204259e-3 * w.T
    ok = np.isfinite(lz_ref)
    np.testing.assert_array_equal(np.isfinite(lz), ok)
    dcfg = np.max(np.abs(kT * (lz[ok] - lz_ref[ok])))
    print(f"  |dB| = {dB:.3g}  |d dG| = {ddg:.3g}  max per-configuration |kT d lnZ| = {dcfg:.3g} kcal/mol", flush=True)
    assert int(P["n_valid"].sum()) == ref["n_samples"]
    assert int(P["n_finite"].sum()) == ref["n_finite"]
    assert abs(res["v_site"][0] - ref["v_site"]) <= 1e-9 * ref["v_site"]
    assert dB < tol and ddg < tol and dcfg < tol
