"""The batched workload (141 ligands of 8-40 atoms, 10 jittered receptor
snapshots, 128^3 FFT; configurations at a tenth of 200-2000 per ligand)
scanned whole on the GPU in one pass on the fused path (chunks of 256: the
clash test on bits, energy channels through the FFT), and
checked against the FP64 oracle on a stratified subset of snapshot 0:
  - 6 ligands (fewest atoms, most atoms, 4 seeded picks) x all their
    configurations: partials of Eq. 2 per configuration (counts bit-exact),
    B per ligand within 0.01 kcal/mol;
  - 10^4 (configuration, translation) spot checks of the raw energy of
    Eq. 8 over 100 seeded configurations of all ligands: max |dPsi| <=
    1e-5 * max |Psi| of that configuration, and the clash flag bit-exact."""
import numpy as np
import pytest

import oracle
from oracle import estimators as est
from workload import synth

pytestmark = pytest.mark.gpu


def _ligand_pick(w, rng):
    na = np.array([L.n_atoms for L in w.ligands])
    first, last = int(np.argmin(na)), int(np.argmax(na))
    rest = [i for i in range(len(w.ligands)) if i not in (first, last)]
    return [first, last] + sorted(int(i) for i in rng.choice(rest, 4, replace=False))


def test_batched_workload_stratified_subset():
    import torch
    import paper_1708_07045_amd as fd
    w = synth.config3(cfg_scale=0.1)
    rng = np.random.default_rng(20171)
    ctx = fd.FFTDG.from_workload(w)
    ctx.set_tuning(configs_per_chunk=256, fused=1)
    gs, os_ = [], []
    for s in range(w.receptor.n_snap):
        g, o = ctx.receptor_grids(w.receptor.xyz[s], w.receptor.q, w.receptor.sigma, w.receptor.eps)
        gs.append(g)
        os_.append(o)
    grids, occ = torch.stack(gs), torch.stack(os_)
    ctx.set_receptors(grids, occ, w.receptor.weights)
    b = fd.Batch(w.ligands)
    print(f"batched subset: {len(w.ligands)} ligands, {b.n_cfg} configurations, {w.receptor.n_snap} snapshots",
          flush=True)
    buf = ctx.scan(b, w.T)
    torch.cuda.synchronize()
    P = ctx.partials_numpy(buf, ctx.n_snap, b.n_cfg)
    B, res = ctx.reduce(b, buf, w.T)
    go, oo = oracle.receptor_grids(w, 0)
    kt = est.kT(w.T)
    for l in _ligand_pick(w, rng):
        c0, c1 = b.cfg_off[l], b.cfg_off[l + 1]
        parts, _ = oracle.scan(w, go, oo, lig_idx=l)
        g = P[0, c0:c1]
        np.testing.assert_array_equal(g["n_valid"], parts[:, 2].astype(np.int64))
        np.testing.assert_array_equal(g["n_finite"], parts[:, 3].astype(np.int64))
        fin = parts[:, 3] > 0
        lz_g = np.where(fin, g["m"] + np.log(np.where(fin, g["s"], 1.0)), -np.inf)
        assert np.max(np.abs(kt * (lz_g[fin] - est.log_z(parts)[fin])), initial=0.0) < 0.01
        Bo = est.bpmf(parts, w.T)
        assert abs(B[l, 0] - Bo) < 0.01, (l, B[l, 0], Bo)
        print(f"ligand {l}: {w.ligands[l].n_atoms} atoms, {c1 - c0} configurations, "
              f"B {B[l, 0]:.6f} vs oracle {Bo:.6f}", flush=True)
    # spot checks of raw energies and clash flags
    cfgs = rng.choice(b.n_cfg, 100, replace=False)
    n_checked = 0
    for cg in cfgs:
        l = int(np.searchsorted(b.cfg_off, cg, side="right") - 1)
        L = w.ligands[l]
        psi, cl = ctx.energy_grid(0, b, int(cg), w.T)
        psi, cl = psi.cpu().numpy(), cl.cpu().numpy()
        u, box = oracle.place_cfg(w, l, int(cg - b.cfg_off[l]))
        if psi.size == 0:
            assert any(w.n_rec - x <= 0 for x in box)
            continue
        flat = rng.choice(psi.size, 100, replace=psi.size < 100)
        want = oracle.direct_energy(w, go, u, oracle.ligand_weights(L), box).ravel()
        wcl = oracle.clash(w, oo, u, oracle.occ_thresholds(L, w.occ_f, w.h), box).ravel()
        scale = np.max(np.abs(want))
        assert np.max(np.abs(psi.ravel()[flat] - want[flat])) <= 1e-5 * scale
        np.testing.assert_array_equal(cl.ravel()[flat], wcl[flat])
        n_checked += flat.size
    assert n_checked >= 9000
