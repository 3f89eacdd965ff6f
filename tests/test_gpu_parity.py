"""Parity of the HIP path (through the C-ABI) with the FP64 oracle.

Tolerances (the FP32 bound: a radix-2 FFT of length N adds about
u sqrt(log2 N) relative error per transform, u = 2^-24, so three 128-point
passes each way stay near 1e-6 normwise, with a margin of 10 for the
spectral product and the sum over channels):
  FP64 path: raw energies normwise <= 1e-10, B and dG <= 1e-8 kcal/mol.
  FP32 path: raw energies ||dPsi||_2 / ||Psi||_2 <= 1e-5 and
             max|dPsi| <= 1e-5 * max|Psi| over the box-valid translations;
             clash masks and box extents bit-exact;
             B and dG within 0.01 kcal/mol.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import estimators as est
from workload import synth

pytestmark = pytest.mark.gpu

TOL_F32 = 1e-5
TOL_F64 = 1e-10


def _ctx(w, precision=None):
    import paper_1708_07045_amd as fd
    return fd.FFTDG.from_workload(w, precision=precision)


def _gpu_setup(w, precision=None, snaps=None, **tuning):
    """Context with GPU-built receptor grids for all (or the chosen) snapshots.
    A schedule knob of the plane path (energy_xy_direct, snapshots_per_pass)
    selects that path unless `fused` is given."""
    import torch
    ctx = _ctx(w, precision)
    if ("energy_xy_direct" in tuning or "snapshots_per_pass" in tuning) and "fused" not in tuning:
        tuning["fused"] = 0
    if tuning:
        ctx.set_tuning(**tuning)
    snaps = range(w.receptor.n_snap) if snaps is None else snaps
    gs, os_ = [], []
    for s in snaps:
        g, o = ctx.receptor_grids(w.receptor.xyz[s], w.receptor.q, w.receptor.sigma, w.receptor.eps)
        gs.append(g)
        os_.append(o)
    grids = torch.stack(gs)
    occ = torch.stack(os_) if w.clash_mode == "occ" else None
    ctx.set_receptors(grids, occ, w.receptor.weights[list(snaps)])
    torch.cuda.synchronize()
    return ctx, grids, occ


def _batch(w, select=None):
    import paper_1708_07045_amd as fd
    return fd.Batch(w.ligands, select)


def _norm_err(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300), np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def _announce(msg):
    print(msg, flush=True)


# ------------------------------------------------------------------ grids
@pytest.mark.parametrize("cfgname", ["c1", "c2"])
def test_receptor_grids_match_oracle(cfgname):
    w = synth.config1() if cfgname == "c1" else synth.config2(n_rot=1, n_conf=1)
    _announce(f"receptor grids {cfgname}")
    # FP64 contexts support n_fft <= 64; the 128^3 case is built in FP32
    prec, tol = ("f64", 1e-12) if cfgname == "c1" else ("f32", 2.0 ** -23)
    ctx = _ctx(w, prec)
    g, o = ctx.receptor_grids(w.receptor.xyz[0], w.receptor.q, w.receptor.sigma, w.receptor.eps)
    go, oo = oracle.receptor_grids(w)
    gg = g.cpu().numpy().reshape(go.shape).astype(np.float64)
    for ch in range(3):
        # element-wise relative error (FP32: one rounding of the FP64 value)
        rel = np.max(np.abs(gg[ch] - go[ch]) / np.maximum(np.abs(go[ch]), 1e-300))
        assert rel <= tol, (ch, rel)
    if w.clash_mode == "occ":
        np.testing.assert_array_equal(o.cpu().numpy().reshape(oo.shape), oo)


# ------------------------------------------------------------------ placement
def test_placement_bit_exact():
    w = synth.config2(n_rot=40, n_conf=2)
    ctx = _ctx(w)
    b = _batch(w)
    for c in range(0, w.ligands[0].n_cfg, 3):
        U, box = ctx.place(b, c)
        u, obox = oracle.place_cfg(w, 0, c)
        np.testing.assert_array_equal(U, np.round(u * 65536).astype(np.int64))
        np.testing.assert_array_equal(box, obox)


# ------------------------------------------------------------------ energies
def _energy_parity(w, cfgs, precision, tol, grids_o=None, **tuning):
    ctx, grids, occ = _gpu_setup(w, precision, **tuning)
    b = _batch(w)
    go, oo = grids_o if grids_o is not None else oracle.receptor_grids(w)
    worst = 0.0
    for c in cfgs:
        _announce(f"energy parity {w.name[:3]} {precision} cfg {c}")
        psi, clash = ctx.energy_grid(0, b, c, w.T)
        r = oracle.config_eval(w, go, oo, 0, c)
        assert psi.shape == r["psi"].shape
        if r["psi"].size == 0:
            continue
        e2, emax = _norm_err(psi.cpu().numpy(), r["psi"])
        worst = max(worst, e2, emax)
        assert e2 <= tol and emax <= tol, (c, e2, emax)
        if r["clash"] is not None:
            np.testing.assert_array_equal(clash.cpu().numpy(), r["clash"])
        else:
            assert int(clash.sum()) == 0
    return worst


def test_energy_c1_fp64_cap():
    w = synth.config1()
    _energy_parity(w, [0, 1, 17, 42, 99], "f64", TOL_F64)


@pytest.mark.parametrize("edirect", [1, 0, 2])
def test_energy_c2_fp32_occ(edirect):
    w = synth.config2(n_rot=12, n_conf=8)
    _energy_parity(w, [0, 13, 27, 40, 66, 95], "f32", TOL_F32, energy_xy_direct=edirect)


@pytest.mark.parametrize("fused", [1, 2])
def test_energy_c2_fp32_occ_fused(fused):
    """Fused path (energy planes from the forward pass, or z inputs formed
    in the z kernel): energies and the clash masks of the bitwise test
    against the oracle's direct sums and exact overlap test."""
    w = synth.config2(n_rot=12, n_conf=8)
    _energy_parity(w, [0, 5, 13, 27, 40, 66, 81, 95], "f32", TOL_F32, fused=fused)


def test_energy_c2_fp32_cap_and_fp64_n64():
    """Ragged smaller grids: 40^3 receptor in a 64^3 FFT, both precisions."""
    w = synth.config2(n_rot=4, n_conf=2)
    w.n_rec, w.n_fft = 60, 64
    w.origin = -0.5 * (60 - 1) * w.h * np.ones(3)
    for prec, tol in [("f32", TOL_F32), ("f64", TOL_F64)]:
        for ed in (1, 0, 2):
            _energy_parity(w, [0, 3, 5], prec, tol, energy_xy_direct=ed)
        for fu in (1, 2):
            _energy_parity(w, [0, 3, 5], prec, tol, fused=fu)
    w.clash_mode = "cap"
    _energy_parity(w, [1, 6], "f32", TOL_F32)
    for fu in (1, 2):
        _energy_parity(w, [1, 6], "f32", TOL_F32, fused=fu)


def test_energy_c2_fp32_cap():
    """Cap mode on the c2 grid (128^3 FFT), plane and fused paths, 1e-5
    normwise and in max (measured: 3e-7 plane path; 2e-6 on the 64^3 grid
    above)."""
    w = synth.config2(n_rot=12, n_conf=8)
    w.clash_mode = "cap"
    _energy_parity(w, [0, 5, 13, 27, 40], "f32", TOL_F32)
    _energy_parity(w, [0, 13, 40], "f32", TOL_F32, fused=1)


@pytest.mark.parametrize("n_fft,h,prec", [(32, 0.8, "f32"), (64, 0.4, "f32"), (32, 0.8, "f64")])
def test_direct_energy_many_atoms_per_plane(n_fft, h, prec):
    """A flat 40-atom ligand with identity rotations puts every atom in two
    z-planes, more than one pass of the per-atom tables of the direct energy
    transform (energy mode 2) at these FFT sizes; modes 0 and 2 both match
    the oracle."""
    n_rec = n_fft - 2
    w = synth.tiny(seed=11, n_rec=n_rec, n_fft=n_fft, h=h, n_rec_atoms=250, n_lig_atoms=40, n_cfg=3,
                   clash_mode="occ", precision=prec, r_ball=0.45 * n_rec * h)
    L = w.ligands[0]
    L.conformers[..., 2] *= 0.02
    L.cfg_quat[:] = [1.0, 0.0, 0.0, 0.0]
    u, box = oracle.place_cfg(w, 0, 0)
    assert len(set(np.floor(u[:, 2]).astype(int).tolist())) <= 2
    for ed in (0, 2):
        _energy_parity(w, [0, 1, 2], prec, TOL_F32 if prec == "f32" else TOL_F64, energy_xy_direct=ed)
    for fu in (1, 2):
        _energy_parity(w, [0, 1, 2], prec, TOL_F32 if prec == "f32" else TOL_F64, fused=fu)


def test_single_point_charge_gpu():
    """One ligand atom of charge 1 (no LJ) at an integer lattice position
    reproduces the shifted receptor ELE grid."""
    w = synth.tiny(seed=3, n_rec=30, n_fft=32, h=0.5, n_rec_atoms=80, n_lig_atoms=1, n_cfg=2,
                   clash_mode="cap", precision="f64", r_ball=6.0)
    L = w.ligands[0]
    L.q[:] = 1.0
    L.eps[:] = 0.0
    ctx, grids, _ = _gpu_setup(w, "f64")
    b = _batch(w)
    psi, _ = ctx.energy_grid(0, b, 0, w.T)
    g = grids[0, 0].cpu().numpy()
    Vz, Vy, Vx = psi.shape
    # a single atom is placed at u = (2,2,2)
    np.testing.assert_allclose(psi.cpu().numpy(), g[2:2 + Vz, 2:2 + Vy, 2:2 + Vx], rtol=1e-12, atol=1e-11)
    ctx32, grids32, _ = _gpu_setup(w, "f32")
    psi32, _ = ctx32.energy_grid(0, b, 0, w.T)
    g32 = grids32[0, 0].cpu().numpy()
    e2, emax = _norm_err(psi32.cpu().numpy(), g32[2:2 + Vz, 2:2 + Vy, 2:2 + Vx])
    assert e2 < 1e-6 and emax < 1e-6


# ------------------------------------------------------------------ partials, B, dG
def _argmin_parity(w, go, oo, lig, c0, am_gpu, parts, precision):
    """argmin (linear index (tz Vy + ty) Vx + tx of the lowest energy, lowest
    index on ties, -1 with nothing finite).  FP64: identical to the oracle's.
    FP32: identical wherever the oracle's minimum is unique by more than
    1e-5 max|Psi| (the energy tolerance); elsewhere the GPU's pick must be a
    clash-free translation whose oracle energy lies within that margin of the
    minimum."""
    am_g = np.asarray(am_gpu, np.int64)
    am_o = parts[:, 5].astype(np.int64)
    fin = parts[:, 3] > 0
    np.testing.assert_array_equal(am_g[~fin], -1)
    if precision == "f64":
        np.testing.assert_array_equal(am_g[fin], am_o[fin])
        return
    for c in np.flatnonzero(fin & (am_g != am_o)):
        r = oracle.config_eval(w, go, oo, lig, int(c))
        psi = r["psi"].ravel()
        ok = np.ones(psi.size, bool) if r["clash"] is None else r["clash"].ravel() == 0
        k = int(am_g[c])
        assert 0 <= k < psi.size and ok[k], (c0 + c, k)
        assert psi[k] - psi[am_o[c]] <= 1e-5 * np.max(np.abs(psi)), (c0 + c, k, am_o[c], psi[k], psi[am_o[c]])


def _scan_parity(w, precision, tolB, **tuning):
    import torch
    ctx, grids, occ = _gpu_setup(w, precision, **tuning)
    b = _batch(w)
    _announce(f"scan {w.name[:3]} {precision} n_cfg={b.n_cfg} n_snap={w.receptor.n_snap}")
    buf = ctx.scan(b, w.T)
    torch.cuda.synchronize()
    P = ctx.partials_numpy(buf, ctx.n_snap, b.n_cfg)
    B, res = ctx.reduce(b, buf, w.T)
    kt = est.kT(w.T)
    for l in range(len(w.ligands)):
        c0, c1 = b.cfg_off[l], b.cfg_off[l + 1]
        Bo = []
        for s in range(w.receptor.n_snap):
            go, oo = oracle.receptor_grids(w, s)
            parts, boxes = oracle.scan(w, go, oo, lig_idx=l)
            g = P[s, c0:c1]
            np.testing.assert_array_equal(g["n_valid"], parts[:, 2].astype(np.int64))
            np.testing.assert_array_equal(g["n_finite"], parts[:, 3].astype(np.int64))
            fin = parts[:, 3] > 0
            # per-configuration log Z and minimum
            lz_g = np.where(fin, g["m"] + np.log(np.where(fin, g["s"], 1.0)), -np.inf)
            lz_o = est.log_z(parts)
            assert np.max(np.abs(kt * (lz_g[fin] - lz_o[fin]))) < tolB
            assert np.max(np.abs(g["psi_min"][fin] - parts[fin, 4])) < tolB
            _argmin_parity(w, go, oo, l, c0, g["argmin"], parts, precision)
            Bo.append(est.bpmf(parts, w.T))
            assert abs(B[l, s] - Bo[-1]) < tolB, (l, s, B[l, s], Bo[-1])
        vs = est.v_site(boxes, w.n_rec, w.h)
        dg = est.dg_standard(np.array(Bo), w.receptor.weights, vs, w.T)
        assert abs(res["v_site"][l] - vs) <= 1e-9 * vs
        assert abs(res["dG"][l] - dg) < tolB, (res["dG"][l], dg)
    return P, B, res


@pytest.mark.parametrize("edirect", [1, 0, 2])
def test_scan_c1_fp64(edirect):
    _scan_parity(synth.config1(), "f64", 1e-8, energy_xy_direct=edirect)


@pytest.mark.parametrize("fused,chunk", [(1, 256), (1, 7), (2, 256), (2, 7)])
def test_scan_c1_fp64_fused(fused, chunk):
    _scan_parity(synth.config1(), "f64", 1e-8, fused=fused, configs_per_chunk=chunk)


@pytest.mark.parametrize("edirect,chunk", [(1, 256), (0, 256), (1, 7), (2, 256), (2, 7)])
def test_scan_c2_subset_fp32(edirect, chunk):
    w = synth.subset(synth.config2(), 96, stride=83)
    _scan_parity(w, "f32", 0.01, energy_xy_direct=edirect, configs_per_chunk=chunk)


@pytest.mark.parametrize("fused,chunk,graph", [(1, 256, 0), (1, 7, 0), (1, 32, 1), (2, 256, 0), (2, 7, 0), (2, 32, 1)])
def test_scan_c2_subset_fp32_fused(fused, chunk, graph):
    w = synth.subset(synth.config2(), 96, stride=83)
    _scan_parity(w, "f32", 0.01, fused=fused, configs_per_chunk=chunk, use_graph=graph)


def test_wide_occupancy_balls_take_the_plane_path():
    """Ligand atoms whose occupancy balls reach more than the clash table's
    8-point margin past the box (sigma x 1.3: radius up to 9.3 points) are
    scanned on the plane path even with the fused path selected; results
    match the oracle."""
    w = synth.subset(synth.config2(), 40, stride=197)
    w.ligands[0].sigma = w.ligands[0].sigma * 1.3
    _scan_parity(w, "f32", 0.01, fused=1, configs_per_chunk=16)


@pytest.mark.parametrize("snap_pass,chunk,edirect", [(16, 256, 0), (1, 256, 0), (2, 5, 0), (1, 64, 2), (16, 9, 2)])
def test_scan_batched_uneven_ligands_three_snapshots(snap_pass, chunk, edirect):
    """Ragged batch: 5 ligands of 8..40 atoms with different configuration
    counts against 3 jittered snapshots; snapshots handled all in one z pass,
    one per pass, or 2 + 1, and chunks that cross ligand boundaries."""
    w = synth.config3(n_ligands=5, n_snap=3, cfg_scale=0.02)
    P, B, res = _scan_parity(w, "f32", 0.01, snapshots_per_pass=snap_pass, configs_per_chunk=chunk,
                             energy_xy_direct=edirect)
    assert P.shape[0] == 3


@pytest.mark.parametrize("fused,chunk", [(1, 256), (1, 5), (2, 256), (2, 5)])
def test_scan_batched_uneven_ligands_three_snapshots_fused(fused, chunk):
    """The ragged three-snapshot batch on the fused path: one occupancy-run
    pass per chunk, the clash test, z pass and inverse per snapshot."""
    w = synth.config3(n_ligands=5, n_snap=3, cfg_scale=0.02)
    P, B, res = _scan_parity(w, "f32", 0.01, fused=fused, configs_per_chunk=chunk)
    assert P.shape[0] == 3


@pytest.mark.parametrize("fused,snap_pass", [(1, 1), (2, 1), (0, 1), (0, 3)])
def test_clash_stream_matches_one_stream(fused, snap_pass):
    """The second stream (fused path: the clash test of the next item beside
    the current z pass and inverse; plane path: the inverse of one z pass
    beside the next; double-buffered, event-ordered) gives the same partials
    bit for bit as one stream, eagerly and as a captured graph replayed
    several times with eager work and synchronizations between replays;
    ragged three-snapshot batch, chunks of 5 (many items)."""
    import torch
    w = synth.config3(n_ligands=5, n_snap=3, cfg_scale=0.02)
    tun = dict(fused=fused, configs_per_chunk=5, clash_stream=0, use_graph=0)
    if fused == 0:
        tun.update(snapshots_per_pass=snap_pass, energy_xy_direct=0)
    ctx, grids, occ = _gpu_setup(w, **tun)
    b = _batch(w)
    _announce(f"second stream vs one stream: fused={fused} snapshots per pass {snap_pass} n_cfg={b.n_cfg} n_snap=3")
    ref = ctx.scan(b, w.T).cpu().numpy()
    ctx.set_tuning(clash_stream=1)
    np.testing.assert_array_equal(ctx.scan(b, w.T).cpu().numpy(), ref)
    ctx.set_tuning(use_graph=1)
    out = ctx.alloc_partials(b)
    for rep in range(3):
        out.zero_()
        ctx.scan(b, w.T, out)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy(), ref)
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()
    assert ctx.get_tuning()["clash_stream"] == 1


def test_cfg_select_and_empty_configs():
    """cfg_select scans a subset; unscanned configurations still count their
    translations; a configuration whose box exceeds the grid has n_valid 0."""
    import torch
    w = synth.config2(n_rot=10, n_conf=2)
    sel = np.zeros(20, np.uint8)
    sel[::3] = 1
    ctx, grids, occ = _gpu_setup(w)
    b = _batch(w, sel)
    P = ctx.partials_numpy(ctx.scan(b, w.T), 1, 20)[0]
    assert np.all(P["scanned"] == sel)
    assert np.all(P["n_finite"][sel == 0] == 0)
    go, oo = oracle.receptor_grids(w)
    parts, _ = oracle.scan(w, go, oo)
    np.testing.assert_array_equal(P["n_valid"], parts[:, 2].astype(np.int64))
    np.testing.assert_array_equal(P["n_finite"][sel == 1], parts[sel == 1, 3].astype(np.int64))
    # a ligand that does not fit anywhere -> E_NOVALID
    import paper_1708_07045_amd as fd
    big = synth.config2(n_rot=2, n_conf=1)
    big.ligands[0].conformers = big.ligands[0].conformers * 4.0
    with pytest.raises(fd.FFTDGError) as ei:
        ctx.scan(_batch(big), w.T)
    assert ei.value.code == fd._lib.E_NOVALID


def test_all_clash_gives_infinite_bpmf():
    """A receptor whose occupancy grid is full: every translation clashes,
    B = +inf and dG = +inf (a result, not an error)."""
    import torch
    w = synth.config2(n_rot=3, n_conf=1)
    ctx = _ctx(w)
    g, o = ctx.receptor_grids(w.receptor.xyz[0], w.receptor.q, w.receptor.sigma, w.receptor.eps)
    o.fill_(1)
    ctx.set_receptors(g[None], o[None])
    b = _batch(w)
    buf = ctx.scan(b, w.T)
    P = ctx.partials_numpy(buf, 1, b.n_cfg)[0]
    assert np.all(P["n_finite"] == 0) and np.all(P["n_valid"] > 0)
    B, res = ctx.reduce(b, buf, w.T)
    assert math.isinf(B[0, 0]) and math.isinf(res["dG"][0])


def test_importance_weights_reduce():
    """Reduce with per-configuration weights equals the oracle's weighted form."""
    import torch
    w = synth.subset(synth.config2(), 40, stride=200)
    ctx, grids, occ = _gpu_setup(w)
    b = _batch(w)
    buf = ctx.scan(b, w.T)
    rng = np.random.default_rng(3)
    wt = rng.uniform(0.0, 3.0, b.n_cfg)
    wt[::7] = 0.0
    B, _ = ctx.reduce(b, buf, w.T, cfg_weight=wt)
    go, oo = oracle.receptor_grids(w)
    parts, _ = oracle.scan(w, go, oo)
    lz = est.log_z(parts)
    ok = (wt > 0) & np.isfinite(lz)
    Bo = -est.kT(w.T) * (est.lse(np.log(wt[ok]) + lz[ok]) - math.log(parts[:, 2].sum()))
    assert abs(B[0, 0] - Bo) < 0.01


def test_rescan_is_deterministic():
    import torch
    w = synth.subset(synth.config2(), 32, stride=100)
    ctx, grids, occ = _gpu_setup(w)
    b = _batch(w)
    a = ctx.scan(b, w.T).cpu().numpy()
    c = ctx.scan(b, w.T).cpu().numpy()
    np.testing.assert_array_equal(a, c)


def test_graph_replays_match_eager():
    """The captured scan graph, replayed several times with other eager work
    and synchronizations in between, gives exactly the eager results; a new
    batch shape re-captures."""
    import torch
    w = synth.subset(synth.config2(), 48, stride=150)
    w2 = synth.subset(synth.config2(), 20, stride=333)
    ctx, grids, occ = _gpu_setup(w)
    b, b2 = _batch(w), _batch(w2)
    ref = ctx.scan(b, w.T).cpu().numpy()
    ref2 = ctx.scan(b2, w.T).cpu().numpy()
    ctx.set_tuning(use_graph=1)
    out = ctx.alloc_partials(b)
    for rep in range(4):
        ctx.scan(b, w.T, out)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy(), ref)
        x = torch.randn(1 << 20, device="cuda")  # unrelated eager work between replays
        (x * 2).sum().item()
        if rep == 2:
            np.testing.assert_array_equal(ctx.scan(b2, w.T).cpu().numpy(), ref2)
    B, _ = ctx.reduce(b, out, w.T)
    ctx.set_tuning(use_graph=0)
    B0, _ = ctx.reduce(b, ctx.scan(b, w.T), w.T)
    assert B[0, 0] == B0[0, 0]


def test_autotune_picks_valid_schedule():
    import torch
    w = synth.subset(synth.config2(), 160, stride=50)
    ctx, grids, occ = _gpu_setup(w)
    b = _batch(w)
    ref = ctx.partials_numpy(ctx.scan(b, w.T), 1, b.n_cfg)
    tun, ms = ctx.autotune(b, w.T, max_cfgs=64)
    assert tun["configs_per_chunk"] in (64, 128, 256, 512)
    assert tun["energy_xy_direct"] in (0, 1, 2) and tun["use_graph"] in (0, 1)
    assert ms > 0 and ctx.get_tuning() == tun
    got = ctx.partials_numpy(ctx.scan(b, w.T), 1, b.n_cfg)
    np.testing.assert_array_equal(got["n_finite"], ref["n_finite"])
    fin = ref["n_finite"] > 0
    kt = est.kT(w.T)
    lz_a = got["m"][fin] + np.log(got["s"][fin])
    lz_b = ref["m"][fin] + np.log(ref["s"][fin])
    assert np.max(np.abs(kt * (lz_a - lz_b))) < 1e-3
