#!/usr/bin/env python3
"""Throughput of the FFT translational BPMF scan on one MI355X.

One step = the whole hot path over the 8000-configuration T4L-sized workload
(2600-atom cavity receptor, 96^3 grid at 0.25 A zero-padded to a 128^3 FFT,
occupancy clash mode, one 25-atom ligand x 8 conformers x 1000 rotations,
FP32 scan, FP64 averages): receptor spectra, placement, ligand FFTs,
spectral products, inverse FFTs, clash masks, log-sum-exp partials, FP64
BPMF and standard binding free energy.  The receptor grids themselves (Eq. 7
from atoms) are prepared once before timing.

Prints one JSON line on stdout.  Progress goes to stderr.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ligand configs/sec (FFT scan) + configs needed for BPMF ±0.1 kcal/mol, MLP vs plain"
HBM_PEAK_GBS = 8000.0
# FP32 vector peak of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x
# 2 (packed FP32, two FMAs per lane per cycle) x 2.4 GHz = 157.3 TFLOP/s.
# The library is compiled without packed-FP32 instructions, so half of it,
# 78.6 TFLOP/s, is the rate its kernels' instructions can issue at.
VALU_FP32_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2 * 2.4e9 / 1e12
VALU_FP32_NONPACKED_TFLOPS = VALU_FP32_PEAK_TFLOPS / 2


def zpass_flops(n_fft: int, n_in: int, n_out: int, occ_product: bool, n_cfg: int, n_snap: int,
                snap_pass: int) -> float:
    """Algorithmic flops of the z pass for n_cfg configurations x n_snap
    snapshots: over the N (N/2 + 1) pencils, 5 N log2 N per complex length-N
    transform (n_in forward, once per pass of snap_pass snapshots; n_out
    inverse per snapshot) and per spectral point 8 flops per energy
    channel's R * conj(L) multiply-add (3 channels), plus 6 for the
    occupancy product on the plane path."""
    N = n_fft
    pencils = N * (N // 2 + 1)
    t = 5.0 * N * math.log2(N)
    passes = -(-n_snap // max(1, snap_pass))
    return float(n_cfg) * pencils * (n_in * t * passes + n_snap * (n_out * t + N * (24 + (6 if occ_product else 0))))


def pruned_bytes_per_cfg(P, n_fft: int, occ: bool, B_rc: int) -> float:
    """Algorithmic bytes per configuration of the scan in the pruned-transform
    traffic model (what the method must move when a 3D FFT does not fit one
    CU's LDS): 16 N (N/2 + 1) (n_in L_z + n_out V_z) + 8 S_h
    n_rc / B_rc, with n_in = n_rc = 4, n_out = 2 in occupancy mode (3, 1 in
    cap mode), L_z = B_z + 1 and V_z from this workload's placements, S_h =
    N^2 (N/2 + 1) and B_rc configurations per receptor read.  Evaluated over
    the scanned configurations: the mean of the per-configuration figure."""
    import numpy as np
    N = n_fft
    nh = N * (N // 2 + 1)
    n_in, n_out = (4, 2) if occ else (3, 1)
    box_z = np.asarray(P["box_z"], dtype=np.float64)
    vz = np.asarray(P["V_z"], dtype=np.float64)
    per = 16.0 * nh * (n_in * (box_z + 1.0) + n_out * vz) + 8.0 * N * nh * n_in / max(1, B_rc)
    return float(per.mean())


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "scan_t4l_8000cfg_hbm_traffic.md")
KERNEL_SOURCES = ["scan_kernels.hip", "fused_kernels.hip", "fft_device.hpp", "scan_types.hpp", "kernels.hpp",
                  "scan_common.hpp", "fused.hpp"]


def kernel_source_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1708_07045_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(tuning: dict):
    """HBM bytes per configuration of one scan (all of its kernels) measured
    by the FETCH_SIZE / WRITE_SIZE counter runs recorded in the profile
    summary, if those runs used these kernel sources and scan path (else
    None)."""
    if not os.path.exists(TRAFFIC_PROFILE):
        return None
    rec = {}
    for line in open(TRAFFIC_PROFILE):
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            rec[k.strip()] = v.strip().strip("`")
    try:
        # per configuration the scan's traffic does not depend on the chunk
        # size except for the receptor spectra read once per chunk (about 1 %
        # of the bytes at 128 configurations per chunk, less above)
        if rec["kernel_source_sha256"] != kernel_source_digest():
            return None
        if int(rec.get("fused", 0)) != tuning.get("fused", 0) or tuning["configs_per_chunk"] < 128:
            return None
        if tuning.get("fused", 0) == 0 and int(rec["energy_xy_direct"]) != tuning["energy_xy_direct"]:
            return None
        return float(rec["hbm_bytes_per_cfg"])
    except (KeyError, ValueError):
        return None


ORACLE_GOLDEN = os.path.join(ROOT, "tests", "golden", "c2_oracle.json")


def precision_vs_oracle(args, result):
    """FP32 scan (FP64 accumulation) against the FP64 oracle's stored results
    of the same T4L-sized workload (written by tests/golden/make_c2_oracle.py)."""
    if args.workload != "c2" or not os.path.exists(ORACLE_GOLDEN):
        return None
    ref = json.load(open(ORACLE_GOLDEN))["occ"]
    B, dG = float(result["B"][0, 0]), float(result["res"]["dG"][0])
    return {"oracle": "FP64 direct trilinear sums, occupancy mode, all 8000 configurations",
            "bpmf_abs_err_kcal_mol": abs(B - ref["B"]), "dG_abs_err_kcal_mol": abs(dG - ref["dG"]),
            "oracle_bpmf_kcal_mol": ref["B"], "oracle_dG_kcal_mol": ref["dG"]}


def pose_resampling(ctx, batch, partials, T, K: int = 100):
    """Sampling importance resampling of K poses from the finished scan
    (the solvation leg's input), timed."""
    import torch
    from workload import synth
    u = synth.uniforms(77, 2 * K)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cfg, t, psi = ctx.sample_poses(batch, partials, 0, 0, T, u)
    dt = time.perf_counter() - t0
    return {"poses": K, "distinct_configurations": int(len(set(cfg.tolist()))), "seconds": dt,
            "mean_psi_kcal_mol": float(psi.mean())}


def spacing_study(w, ctx, batch, partials):
    """Grid energies at 0.125 / 0.25 / 0.5 / 0.8 A against direct pair sums
    over 200 resampled poses (the paper's spacing comparison), timed."""
    import torch
    from paper_1708_07045_amd import spacing
    t0 = time.perf_counter()
    res = spacing.study(w, ctx, batch, partials, n_poses=200)
    torch.cuda.synchronize()
    res["seconds"] = time.perf_counter() - t0
    return res


def copy_calibration():
    """One 1 GiB device-to-device copy (a plain copy kernel of known size),
    for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    n = 1 << 28
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    log(f"copy calibration: {4 * n} bytes read and written by one copy kernel")
    del a, b
    torch.cuda.empty_cache()


def copy_bandwidth(stream=None, n_bytes: int = 1 << 31, reps: int = 5) -> float:
    """Measured device-to-device copy rate (bytes read + bytes written per
    second, GB/s) of a plain copy kernel over n_bytes, timed with HIP events."""
    import torch
    a = torch.ones(n_bytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbps = 2.0 * n_bytes * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbps


def cpu_fft_baseline(w, budget_s: float):
    """The paper's own method on the host: FP64 real-to-complex 3D FFTs
    (scipy.fft, all host threads) for each configuration, over a bounded,
    evenly strided sample of the same configurations."""
    import numpy as np
    import oracle
    from oracle import fft_cpu
    go, oo = oracle.receptor_grids(w)
    spec = fft_cpu.receptor_spectra(w, go, oo)
    n_all = w.ligands[0].n_cfg
    fft_cpu.scan(w, spec, 0, np.array([0]))  # transform plans and first-touch pages, untimed
    t0 = time.perf_counter()
    fft_cpu.scan(w, spec, 0, np.array([1, n_all // 3, n_all // 2, n_all - 1]))
    rate = 4 / (time.perf_counter() - t0)
    n = int(min(n_all, max(4, rate * budget_s)))
    sel = np.linspace(0, n_all - 1, n).astype(int)
    t0 = time.perf_counter()
    fft_cpu.scan(w, spec, 0, sel)
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "configs/s", "cores": fft_cpu._workers(), "kind": "fft_cpu",
            "cpu_model": cpu_model(),
            "sample": f"{n} of {n_all} configurations (evenly strided), FP64 scipy.fft (pocketfft) rfftn/irfftn "
                      f"of the {w.n_fft}^3 grids, 4 forward + 2 inverse transforms per configuration, {dt:.1f} s"}


# Timings the paper quotes for this path (Table 4): CPU wall time for one
# ligand's gas-phase BPMF on T4L, CPU model and precision not stated.  The
# configurations per BPMF are not stated for the table; ~1000 is assumed
# for the rates.
PAPER_CPU_TIMES = {
    "source": "Table 4 (CPU time per ligand, p-xylene; CPU not specified, precision not stated)",
    "fft_16A_0.25A_s": 2 * 60 + 19, "fft_16A_0.125A_s": 28 * 60 + 26, "fft_62A_0.25A_s": 7 * 3600 + 3 * 60 + 10,
    "configs_per_s_if_1000_configs": {"16A_0.25A": 1000 / 139.0, "16A_0.125A": 1000 / 1706.0,
                                      "62A_0.25A": 1000 / 25390.0},
}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def oracle_c1_rate():
    """The oracle over the whole tiny FP64 workload (300-atom receptor, 32^3
    grid, one 12-atom ligand x 100 rotations, cap mode): configurations/s."""
    import oracle
    from workload import synth
    w = synth.config1()
    go, oo = oracle.receptor_grids(w)
    t0 = time.perf_counter()
    oracle.scan(w, go, oo)
    dt = time.perf_counter() - t0
    return {"value": w.ligands[0].n_cfg / dt, "unit": "configs/s", "sample": "all 100 configurations",
            "seconds": dt}


def cpu_baseline(w, budget_s: float):
    """The FP64 oracle on the host cores over a bounded, evenly strided sample
    of the same configurations; returns configs/s and the sample."""
    import numpy as np
    import oracle
    t = time.perf_counter()
    go, oo = oracle.receptor_grids(w)
    log(f"cpu baseline: oracle receptor grids {time.perf_counter() - t:.1f}s (not timed)")
    n_all = w.ligands[0].n_cfg
    probe = np.arange(0, n_all, max(1, n_all // 32))[:32]
    t0 = time.perf_counter()
    oracle.scan(w, go, oo, cfgs=probe)
    dt = time.perf_counter() - t0
    rate = len(probe) / dt
    n_more = int(min(n_all, max(len(probe), rate * budget_s)))
    sel = np.linspace(0, n_all - 1, n_more).astype(int)
    t0 = time.perf_counter()
    oracle.scan(w, go, oo, cfgs=sel)
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or len(os.sched_getaffinity(0))
    return {"value": len(sel) / dt, "unit": "configs/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{len(sel)} of {n_all} configurations (evenly strided), FP64 direct trilinear sum "
                      f"+ exact clash test + partials, OpenMP over configurations, {dt:.1f} s",
            "tiny_workload": oracle_c1_rate()}


def batched_timing(reps: int = 3):
    """The whole batched workload (141 ligands of 8-40 atoms, 200-2000
    configurations each, 10 jittered receptor snapshots, 128^3 FFT) scanned
    exhaustively under the autotuned schedule: the median of `reps` scans
    timed with HIP events on the library's stream (receptor spectra built
    beforehand), the per-kernel table of one more, profiled, scan, and the
    pruned-transform model's bytes per configuration at that rate."""
    import numpy as np
    import torch
    import paper_1708_07045_amd as fd
    from workload import synth
    w = synth.config3(cfg_scale=1.0)
    S = w.receptor.n_snap
    ctx = fd.FFTDG.from_workload(w)
    gl, ol = [], []
    for sn in range(S):
        g, o = ctx.receptor_grids(w.receptor.xyz[sn], w.receptor.q, w.receptor.sigma, w.receptor.eps)
        gl.append(g)
        ol.append(o)
    ctx.set_receptors(torch.stack(gl).contiguous(), torch.stack(ol).contiguous(), w.receptor.weights)
    del gl, ol
    b = fd.Batch(w.ligands)
    log(f"batched timing: {len(w.ligands)} ligands, {b.n_cfg} configurations x {S} snapshots")
    # 1024 sampled configurations x 10 snapshots per candidate schedule keep
    # the tuner within a couple of minutes
    tun, _ = ctx.autotune(b, w.T, max_cfgs=1024)
    log(f"batched schedule {tun}")
    out = ctx.alloc_partials(b)
    ctx.scan(b, w.T, out)
    torch.cuda.synchronize()
    ms = []
    for r in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ctx.scan(b, w.T, out)
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
        log(f"batched scan {r + 1}/{reps}: {ms[-1]:.0f} ms")
    ctx.profile(True)
    ctx.scan(b, w.T, out)
    prof = ctx.profile_read()
    ctx.profile(False)
    med = float(np.median(ms))
    scans = b.n_cfg * S
    boxes = ctx.boxes(b)
    pb = pruned_bytes_per_cfg({"box_z": boxes[:, 2], "V_z": np.maximum(w.n_rec - boxes[:, 2], 0)}, w.n_fft,
                              w.clash_mode == "occ", tun["configs_per_chunk"])
    rate = scans / (med / 1e3)
    B, res = ctx.reduce(b, out, w.T)
    return {"workload": f"batched: {len(w.ligands)} ligands of 8-40 atoms, {b.n_cfg} configurations, {S} jittered "
                        f"receptor snapshots, {w.n_rec}^3 grid in a {w.n_fft}^3 FFT, occupancy clash mode",
            "tuning": tun, "scan_ms": ms, "scan_ms_median": med, "scans_per_s": rate,
            "configs_per_s": b.n_cfg / (med / 1e3),
            "kernels_ms": {k: v[0] for k, v in prof.items() if v[1] > 0},
            "pruned_bytes_per_scan": pb, "pruned_GBps": pb * rate / 1e9, "pruned_frac_of_peak": pb * rate / 1e9 / HBM_PEAK_GBS,
            "dG_mean_kcal_mol": float(np.mean(res["dG"]))}


def mlp_rates(X, t, wt, rows, train_batch: int = 512, reps: int = 5):
    """Proposal-network throughput in samples per second on a throwaway
    network of the proposal's shape (residual form, width 256): forward
    over every row of X in blocks of 512 (the batch the proposal predicts
    with) and of 4096, and Adam training steps of train_batch rows.  HIP
    events on the network's stream (torch's current stream); median of
    reps after one untimed pass."""
    import numpy as np
    import torch
    from paper_1708_07045_amd import proposal as prop

    def timed(fn):
        fn()
        ms = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        return float(np.median(ms))

    n = int(X.shape[0])
    out = {"rows": n, "n_in": int(X.shape[1]), "width": 256}
    for mb in (512, 4096):
        net = prop.make_network(int(X.shape[1]), 256, residual=True, max_batch=mb)
        out[f"forward_samples_per_s_block{mb}"] = n / (timed(lambda: net.forward(X)) * 1e-3)
        if mb == train_batch:
            steps = max(1, min(rows.size // train_batch, 64))
            idx = torch.as_tensor(np.asarray(rows[:steps * train_batch], np.int32), device=X.device)

            def train():
                for k in range(steps):
                    net.train_step(X, t, wt, idx[k * train_batch:(k + 1) * train_batch], 1e-3)

            out["train_samples_per_s"] = int(idx.shape[0]) / (timed(train) * 1e-3)
            out["train_batch"] = train_batch
        net.close()
    return out


def configs_needed(args, fine_tuning=None):
    """Configurations a BPMF estimate needs for +-0.1 kcal/mol in every
    snapshot, plain uniform sampling vs the learned proposal, on the batched
    141-ligand x 10-snapshot workload (seeded split: 101 training ligands,
    40 held out).  Costs are fine-scan equivalents; a coarse pre-scan counts
    at its measured cost ratio.  fine_tuning: the fine scans' schedule
    (else autotuned here)."""
    import numpy as np
    import torch
    import paper_1708_07045_amd as fd
    from paper_1708_07045_amd import proposal as prop
    from workload import synth

    w = synth.config3(cfg_scale=1.0)
    T = w.T
    kT = prop.KCAL_R * T
    b = fd.Batch(w.ligands)
    S = w.receptor.n_snap
    log(f"configs needed: {len(w.ligands)} ligands, {b.n_cfg} configurations x {S} snapshots")
    ctx_f = prop.make_context(w)
    # coarse pre-scan at twice the spacing: against every snapshot, one
    # receptor at the snapshots' mean coordinates, every other snapshot, the
    # first snapshot, or a cascade (default: the mean receptor for every
    # configuration, then every snapshot for each ligand's top fraction by
    # that score); repulsion capped (default) or overlaps excluded
    cascade = args.is_coarse == "cascade"
    cdesc = prop.coarse_desc(w, args.is_coarse_factor)
    csnaps = None if cascade else args.is_coarse_snapshots
    if csnaps == "half":
        csnaps = list(range(0, S, 2))
    ctx_c = prop.make_context(w, cdesc, snapshots=csnaps, clash_mode=args.is_coarse_clash)
    if fine_tuning:  # the batched timing tuned this same workload already
        ctx_f.set_tuning(**fine_tuning)
        log(f"fine schedule {fine_tuning} (from the batched timing)")
    else:
        log(f"fine schedule {ctx_f.autotune(b, T, max_cfgs=1024)[0]}")
    log(f"coarse schedule {ctx_c.autotune(b, T, max_cfgs=2048)[0]}")

    def timed_scan(ctx, bb):
        out = ctx.scan(bb, T)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.scan(bb, T, out)
        torch.cuda.synchronize()
        return out, time.perf_counter() - t0

    part_f, t_f = timed_scan(ctx_f, b)
    log(f"exhaustive fine scan {t_f:.2f}s")
    per_fine = t_f / b.n_cfg          # seconds per configuration of the fine scan
    if cascade:
        ctx_m = prop.make_context(w, cdesc, snapshots="mean", clash_mode=args.is_coarse_clash)
        log(f"mean-receptor schedule {ctx_m.autotune(b, T, max_cfgs=2048)[0]}")
        part_m, t_m = timed_scan(ctx_m, b)
        y_mean = prop.coarse_score(ctx_m, b, part_m)
        cand = np.zeros(b.n_cfg, np.uint8)
        for l in range(b.n_lig):
            a0, a1 = b.cfg_off[l], b.cfg_off[l + 1]
            k = int(np.ceil(args.is_cascade_frac * (a1 - a0)))
            cand[a0 + np.argsort(-y_mean[a0:a1], kind="stable")[:k]] = 1
        part_c, t_c = timed_scan(ctx_c, b.with_select(cand))
        # fine-scan equivalents per configuration: the mean-receptor scan for
        # all, the every-snapshot scan for the candidates
        extra_cfg = t_m / t_f + cand * (t_c / max(1, int(cand.sum()))) / per_fine
        log(f"cascade: mean receptor {t_m:.2f}s for all, every snapshot {t_c:.2f}s for {int(cand.sum())} candidates")
    else:
        part_c, t_c = timed_scan(ctx_c, b)
        extra_cfg = np.full(b.n_cfg, t_c / t_f)
    rho = float(np.mean(extra_cfg))
    B_ex, res_ex = ctx_f.reduce(b, part_f, T)
    log(f"exhaustive fine scan {t_f:.2f}s, coarse pre-scan cost ratio {rho:.3f}")
    train_l, test_l = prop.split_ligands(len(w.ligands), 101)
    # the training ligands split again: 81 to fit, 20 to choose the mixture
    # temperature and the number of epochs (the held-out 40 decide nothing)
    vperm = np.random.Generator(np.random.PCG64(np.random.SeedSequence([170807045, 12]))).permutation(train_l)
    fit_l, val_l = np.sort(vperm[:81]), np.sort(vperm[81:])
    rows = prop.rows_of(b.cfg_off, fit_l)
    X = prop.inputs(ctx_f, ctx_c, b, part_c, with_scan=True)
    # the coarse prediction (skip input): per-receptor maximum of the relative
    # log weight (the first scan descriptor when there is one coarse receptor);
    # in the cascade, non-candidates keep their mean-receptor score 5 nats down
    y_c = prop.coarse_score(ctx_c, b, part_c)
    if cascade:
        y_c = np.where(cand == 1, y_c, y_mean - 1.0)
    X[:, fd.N_FEATURES] = torch.as_tensor(y_c.astype(np.float32), device=X.device)
    Xc = X[:, :fd.N_FEATURES].contiguous()
    P_f = ctx_f.partials_numpy(part_f, S, b.n_cfg)
    if args.is_target == "snapmax":
        t, wt = prop.targets_snapmax(P_f, b.cfg_off, device=X.device)
    else:
        t, wt = prop.targets(ctx_f, b, part_f)
    alpha = 0.1
    # plan (mixture temperature, exact share of the budget) chosen on the
    # validation ligands with the epochs
    plans = [(tau, share) for share in args.is_exact_shares for tau in (0.5, 1.0, 2.0)]
    val_score = prop.pool_fraction_scorer(w, b, P_f, val_l, alpha, plans, kT, reps=50)
    pred, tau_of, t_train, epochs_of, val_of = {}, {}, {}, {}, {}
    y_coarse = X[:, fd.N_FEATURES].cpu().numpy()
    val_of["coarse"], tau_of["coarse"] = val_score(y_coarse)
    pred["coarse"] = y_coarse
    log(f"coarse: validation mean fraction {val_of['coarse']:.3f} at plan {tau_of['coarse']}")
    # net_scan: residual form (coarse relative log weight through the skip;
    # at epoch 0 it is the coarse score); net_cfg: configuration descriptors
    # only.  The epoch count is chosen on the validation ligands.
    for name, xin, resid in (("net_scan", X, True), ("net_cfg", Xc, False)):
        net = prop.make_network(int(xin.shape[1]), 256, residual=resid)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        keep = prop.fit_selected(net, xin, t, wt, rows, val_score, args.is_epochs, log=log, name=name)
        torch.cuda.synchronize()
        t_train[name] = time.perf_counter() - t0
        pred[name] = net.forward(xin).cpu().numpy()
        tau_of[name], epochs_of[name], val_of[name] = keep["tau"], keep["epoch"], keep["score"]
        log(f"{name}: {args.is_epochs} epochs on {rows.size} rows in {t_train[name]:.1f}s (with validation), "
            f"last batch loss {keep['loss']:.4f}; kept epoch {keep['epoch']}")
    log(f"plans (mixture temperature in nats, exact share) chosen on validation ligands: {tau_of}")
    mlp = mlp_rates(X, t, wt, rows)
    log(f"proposal network: forward {mlp['forward_samples_per_s_block512']:.3g} samples/s (blocks of 512), "
        f"{mlp['forward_samples_per_s_block4096']:.3g} (4096); training {mlp['train_samples_per_s']:.3g} samples/s")
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([170807045, 21])))
    per = []
    for l in test_l:
        Zs = prop.ligand_weights(P_f, b.cfg_off, l)
        Pl = Zs.shape[1]
        row = {"ligand": int(l), "n_cfg": int(Pl), "plain": prop.kstar_plain(Zs, kT, rng, reps=args.is_reps)}
        for name in pred:
            yl = pred[name][b.cfg_off[l]:b.cfg_off[l + 1]]
            k, bf = prop.kstar_is(prop.sub_batch(w, l), Zs, yl, alpha, tau_of[name][0], kT, 2000 + int(l),
                                  reps=args.is_reps, exact_share=tau_of[name][1])
            extra = float(extra_cfg[b.cfg_off[l]:b.cfg_off[l + 1]].sum()) if name in ("net_scan", "coarse") else 0.0
            row[name] = min(float(Pl), k + extra)
            row[name + "_budget"] = bf
        # gain test: the network's plan with its proposal replaced by a
        # uniform one (no pre-scan, so no extra cost)
        k, bf = prop.kstar_is(prop.sub_batch(w, l), Zs, np.zeros(Pl, np.float32), alpha, tau_of["net_scan"][0],
                              kT, 2000 + int(l), reps=args.is_reps, exact_share=tau_of["net_scan"][1])
        row["uniform"], row["uniform_budget"] = min(float(Pl), k), bf
        per.append(row)
        log(f"ligand {l}: P={Pl} plain {row['plain']:.0f}  net_scan {row['net_scan']:.0f}  "
            f"coarse {row['coarse']:.0f}  net_cfg {row['net_cfg']:.0f}  uniform {row['uniform']:.0f}")
    med = lambda key: float(np.median([r["plain"] / r[key] for r in per]))
    # one real importance-sampled scan of the held-out ligands at 10 % of
    # the configurations (exact top and draws split as the plan chosen on the
    # validation ligands), against the exhaustive, with the network's
    # proposal and with the coarse score's
    bt = fd.Batch([w.ligands[l] for l in test_l])
    u = synth.uniforms(31, bt.n_cfg)
    Bref = B_ex[test_l]
    dref = res_ex["dG"][test_l]
    is_runs = {}
    for name in ("net_scan", "coarse"):
        yt = np.concatenate([pred[name][b.cfg_off[l]:b.cfg_off[l + 1]] for l in test_l])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tau, share = tau_of[name]
        est = prop.is_estimate(ctx_f, bt, yt, 0.1 * share, 0.1 * (1.0 - share), alpha, tau, u, T)
        torch.cuda.synchronize()
        t_is = time.perf_counter() - t0
        dB = est["B"] - Bref
        ddg = est["res"]["dG"] - dref
        n_is = int(est["n_scanned"].sum())
        fin = np.isfinite(dB)
        is_runs[name] = {
            "configs_scanned": n_is, "configs_total": int(bt.n_cfg),
            "cost_fine_equivalents": n_is + float(sum(extra_cfg[b.cfg_off[l]:b.cfg_off[l + 1]].sum() for l in test_l)),
            "fallback_ligands": int(est["fallback"].sum()),
            "fallback_rule": "predicted weight outside the exact stratum > 0.5 (decided before the draw)",
            "max_sampled_share": float(np.max(est["share"])),
            "rms_dB_kcal_mol": float(np.sqrt(np.mean(dB[fin] ** 2))) if np.any(fin) else None,
            "max_abs_dB_kcal_mol": float(np.max(np.abs(dB[fin]))) if np.any(fin) else None,
            "n_infinite_dB": int(np.count_nonzero(~fin)),
            "rms_ddG_kcal_mol": float(np.sqrt(np.mean(ddg ** 2))),
            "seconds_is_path_fine_only": t_is,
            "seconds_exhaustive_fine_same_ligands": t_f * bt.n_cfg / b.n_cfg}
        log(f"10% IS run ({name}): {n_is} of {bt.n_cfg} scanned, {is_runs[name]['fallback_ligands']} fallbacks, "
            f"RMS dB {is_runs[name]['rms_dB_kcal_mol']}, max {is_runs[name]['max_abs_dB_kcal_mol']}")
    return {
        "workload": f"batched: {len(w.ligands)} ligands x {S} snapshots, {b.n_cfg} configurations, "
                    f"101 training / {len(test_l)} held-out ligands (seeded split)",
        "criterion": "RMS over replicates of (B_hat - B_exhaustive) <= 0.1 kcal/mol in every snapshot; "
                     "cost = distinct fine-scanned configurations (+ coarse pre-scan at its cost ratio)",
        "replicates": args.is_reps,
        "coarse_cost_ratio": rho,
        "coarse_receptors": args.is_coarse,
        "cascade_fraction": args.is_cascade_frac if cascade else None,
        "coarse_spacing_factor": args.is_coarse_factor,
        "coarse_clash_mode": args.is_coarse_clash,
        "target": args.is_target,
        "split": "101 training ligands = 81 fitted + 20 validation (temperature, epochs); 40 held out",
        "mixture_alpha": alpha,
        "mixture_tau_nats": {k: v[0] for k, v in tau_of.items()},
        "exact_share": {k: v[1] for k, v in tau_of.items()},
        "epochs_kept": epochs_of,
        "validation_mean_fraction": val_of,
        "train_seconds": t_train,
        "network_throughput": mlp,
        "median_plain_over": {"net_scan": med("net_scan"), "net_cfg": med("net_cfg"), "coarse": med("coarse"),
                              "uniform": med("uniform")},
        "median_fraction_of_pool": {k: float(np.median([r[k] / r["n_cfg"] for r in per]))
                                    for k in ("plain", "net_scan", "net_cfg", "coarse", "uniform")},
        "gain_test": "uniform: the net_scan plan (temperature, exact share) with a uniform proposal in place "
                     "of the network",
        "is_run_10pct": is_runs["net_scan"],
        "is_run_10pct_coarse": is_runs["coarse"],
        "per_ligand": per,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--chunk", type=int, default=0, help="configurations per chunk (0 = library default)")
    ap.add_argument("--energy-direct", type=int, default=-1, help="energy xy transforms: 0 FFT pass, 1 in the z kernel, 2 direct in the forward pass (default: autotuned)")
    ap.add_argument("--snap-pass", type=int, default=0, help="snapshots per z pass (0 = library default)")
    ap.add_argument("--fused", type=int, default=-1,
                    help="0: plane path; 1: fused path, energy planes from the forward pass; 2: fused path, "
                         "z inputs formed in the z kernel (default: autotuned)")
    ap.add_argument("--clash-stream", type=int, default=-1,
                    help="1 uses a second stream (fused path: the clash test of the next item; plane path: the "
                         "inverse of one z pass beside the next), 0 one stream (default: autotuned, or the library "
                         "default with --fused)")
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "c6"],
                    help="c2: the 8000-configuration T4L-sized scan (the metric's workload); "
                         "c3: 141 ligands x 10 receptor snapshots (batched); "
                         "c6: the c2 ligand on the 62 A whole-surface grid (248^3 in a 256^3 FFT)")
    ap.add_argument("--n-rot", type=int, default=125, help="c6 only: rotations per conformer (8 conformers)")
    ap.add_argument("--cfg-scale", type=float, default=0.1, help="c3 only: scale of the 200-2000 configurations per ligand")
    ap.add_argument("--no-autotune", action="store_true", help="skip the schedule autotuner (setup, untimed)")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-is", action="store_true", help="skip the configurations-needed measurement")
    ap.add_argument("--no-batched", action="store_true", help="skip the timed batched (141-ligand) scan")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the pose-resampling and grid-spacing measurements after the timed steps "
                         "(for profiler runs that should hold the timed kernels only)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 1 GiB device copy before timing (counter calibration)")
    ap.add_argument("--is-only", action="store_true", help="only the configurations-needed measurement")
    ap.add_argument("--is-reps", type=int, default=200, help="replicates per budget (configurations needed)")
    ap.add_argument("--is-epochs", type=int, default=20)
    ap.add_argument("--is-coarse-factor", type=int, default=2,
                    help="coarse spacing = factor x the fine spacing (2: 64-point FFT, 4: 32-point)")
    ap.add_argument("--is-target", default="snapmax", choices=["snapmax", "sum"],
                    help="training target: largest per-snapshot relative log weight, or the log of the "
                         "snapshot-weighted sum")
    ap.add_argument("--is-detail", default="", help="write per-ligand configurations-needed results here (JSON)")
    ap.add_argument("--is-coarse", default="cascade", choices=["mean", "all", "half", "first", "cascade"],
                    help="coarse pre-scan receptors: one at the snapshots' mean coordinates, every snapshot, "
                         "every other snapshot, the first snapshot, or a cascade (default: the mean receptor for "
                         "every configuration, then every snapshot for each ligand's top --is-cascade-frac by that "
                         "score)")
    ap.add_argument("--is-cascade-frac", type=float, default=0.4)
    ap.add_argument("--is-exact-shares", default="0.5,0.75,0.9",
                    help="candidate shares of the budget scanned exactly (the top of the proposal), chosen with the "
                         "mixture temperature on the validation ligands")
    ap.add_argument("--is-coarse-clash", default="cap", choices=["occ", "cap"],
                    help="clash handling of the coarse pre-scan: capped repulsion (one inverse channel; default) "
                         "or occupancy exclusion (as the fine scan)")
    args = ap.parse_args()
    try:
        args.is_exact_shares = [float(x) for x in args.is_exact_shares.split(",")]
    except ValueError:
        args.is_exact_shares = []
    if not args.is_exact_shares or any(not 0.0 <= x < 1.0 for x in args.is_exact_shares):
        ap.error("--is-exact-shares: comma-separated fractions in [0, 1)")
    args.is_coarse_snapshots = {"mean": "mean", "all": None, "half": "half", "first": [0],
                                "cascade": None}[args.is_coarse]
    if args.is_coarse_factor not in (2, 4):
        ap.error("--is-coarse-factor must be 2 or 4")
    if args.gpus != 1:
        print(f"bench.py: this implementation runs on one GPU; --gpus {args.gpus} is not supported "
              "(the scan would shard by ligand, snapshot and configuration chunk)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1708_07045_amd as fd
    from workload import synth

    if args.is_only:
        cn = configs_needed(args)
        if args.is_detail:
            with open(args.is_detail, "w") as f:
                json.dump(cn, f, indent=1)
        print(json.dumps({"metric": "configs needed for BPMF ±0.1 kcal/mol, MLP vs plain",
                          "configs_needed": {k: v for k, v in cn.items() if k != "per_ligand"}}), flush=True)
        return

    if args.workload == "c2":
        w = synth.config2()
    elif args.workload == "c3":
        w = synth.config3(cfg_scale=args.cfg_scale)
    else:
        w = synth.config6(n_rot=args.n_rot)
    n_snap = w.receptor.n_snap
    log(f"workload: {w.name}; {len(w.ligands)} ligands, {w.n_cfg_total} configurations, {n_snap} snapshots")
    ctx = fd.FFTDG.from_workload(w)
    if args.chunk:
        ctx.set_tuning(configs_per_chunk=args.chunk)
    if args.energy_direct in (0, 1, 2):
        ctx.set_tuning(energy_xy_direct=args.energy_direct)
    if args.snap_pass:
        ctx.set_tuning(snapshots_per_pass=args.snap_pass)
    if args.fused in (0, 1, 2):
        ctx.set_tuning(fused=args.fused)
    if args.clash_stream in (0, 1):
        ctx.set_tuning(clash_stream=args.clash_stream)
    gl, ol = [], []
    for sn in range(n_snap):
        g, o = ctx.receptor_grids(w.receptor.xyz[sn], w.receptor.q, w.receptor.sigma, w.receptor.eps)
        gl.append(g)
        ol.append(o)
    grids, occ = torch.stack(gl).contiguous(), torch.stack(ol).contiguous()
    del gl, ol
    batch = fd.Batch(w.ligands)
    ctx.set_receptors(grids, occ, w.receptor.weights)
    out = ctx.alloc_partials(batch)
    torch.cuda.synchronize()
    autotuned = None
    if not args.no_autotune and not (args.chunk or args.energy_direct in (0, 1, 2) or args.snap_pass or
                                     args.fused in (0, 1, 2) or args.clash_stream in (0, 1)):
        t0 = time.perf_counter()
        # the T4L-sized workload is tuned on all of its 8000 configurations
        # (a small sample leaves chunk sizes within noise of each other)
        tun, ms = ctx.autotune(batch, w.T, max_cfgs=8192 if args.workload == "c2" else 2048)
        autotuned = {"choice": tun, "ms_per_cfg_snapshot": ms, "seconds": time.perf_counter() - t0}
        log(f"autotuned schedule {tun} ({ms * 1e3:.2f} us per configuration and snapshot on the sample)")

    copy_gbps = copy_bandwidth()
    log(f"device copy: {copy_gbps:.0f} GB/s (read + write)")
    if args.copy_calibration:
        copy_calibration()
    result = {}

    scan_ev = []

    def step(timed_scan=False):
        ctx.set_receptors(grids, occ, w.receptor.weights)
        if timed_scan:  # HIP events on the library's stream (torch's current stream) around the scan
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
        ctx.scan(batch, w.T, out)
        if timed_scan:
            e1.record()
            scan_ev.append((e0, e1))
        B, res = ctx.reduce(batch, out, w.T)
        result["B"], result["res"] = B, res

    for i in range(args.warmup):
        step()
        log(f"warmup step {i + 1}/{args.warmup} done")
    # Timed steps with profiling off: the schedule as tuned (a captured
    # graph replays when the autotuner chose one).  Each step ends in the
    # reduce, which synchronizes, so per-step host times are step times.
    torch.cuda.synchronize()
    step_ms = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        step(timed_scan=True)
        step_ms.append((time.perf_counter() - ts) * 1e3)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    scan_ms = [a.elapsed_time(b) for a, b in scan_ev]
    log(f"timed {args.steps} steps in {t1 - t0:.3f}s")
    # Separate profiled steps for the per-kernel table: HIP events around
    # every launch on the library's stream (graphs are not replayed while
    # profiling, so these steps run the same kernels eagerly).
    n_prof = max(2, min(args.steps, 5))
    ctx.profile(True)
    tp0 = time.perf_counter()
    for i in range(n_prof):
        step()
    torch.cuda.synchronize()
    tp1 = time.perf_counter()
    prof = ctx.profile_read()
    ctx.profile(False)
    log(f"profiled {n_prof} more steps in {tp1 - tp0:.3f}s")

    ms_step = (t1 - t0) * 1e3 / args.steps
    n_cfg = batch.n_cfg
    cfg_s = n_cfg / (ms_step / 1e3)
    P = ctx.partials_numpy(out, n_snap, n_cfg)[0]
    n_valid = int(P["n_valid"].sum())
    tun = ctx.get_tuning()
    fused = tun.get("fused", 0) != 0

    kernels = {}
    for name, (ms, n, b) in prof.items():
        if n == 0:
            continue
        kernels[name] = {"ms_per_step": ms / n_prof, "launches_per_step": n / n_prof,
                         "avg_launch_us": 1e3 * ms / n, "alg_GBps": (b / 1e9) / (ms / 1e3) if ms > 0 else None,
                         "alg_bytes_per_launch": b / n}
    boxes = ctx.boxes(batch)
    pb = pruned_bytes_per_cfg({"box_z": boxes[:, 2], "V_z": np.maximum(w.n_rec - boxes[:, 2], 0)}, w.n_fft,
                              w.clash_mode == "occ", tun["configs_per_chunk"])
    # Roofline.  The unit is one scan (every configuration of the batch
    # against every snapshot): on the fused path no single kernel moves the
    # method's data and the clash test runs on a second stream beside the z
    # pass, so the pruned-transform model's algorithmic bytes per
    # configuration-snapshot scan are rated against the scan's GPU time, HIP events on the
    # library's stream around each timed scan (median).
    scan_med = float(np.median(scan_ms))
    scans = n_cfg * n_snap
    achieved = pb * scans / (scan_med * 1e-3) / 1e9
    traffic = None
    if args.workload == "c2":
        per_cfg = recorded_traffic(tun)
        if per_cfg is not None:
            traffic = per_cfg * n_cfg   # bytes per scan
    chunk_kernels = [k for k in ("lig_runs", "lig_fwd_xy", "clash", "zprod", "inv_xy_lse", "merge") if k in kernels]
    seq_ms = sum(kernels[k]["ms_per_step"] for k in chunk_kernels)
    # the z pass alone: bound by vector-ALU issue (VALU busy 0.9 and more in
    # the counter runs); its flops against the FP32 vector peaks and its own
    # algorithmic bytes against HBM
    zk = None
    if "zprod" in kernels:
        kd = kernels["zprod"]
        occ_mode = w.clash_mode == "occ"
        n_in, n_out = (3, 1) if (fused or not occ_mode) else (4, 2)
        fl = zpass_flops(w.n_fft, n_in, n_out, occ_mode and not fused, n_cfg, n_snap,
                         tun["snapshots_per_pass"] if (tun["snapshots_per_pass"] > 0 and not fused) else 1)
        fl_launch = fl * n_prof / prof["zprod"][1]
        tf = fl_launch / (kd["avg_launch_us"] * 1e-6) / 1e12
        zk = {"kernel": "zprod", "avg_launch_us": kd["avg_launch_us"],
              "alu": {"achieved": tf, "unit": "TFLOP/s", "alg_flops_per_launch": fl_launch,
                      "peak": VALU_FP32_PEAK_TFLOPS, "frac": tf / VALU_FP32_PEAK_TFLOPS,
                      "peak_nonpacked_fp32": VALU_FP32_NONPACKED_TFLOPS,
                      "frac_of_nonpacked": tf / VALU_FP32_NONPACKED_TFLOPS},
              "hbm": {"achieved": kd["alg_GBps"], "unit": "GB/s", "frac": kd["alg_GBps"] / HBM_PEAK_GBS,
                      "alg_bytes_per_launch": kd["alg_bytes_per_launch"]}}
    roof = {"bound": "hbm", "kernel": "scan: " + " + ".join(chunk_kernels) + (
                " (clash test on a second stream)" if tun.get("clash_stream") and fused else ""),
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "per_unit": "pruned-transform algorithmic bytes per configuration-snapshot scan (pruned_bytes_per_cfg) x scans",
            "alg_bytes_per_launch": pb * scans, "avg_launch_us": 1e3 * scan_med,
            "scan_ms": scan_ms, "copy_GBps": copy_gbps, "frac_of_copy": achieved / copy_gbps,
            "profiled_kernels_sum_ms": seq_ms,
            "note": "one launch = one scan; its kernels' profiled times (one stream, no overlap) sum to "
                    "profiled_kernels_sum_ms",
            "z_kernel": zk}
    # whole path: algorithmic bytes of all scan kernels per configuration
    path_bytes = sum(prof[k][2] for k in ("lig_fwd_xy", "zprod", "inv_xy_lse", "merge", "lig_runs", "clash")
                     if k in prof) / n_prof
    rec = {
        "metric": METRIC,
        "value": cfg_s,
        "unit": "configs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "ms_per_step_median": float(np.median(step_ms)),
        "ms_per_step_min": float(np.min(step_ms)),
        "profiled_ms_per_step": (tp1 - tp0) * 1e3 / n_prof,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": ("T4L-sized plain scan: 2600-atom cavity receptor, 96^3 grid @ 0.25 A -> 128^3 FFT, "
                                "occupancy clash mode, 25-atom ligand x 8 conformers x 1000 rotations, 300 K")
                   if args.workload == "c2" else
                   (f"batched: {len(w.ligands)} ligands of 8-40 atoms, {n_cfg} configurations "
                    f"(200-2000 per ligand x {args.cfg_scale}), {n_snap} jittered receptor snapshots, 128^3 FFT, "
                    "occupancy clash mode, 300 K") if args.workload == "c3" else
                   (f"whole-surface scan: 2600-atom cavity receptor, 248^3 grid @ 0.25 A (62 A) -> 256^3 FFT, "
                    f"occupancy clash mode, 25-atom ligand x 8 conformers x {args.n_rot} rotations, 300 K"),
                   "n_cfg": n_cfg, "n_fft": w.n_fft, "n_rec": w.n_rec, "clash_mode": w.clash_mode,
                   "n_snap": n_snap, "parallelism": "single GPU", "tuning": ctx.get_tuning(),
                   "autotune": autotuned},
        "scans_per_s": cfg_s * n_snap,
        "translations_per_s": cfg_s * n_snap * n_valid / n_cfg,
        "evaluated_translations_per_s": cfg_s * n_snap * w.n_fft ** 3,
        "path_alg_bytes_per_cfg": path_bytes / n_cfg,
        "path_alg_GBps": path_bytes / (ms_step / 1e3) / 1e9,
        "path_frac_of_peak": path_bytes / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS,
        "path_frac_of_copy": path_bytes / (ms_step / 1e3) / 1e9 / copy_gbps,
        "pruned_bytes_per_cfg": pb,
        "pruned_GBps": pb * cfg_s * n_snap / 1e9,
        "pruned_frac_of_peak": pb * cfg_s * n_snap / 1e9 / HBM_PEAK_GBS,
        "roofline": roof,
        "kernels": kernels,
        "precision": precision_vs_oracle(args, result),
        "pose_resampling": pose_resampling(ctx, batch, out, w.T)
        if args.workload == "c2" and not args.no_extras else None,
        "spacing_study": spacing_study(w, ctx, batch, out) if args.workload == "c2" and not args.no_extras else None,
        "bpmf_kcal_mol": float(result["B"][0, 0]),
        "dG_kcal_mol": float(result["res"]["dG"][0]),
        "psi_min_kcal_mol": float(result["res"]["psi_min"][0]),
    }
    if args.workload != "c2":
        rec["metric"] = METRIC + (" [batched workload; not the headline line]" if args.workload == "c3"
                                  else " [whole-surface workload; not the headline line]")
        rec["dG_kcal_mol_per_ligand"] = [float(x) for x in result["res"]["dG"]]
        args.no_cpu_baseline = True
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        rec["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
        log("cpu baseline (FFT method, scipy) ...")
        rec["cpu_fft_baseline"] = cpu_fft_baseline(w, args.cpu_budget * 2 / 3)
        rec["paper_cpu_times"] = PAPER_CPU_TIMES
    else:
        rec["cpu_baseline"] = None
    if args.workload == "c2" and not (args.no_is and args.no_batched):
        del ctx, out, grids, occ
        torch.cuda.empty_cache()
    if args.workload == "c2" and not args.no_batched:
        rec["batched"] = batched_timing()
        torch.cuda.empty_cache()
    if args.workload == "c2" and not args.no_is:
        cn = configs_needed(args, rec["batched"]["tuning"] if rec.get("batched") else None)
        rec["configs_needed"] = {k: v for k, v in cn.items() if k != "per_ligand"}
        rec["configs_needed_median_plain_over_learned"] = cn["median_plain_over"]["net_scan"]
        if args.is_detail:
            with open(args.is_detail, "w") as f:
                json.dump(cn, f, indent=1)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
