"""Bookkeeping of the benchmark line (CPU only): the z pass's algorithmic
flops, the FP32 vector peak it is rated against, and the recorded HBM
traffic, which applies only while the kernel sources match."""
import importlib.util
import math
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_vector_peak_from_unit_counts(bench):
    # 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2 (packed FP32) x 2.4 GHz
    assert bench.VALU_FP32_PEAK_TFLOPS == pytest.approx(157.2864)
    assert bench.VALU_FP32_NONPACKED_TFLOPS == pytest.approx(78.6432)


def test_zpass_flops_count(bench):
    N = 128
    pencils = N * (N // 2 + 1)
    t = 5 * N * math.log2(N)
    # plane path, occupancy mode: 4 forward + 2 inverse transforms, 3 x 8 + 6 flops per point
    want = pencils * (6 * t + N * 30)
    assert bench.zpass_flops(N, 4, 2, True, 1, 1, 1) == pytest.approx(want)
    assert bench.zpass_flops(N, 4, 2, True, 1, 1, 1) == pytest.approx(255.5904e6)
    # energy channels only (cap mode, or the fused path): 3 forward + 1 inverse, 3 x 8 flops per point
    assert bench.zpass_flops(N, 3, 1, False, 1, 1, 1) == pytest.approx(pencils * (4 * t + N * 24))
    # linear in configurations; forward transforms shared by the snapshots of a pass
    assert bench.zpass_flops(N, 4, 2, True, 10, 1, 1) == pytest.approx(10 * want)
    one_pass = bench.zpass_flops(N, 4, 2, True, 1, 4, 4)
    per_snap = bench.zpass_flops(N, 4, 2, True, 1, 4, 1)
    assert one_pass == pytest.approx(per_snap - 3 * pencils * 4 * t)


def test_pruned_bytes_per_configuration(bench):
    """16 N (N/2+1) (n_in L_z + n_out V_z) + 8 S_h n_rc / B_rc, worked by hand
    for one configuration: N = 128, box_z = 37 (L_z = 38), V_z = 59,
    occupancy mode (n_in = n_rc = 4, n_out = 2), B_rc = 16."""
    nh = 128 * 65
    want = 16 * nh * (4 * 38 + 2 * 59) + 8 * 128 * nh * 4 / 16
    assert want == pytest.approx(35_942_400.0 + 2_129_920.0)
    got = bench.pruned_bytes_per_cfg({"box_z": [37], "V_z": [59]}, 128, True, 16)
    assert got == pytest.approx(want)
    # cap mode: 3 input channels, 1 output; the mean over configurations
    two = bench.pruned_bytes_per_cfg({"box_z": [37, 41], "V_z": [59, 55]}, 128, False, 16)
    a = 16 * nh * (3 * 38 + 59) + 8 * 128 * nh * 3 / 16
    b = 16 * nh * (3 * 42 + 55) + 8 * 128 * nh * 3 / 16
    assert two == pytest.approx((a + b) / 2)


def test_recorded_traffic_follows_sources_and_schedule(bench, tmp_path, monkeypatch):
    prof = tmp_path / "traffic.md"
    digest = bench.kernel_source_digest()
    prof.write_text("\n".join([
        "# summary", "", f"- hbm_bytes_per_cfg: 1234.5", "- configs_per_chunk: 512", "- energy_xy_direct: 2",
        f"- kernel_source_sha256: `{digest}`", ""]))
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(prof))
    tun = {"configs_per_chunk": 256, "energy_xy_direct": 2, "fused": 0}
    assert bench.recorded_traffic(tun) == pytest.approx(1234.5)
    assert bench.recorded_traffic({"configs_per_chunk": 64, "energy_xy_direct": 2, "fused": 0}) is None
    assert bench.recorded_traffic({"configs_per_chunk": 512, "energy_xy_direct": 0, "fused": 0}) is None
    assert bench.recorded_traffic({"configs_per_chunk": 512, "energy_xy_direct": 2, "fused": 1}) is None
    prof.write_text(prof.read_text().replace(digest, "0" * 64))
    assert bench.recorded_traffic(tun) is None


def test_committed_traffic_profile_is_parsable(bench):
    rec = {}
    for line in open(bench.TRAFFIC_PROFILE):
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            rec[k.strip()] = v.strip().strip("`")
    assert float(rec["hbm_bytes_per_cfg"]) > 1e6
    assert len(rec["kernel_source_sha256"]) == 64


def test_more_than_one_gpu_is_refused_before_any_work():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and not r.stdout


@pytest.mark.parametrize("shares", ["1.0", "0.5,-0.1", ""])
def test_exact_shares_outside_unit_interval_are_rejected(shares):
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--is-exact-shares", shares],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "--is-exact-shares" in r.stderr and not r.stdout


def test_traffic_digest_covers_every_scan_kernel_source(bench):
    """The recorded HBM traffic is trusted only while the scan kernels'
    sources are unchanged, so the digest must cover every HIP source and
    header of the library except the network's."""
    csrc = os.path.join(ROOT, "paper_1708_07045_amd", "csrc")
    kernel_files = {f for f in os.listdir(csrc) if f.endswith((".hip", ".hpp"))} - {"mlp.hip"}
    assert kernel_files == set(bench.KERNEL_SOURCES)
