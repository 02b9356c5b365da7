"""Host-side logic of bench.py (no GPU): algorithmic bytes per launch, the
names and validity checks of the committed counter summaries, and the
one-GPU guard."""
import json
import os
import subprocess
import sys

import bench
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_algorithmic_bytes_channel():
    case = W.channel_case()
    n = 384 * 192 * 192
    fluid = 384 * 190 * 192  # walls at y = 0 and y = ny - 1
    assert bench.fluid_nodes(case) == fluid
    assert bench.algorithmic_bytes(case, 0) == 10 * 4 * (n + fluid) == 1126563840
    assert bench.algorithmic_bytes(case, 1) == bench.algorithmic_bytes(case, 0) // 2
    assert bench.algorithmic_bytes(case, 2) == bench.algorithmic_bytes(case, 1)


def test_algorithmic_bytes_d2q9_six_fields():
    case = W.channel2d_case()
    assert case.lattice == 9
    n = case.nx * case.ny
    assert bench.algorithmic_bytes(case, 0) == 6 * 4 * (n + bench.fluid_nodes(case))


def test_counter_summary_names_and_checks():
    p0 = bench._pmc_path("update_tiled", "channel_384x192x192", 0)
    p1 = bench._pmc_path("update_tiled", "channel_512x256x256", 1)
    assert os.path.basename(p0) == "pmc_update_tiled_channel_384x192x192.json"
    assert os.path.basename(p1) == "pmc_update_tiled_channel_512x256x256_fp16.json"
    rec = json.load(open(p0))
    assert rec["storage"] == 0
    scaled = (rec["fetch_kib_per_dispatch"] * rec["copy_fetch_factor"] +
              rec["write_kib_per_dispatch"] * rec["copy_write_factor"]) * 1024.0
    assert abs(scaled - rec["hbm_bytes_per_launch"]) < 1e-6 * scaled
    # reported only while the kernel sources are those the counters were taken on
    want = rec["hbm_bytes_per_launch"] if rec["source_hash"] == bench._source_hash() else None
    assert bench.load_traffic("update_tiled", "channel_384x192x192", 0) == want
    # FETCH_SIZE counted half the bytes of a plain copy, WRITE_SIZE all of them
    assert abs(rec["copy_fetch_factor"] - 2.0) < 1e-3 and abs(rec["copy_write_factor"] - 1.0) < 1e-3
    assert 1.0 <= rec["traffic_over_algorithmic"] < 1.2
    # no summary for another storage of the same workload
    assert bench.load_traffic("update_tiled", "channel_384x192x192", 2) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_valu_view_of_the_roofline(monkeypatch, tmp_path):
    """A counter summary that carries SQ_INSTS_VALU adds the VALU view:
    thread-level instructions per second against the non-packed FP32 issue
    ceiling (256 CUs x 64 lanes x 2.4 GHz), only on the current sources."""
    case = W.channel_case(nx=512, ny=256, nz=256)
    path = tmp_path / "pmc.json"
    rec = {"storage": 1, "source_hash": bench._source_hash(), "hbm_bytes_per_launch": 1.4e9,
           "valu_insts_per_dispatch": 166969448.0}
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "_pmc_path", lambda k, c, s: str(path))
    roof = bench.kernel_roofline(case, 1, 0.4358, "update_tiled", 5900.0)
    v = roof["valu"]
    assert v["bound"] == "alu" and abs(v["peak"] - 39.32) < 0.01
    lane_ops = 166969448.0 * 64 / 0.4358e-3
    assert abs(v["achieved"] - lane_ops / 1e12) < 0.01
    assert abs(v["frac"] - lane_ops / (256 * 64 * 2.4e9)) < 1e-4
    assert abs(v["insts_per_node"] - 166969448.0 * 64 / case.nodes) < 0.1
    rec["source_hash"] = "0" * 16
    path.write_text(json.dumps(rec))
    assert "valu" not in bench.kernel_roofline(case, 1, 0.4358, "update_tiled", 5900.0)
