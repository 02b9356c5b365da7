"""Host-side work list of the tiled update (no GPU): compiled from the
library's own header as host code and run on representative grids (the
channel, cube, jet and paper-jet tile counts, tiny and maximum grids, a
small resident count).  Every (tile column, plane) must be covered exactly
once and the per-block cost must stay within 5 % of the balanced ideal
(total planes / blocks + 2 halo planes)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def schedule_lines(tmp_path_factory):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc) and not shutil.which("hipcc"):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("sched") / "sched_check")
    subprocess.check_call([hipcc, "--cuda-host-only", "-x", "hip", "-std=c++20", "-O1",
                           "-I", os.path.join(ROOT, "paper_2401_17074_amd", "csrc"),
                           os.path.join(ROOT, "tests", "schedule_check.cpp"), "-o", exe],
                          stderr=subprocess.DEVNULL)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout
    return [list(map(int, ln.split())) for ln in r.stdout.strip().splitlines()]


def test_every_plane_once_and_balanced(schedule_lines):
    assert len(schedule_lines) == 13
    for columns, nz, resident, tz, grid, nseg, cost, ideal, split, _ in schedule_lines:
        assert 1 <= tz <= 64 and 1 <= split <= 8 and grid % 8 == 0 and grid <= resident
        # within 5 % (plus one segment's halo planes) of the balanced ideal
        assert cost <= 1.05 * ideal + 2, (columns, nz, cost, ideal)


def test_channel_512x256x256_beats_whole_tile_rounds(schedule_lines):
    # 176 tile columns x 256 planes on 256 blocks: whole 64-plane tiles
    # alone need 3 rounds of 66 plane-steps
    row = [r for r in schedule_lines if r[:3] == [176, 256, 256]][0]
    assert row[6] <= 186 < 3 * 66


def test_odd_segment_followed_by_another(schedule_lines):
    # the 256 x 60 x 457 grid of the GPU parity test of the FP32 register-set
    # swap (20 tile columns): some block marches a segment of an odd number of
    # planes and then another one
    row = [r for r in schedule_lines if r[:3] == [20, 457, 256]][0]
    assert row[9] > 0
