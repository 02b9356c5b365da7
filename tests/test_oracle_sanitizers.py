"""The FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer:
tests/sanitize_oracle.c compiles the oracle source into a small driver that
calls every exported entry point on small grids (periodic, walls, inflow and
outflow ghosts, the sponge profile, D3Q27 / D3Q19 / D2Q9, orders 2 and 3,
forward, adjoint, JVP and rollout gradients); any out-of-bounds access, leak
or undefined operation aborts it."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_oracle_is_clean_under_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "sanitize_oracle")
    cmd = ["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-fopenmp", "-std=c11", os.path.join(HERE, "sanitize_oracle.c"), "-o", exe, "-lm"]
    build = subprocess.run(cmd, capture_output=True, text=True)
    if build.returncode != 0 and "sanitize" in build.stderr:
        pytest.skip("the compiler has no sanitizer runtime: " + build.stderr[-200:])
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, run.stdout[-2000:] + run.stderr[-4000:]
    assert "sanitizer run done, rc 0" in run.stdout
