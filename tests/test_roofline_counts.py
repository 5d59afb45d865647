"""The roofline's algorithmic flops per rollout-step come from a host build of the device
step on a counting number type (paper_2409_10469_amd/csrc/flop_count.cpp): this builds it
with g++ (CPU) and requires the per-scene counts to equal the constants the bench uses."""
import os
import shutil
import subprocess

import pytest

from paper_2409_10469_amd import roofline

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CS = os.path.join(ROOT, "paper_2409_10469_amd", "csrc")


def test_flop_counts_match_the_counting_build(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ is not available")
    shim = tmp_path / "hip"
    shim.mkdir()
    # the counting build reads the device header through a host stand-in of the runtime
    (shim / "hip_runtime.h").write_text('#include "flop_count_stub.h"\n')
    exe = tmp_path / "flop_count"
    r = subprocess.run(["g++", "-O1", "-std=c++17", "-I", str(tmp_path), "-I", CS, "-I", os.path.join(ROOT, "include"),
                        os.path.join(CS, "flop_count.cpp"), "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    for scene, want in roofline.FLOPS_DYN_PER_STEP.items():
        out = subprocess.run([str(exe), str(scene)], capture_output=True, text=True, check=True).stdout
        line = [l for l in out.splitlines() if l.startswith("ALGORITHMIC")][-1]
        assert int(line.split()[-1]) == want, (scene, line)
