"""The serving engine compiled for the CPU with AddressSanitizer and
UndefinedBehaviorSanitizer, against a stand-in HIP runtime (tests/engine_host):
device memory is tracked host memory, so a solve or precompute that would use
freed device memory is counted as a device fault.  The scenarios (a budget that
forces evictions, and 60 random mixes of sizes, kernels, precisions, boxes,
budgets, slots and fold limits) must run with no sanitizer report, no device
fault, the bytes held never above the budget, and every request done or (only
when it alone exceeds the budget) rejected.

This is the regression test of a fault found on the GPU: the engine picked an
idle workspace for a request and then, making room for that request, could
free that same workspace (and the host record of it) before launching."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_engine_under_sanitizers(tmp_path):
    # the engine source is compiled as plain C++ from a copy with a .cpp name
    src = tmp_path / "serve_engine.cpp"
    shutil.copy(os.path.join(ROOT, "paper_2405_02603_amd", "csrc", "serve_engine.hip"), src)
    exe = tmp_path / "drive"
    inc = ["-I", os.path.join(ROOT, "tests", "engine_host"), "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_2405_02603_amd", "csrc")]
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-DFSP_SERVER_ENABLED", *san, *inc, str(src),
           os.path.join(ROOT, "tests", "engine_host", "mock_device.cpp"),
           os.path.join(ROOT, "tests", "engine_host", "drive.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    out = r.stdout
    assert r.returncode == 0, out[-3000:] + r.stderr[-3000:]
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]
    vals = {}
    for line in out.splitlines():
        name, key, value = line.split()
        vals[(name, key)] = value
    assert vals[("all", "ok")] == "1"
    # the tight budget does evict, stays under the budget and finishes everything
    assert int(vals[("tight", "evictions")]) > 0
    assert int(vals[("tight", "done")]) == 12
    assert int(vals[("tight", "peak_held")]) <= int(vals[("tight", "budget")])
    assert all(vals[(f"random{t}", "faults")] == "0" for t in range(60))
