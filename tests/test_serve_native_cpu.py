"""The serving engine's C ABI on the host (no GPU): struct layouts agree between
include/fsp_serve.h and the binding (checked by compiling the header with gcc),
arguments are validated before any device work, and the report arithmetic."""
import ctypes
import os
import subprocess

import pytest

from paper_2405_02603_amd import _lib
from paper_2405_02603_amd.serve_native import percentile, summarize

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROBE = r"""
#include <stdio.h>
#include <stddef.h>
#include "fsp_serve.h"
#define F(T, m) printf("%s.%s %zu\n", #T, #m, offsetof(T, m))
int main(void) {
  printf("fsp_request %zu\nfsp_request_result %zu\nfsp_server_stats %zu\n", sizeof(fsp_request),
         sizeof(fsp_request_result), sizeof(fsp_server_stats));
  F(fsp_request, t_arrival); F(fsp_request, n); F(fsp_request, greens); F(fsp_request, prec);
  F(fsp_request, lo); F(fsp_request, hi); F(fsp_request, alpha); F(fsp_request, rho); F(fsp_request, phi);
  F(fsp_request_result, t_arrival); F(fsp_request_result, t_admit); F(fsp_request_result, t_done);
  F(fsp_request_result, t_seen); F(fsp_request_result, refresh_ms); F(fsp_request_result, status);
  F(fsp_request_result, slot); F(fsp_request_result, launch_size);
  F(fsp_server_stats, budget_bytes); F(fsp_server_stats, peak_held_bytes); F(fsp_server_stats, held_bytes);
  F(fsp_server_stats, launches); F(fsp_server_stats, refreshes); F(fsp_server_stats, evictions);
  F(fsp_server_stats, rejected); F(fsp_server_stats, refresh_ms_total);
  return 0;
}
"""


def test_struct_layouts_match_the_header(tmp_path):
    src = tmp_path / "probe.c"
    src.write_text(PROBE)
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                         check=True).stdout.splitlines())
    for cname, cls in (("fsp_request", _lib.Request), ("fsp_request_result", _lib.RequestResult),
                       ("fsp_server_stats", _lib.ServerStats)):
        assert int(out[cname]) == ctypes.sizeof(cls), cname
        for field, _ in cls._fields_:
            assert int(out[f"{cname}.{field}"]) == getattr(cls, field).offset, (cname, field)


def test_server_arguments_are_checked_on_the_host():
    lib = _lib.load()
    h = ctypes.c_void_p()
    assert lib.fsp_server_create(0, 4, 4, ctypes.byref(h)) == _lib.FSP_ERR_INVALID_ARG
    assert lib.fsp_server_create(1 << 20, 0, 4, ctypes.byref(h)) == _lib.FSP_ERR_INVALID_ARG
    assert lib.fsp_server_create(1 << 20, 4, 0, ctypes.byref(h)) == _lib.FSP_ERR_INVALID_ARG
    assert lib.fsp_server_create(1 << 20, 4, 4, None) == _lib.FSP_ERR_INVALID_ARG
    assert lib.fsp_server_run(None, 0, None, None, 1.0, 1.0) == _lib.FSP_ERR_INVALID_ARG
    assert lib.fsp_server_get_stats(None, None) == _lib.FSP_ERR_INVALID_ARG
    assert lib.fsp_server_destroy(None) == _lib.FSP_ERR_INVALID_ARG


def test_serve_exports():
    lib = _lib.load()
    text = open(os.path.join(ROOT, "include", "fsp_serve.h")).read()
    import re
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    decl = sorted(set(re.findall(r"\b(fsp_server_[a-z_]+)\s*\(", text)))
    assert decl == sorted(_lib.SERVE_EXPORTS)
    for name in decl:
        assert hasattr(lib, name)


def test_percentile():
    assert percentile([], 50) != percentile([], 50)  # NaN
    assert percentile([3.0], 99) == 3.0
    assert percentile([1.0, 2.0, 3.0, 4.0], 50) == 2.5
    assert percentile(list(range(101)), 99) == 99.0


def test_summarize_latency_throughput_and_refresh_share():
    res = [
        {"t_arrival": 0.0, "t_admit": 0.0, "t_done": 0.010, "t_seen": 0.0101, "refresh_ms": 4.0, "status": 0,
         "slot": 0, "launch_size": 1},
        {"t_arrival": 0.005, "t_admit": 0.006, "t_done": 0.011, "t_seen": 0.0112, "refresh_ms": 0.0, "status": 0,
         "slot": 1, "launch_size": 2},
        {"t_arrival": 0.006, "t_admit": 0.006, "t_done": 0.011, "t_seen": 0.0112, "refresh_ms": 0.0, "status": 0,
         "slot": 1, "launch_size": 2},
        {"t_arrival": 0.007, "t_admit": 0.0, "t_done": 0.0, "t_seen": 0.0, "refresh_ms": 0.0,
         "status": _lib.FSP_ERR_OUT_OF_MEMORY, "slot": -1, "launch_size": 0},
    ]
    rep = summarize(res)
    assert rep["done"] == 3 and rep["rejected"] == 1
    assert rep["p50_ms"] == pytest.approx(6.0)
    assert rep["solves_per_s"] == pytest.approx(3 / 0.011)
    assert rep["refreshed_requests"] == 1
    assert rep["refresh_share"] == pytest.approx(4.0 / (10.0 + 6.0 + 5.0))
    assert rep["mean_launch_size"] == pytest.approx(5 / 3)
