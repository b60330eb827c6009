"""Host logic of bench.py (no GPU): the byte models the roofline divides by, the
refusal of multi-GPU runs, and the lookup of the committed counter summary."""
import json
import os

import pytest

import bench


@pytest.mark.parametrize("n", [64, 256, 512])
@pytest.mark.parametrize("rb", [4, 8])
def test_pass_bytes_sum_to_the_five_pass_model(n, rb):
    """(2 N^3 + 24 (N+1) N^2 + (N+1)^3) s: the five passes' reads and writes."""
    pb = bench.pass_bytes((n, n, n), rb)
    assert sum(pb) == (2 * n ** 3 + 24 * (n + 1) * n * n + (n + 1) ** 3) * rb
    # P1 and P5 mirror each other, so do P2 and P4
    assert pb[0] == pb[4] and pb[1] == pb[3]


def test_pass_bytes_of_an_anisotropic_grid():
    n0, n1, n2, rb = 32, 64, 48, 4
    half1 = n0 * n1 * (n2 + 1) * 2 * rb
    half2 = 2 * half1
    pb = bench.pass_bytes((n0, n1, n2), rb)
    assert pb[0] == n0 * n1 * n2 * rb + half1
    assert pb[2] == 2 * half2 + (n0 + 1) * (n1 + 1) * (n2 + 1) * rb


def test_gradient_bytes_read_the_spectrum_once():
    n, rb = 256, 4
    pb = bench.pass_bytes((n, n, n), rb)
    half2 = n * 2 * n * (n + 1) * 2 * rb
    octant = (n + 1) ** 3 * rb
    g = bench.grad_bytes((n, n, n), rb)
    assert g == pb[0] + pb[1] + half2 + 4 * (half2 + octant) + 4 * (pb[3] + pb[4])
    # against four separate solves' axis-0 passes: three reads of the spectrum saved
    assert pb[0] + pb[1] + 4 * (pb[2] + pb[3] + pb[4]) - g == 3 * half2


def test_more_than_one_gpu_is_refused_with_a_message(capsys):
    assert bench.main(["--gpus", "2"]) == 2
    line = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    assert "error" in line and line["n_gpus"] == 2


def test_workloads_parse():
    for w in ("single", "batch", "serve", "shard"):
        assert bench.parse(["--workload", w]).workload == w
    a = bench.parse([])
    assert a.gpus == 1 and a.n == 256 and a.greens == "vico_dct"


def test_traffic_lookup_follows_the_source_digest():
    """The committed summary is used only while the kernel sources match its digest."""
    d = bench.source_digest()
    assert len(d) == 16 and d == bench.source_digest()
    with open(bench.TRAFFIC_FILE) as fh:
        src = [ln.split()[1] for ln in fh if ln.startswith("source ")]
    t = bench.measured_traffic("vico_dct", 256, "f32", 2, 0)
    if src and src[0] == d:
        algo = bench.pass_bytes((256, 256, 256), 4)[2]
        assert isinstance(t, int) and algo <= t <= 1.1 * algo
    else:
        assert t is None
    assert bench.measured_traffic("vico_dct", 256, "f32", 2, 7) is None
    assert os.path.isfile(bench.TRAFFIC_FILE)
