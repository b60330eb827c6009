"""GPU: fsp_solve_static (the entry point that allocates nothing) against fsp_solve.

Both calls go through the C ABI on the same plan, input and stream; they run
the same kernels with the same schedule, so the results must be bit for bit
equal, and both must meet the oracle bar (float64 1e-12, float32 1e-6 relative
L2).  Two calls in a row on one GPU, the second on a smaller grid, check that
the shared static workspace carries nothing from one call into the next."""
import ctypes

import numpy as np
import pytest

import workloads as W

from gpu_util import reference, rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-6, "f64": 1e-12}


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _static(torch, lib, plan, rho, phi):
    from paper_2405_02603_amd import _lib
    stream = torch.cuda.current_stream()
    st = lib.fsp_solve_static(plan.handle, ctypes.c_void_p(rho.data_ptr()), ctypes.c_void_p(phi.data_ptr()),
                              ctypes.c_void_p(int(stream.cuda_stream)))
    assert st == _lib.FSP_OK, lib.fsp_last_error().decode()


def _case(torch, lib, n, lo, hi, kind, prec, seed, in_place=False, sched=None):
    from paper_2405_02603_amd import Plan
    dt = torch.float64 if prec == "f64" else torch.float32
    print(f"no-alloc case n={n} {kind} {prec} seed={seed} in_place={in_place} sched={sched}", flush=True)
    plan = Plan(n=n, lo=lo, hi=hi, greens=kind, prec=prec)
    if sched is not None:
        plan.schedule = sched
    host = W.random_field(n, seed)
    rho = to_dev(host, dt)
    ref = plan.solve(rho)                          # fsp_solve: the plan's own workspace
    if in_place:
        phi = rho.clone()
        _static(torch, lib, plan, phi, phi)
    else:
        phi = torch.full_like(rho, float("nan"))
        _static(torch, lib, plan, rho, phi)
    torch.cuda.synchronize()
    assert torch.equal(phi, ref), f"fsp_solve_static differs from fsp_solve at n={n} {prec}"
    assert rel_l2(to_host(phi), reference(host, kind, lo, hi)) <= TOL[prec]
    return plan


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_static_equals_solve_two_calls_second_smaller(torch_cuda, prec):
    from paper_2405_02603_amd import _lib
    lib = _lib.load()
    # first call: the largest grid the scratch holds in float64, a 3 * 2^a axis and a ragged tail
    _case(torch_cuda, lib, (128, 96, 48), (-1.0, -0.75, -0.5), (1.0, 0.75, 0.5), "vico_dct", prec, 11)
    _case(torch_cuda, lib, (24, 16, 32), (-0.5,) * 3, (0.5,) * 3, "hockney", prec, 12)


def test_static_in_place_and_largest(torch_cuda):
    from paper_2405_02603_amd import _lib
    lib = _lib.load()
    _case(torch_cuda, lib, (128, 128, 128), (-1.0,) * 3, (1.0,) * 3, "hockney", "f64", 13)
    _case(torch_cuda, lib, (16, 24, 12), (-0.5,) * 3, (0.5,) * 3, "vico_dct", "f32", 14, in_place=True)


def test_static_rejects_oversize_plan(torch_cuda):
    from paper_2405_02603_amd import Plan, _lib
    lib = _lib.load()
    plan = Plan(n=(256, 256, 128), lo=(-1.0,) * 3, hi=(1.0,) * 3, greens="hockney", prec="f32", bind=False)
    x = torch_cuda.zeros(4, device="cuda")
    st = lib.fsp_solve_static(plan.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr()), None)
    assert st == _lib.FSP_ERR_UNSUPPORTED_SIZE
    assert b"scratch" in lib.fsp_last_error()


def test_static_with_fused_schedules(torch_cuda):
    """The static workspace serves the plane kernels and the fused slab as well (one spectrum)."""
    from paper_2405_02603_amd import _lib
    lib = _lib.load()
    P, F = _lib.PLANE, _lib.FUSED
    _case(torch_cuda, lib, (24, 64, 64), (-1.0,) * 3, (1.0,) * 3, "vico_dct", "f32", 15, sched=[P, P, 0, P, P])
    _case(torch_cuda, lib, (32, 32, 32), (-0.5,) * 3, (0.5,) * 3, "hockney", "f64", 16, sched=[P, P, 1, 0, 0])
    _case(torch_cuda, lib, (32, 32, 16), (-0.5,) * 3, (0.5,) * 3, "vico_dct", "f32", 17, sched=[0, F, F, F, 0])
