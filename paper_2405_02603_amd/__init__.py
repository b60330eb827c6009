"""Free-space Poisson solver on MI355X (gfx950): Python binding of libfsp.so.

This module marshals arguments only.  Every step of a solve runs in the HIP
kernels of libfsp.so; PyTorch supplies device memory and streams.  Importing
the package does not load the library; the first ``Plan`` does, and it raises
if ``libfsp.so`` has not been built.

    from paper_2405_02603_amd import Plan
    plan = Plan(n=256, lo=(-1, -1, -1), hi=(1, 1, 1), greens="vico_dct", prec="f32")
    phi = plan.solve(rho)          # rho: float32 CUDA tensor of shape (256, 256, 256)
"""
from __future__ import annotations

import ctypes
import math
from typing import Iterable, List, Optional, Sequence

from . import _lib
from ._lib import FspError, GREENS, PREC, check

__all__ = ["Plan", "Batch", "solve_batched", "autotune_batch", "FspError", "GREENS", "PREC", "library_path", "version"]

_DTYPES = {"f32": "float32", "f64": "float64"}


def library_path() -> str:
    return _lib.LIB_PATH


def version() -> str:
    return _lib.load().fsp_version().decode()


def _torch():
    import torch
    return torch


def _as3(v, t=float):
    if isinstance(v, (int, float)):
        return (t(v),) * 3
    v = tuple(t(x) for x in v)
    if len(v) != 3:
        raise ValueError("expected a scalar or a 3-sequence")
    return v


def _stream_ptr(stream) -> ctypes.c_void_p:
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def _aligned_bytes(nbytes: int, device, align: int = 256):
    """A uint8 device tensor of nbytes whose data pointer is align-byte aligned."""
    torch = _torch()
    raw = torch.empty(nbytes + align, dtype=torch.uint8, device=device)
    off = (-raw.data_ptr()) % align
    return raw[off:off + nbytes]


class Plan:
    """One grid size, box, Green's function and precision, with its device buffers.

    ``greens``: "hockney" (Section 2.2), "vico" (Section 2.3, 4N precompute) or
    "vico_dct" (Section 2.4, (2N+1)^3 DCT-I precompute).
    ``prec``: "f32" or "f64" (precision of rho, phi and the solve passes; the
    precompute always runs in float64).
    ``grad``: also build the derivative tables for ``solve_grad``.
    ``periodic``: per axis, a periodic boundary instead of an open one (see FSP_PERIODIC_0 in fsp.h).
    """

    def __init__(self, n, lo=(-0.5, -0.5, -0.5), hi=(0.5, 0.5, 0.5), greens: str = "vico_dct",
                 prec: str = "f32", alpha: float = 1.1, g0: Optional[float] = None, device=None,
                 precompute: bool = True, stream=None, bind: bool = True, grad: bool = False,
                 periodic=(False, False, False)):
        torch = _torch()
        self._lib = _lib.load()
        if greens not in GREENS:
            raise ValueError(f"greens must be one of {sorted(GREENS)}")
        if prec not in PREC:
            raise ValueError(f"prec must be one of {sorted(PREC)}")
        self.n = _as3(n, int)
        self.lo = _as3(lo)
        self.hi = _as3(hi)
        self.greens = greens
        self.prec = prec
        self.alpha = float(alpha)
        self.g0 = g0
        self.dtype = getattr(torch, _DTYPES[prec])
        self.device = torch.device(device if device is not None else "cuda")
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        desc = _lib.PlanDesc()
        desc.n[:] = list(self.n)
        desc.lo[:] = list(self.lo)
        desc.hi[:] = list(self.hi)
        desc.greens = GREENS[greens]
        desc.prec = PREC[prec]
        desc.alpha = self.alpha
        desc.g0 = float("nan") if g0 is None else float(g0)
        self.grad = bool(grad)
        self.periodic = tuple(bool(x) for x in periodic)
        desc.flags = (_lib.FSP_WANT_GRAD if self.grad else 0) | sum(
            f for f, on in zip(_lib.FSP_PERIODIC, self.periodic) if on)
        h = ctypes.c_void_p()
        check(self._lib.fsp_plan_create(ctypes.byref(desc), ctypes.byref(h)), "fsp_plan_create")
        self._h = h
        gb, wb = ctypes.c_size_t(), ctypes.c_size_t()
        check(self._lib.fsp_plan_bytes(h, ctypes.byref(gb), ctypes.byref(wb)), "fsp_plan_bytes")
        self.ghat_bytes, self.work_bytes = int(gb.value), int(wb.value)
        pb = ctypes.c_size_t()
        check(self._lib.fsp_plan_precompute_bytes(h, ctypes.byref(pb)), "fsp_plan_precompute_bytes")
        self.precompute_bytes = int(pb.value)
        off, tile = ctypes.c_size_t(), ctypes.c_int()
        check(self._lib.fsp_plan_ghat_layout(h, ctypes.byref(off), ctypes.byref(tile)), "fsp_plan_ghat_layout")
        self.octant_offset, self.octant_tile = int(off.value), int(tile.value)
        mb = ctypes.c_double()
        check(self._lib.fsp_plan_model_bytes(h, ctypes.byref(mb)), "fsp_plan_model_bytes")
        self.model_bytes = float(mb.value)
        self.ghat_buf = None
        self.work_buf = None
        self._shared_from = None
        if bind:
            self.bind()
            if precompute:
                self.precompute(stream)

    # ------------------------------------------------------------ buffers
    def bind(self, ghat=None, work=None) -> None:
        """Attach device buffers (uint8 tensors, 256-byte aligned); None allocates them with torch."""
        torch = _torch()
        with torch.cuda.device(self.device):
            self.ghat_buf = ghat if ghat is not None else _aligned_bytes(self.ghat_bytes, self.device)
            self.work_buf = work if work is not None else _aligned_bytes(self.work_bytes, self.device)
            if self.ghat_buf.numel() < self.ghat_bytes or self.work_buf.numel() < self.work_bytes:
                raise ValueError("bound buffers are smaller than fsp_plan_bytes")
            check(self._lib.fsp_plan_bind(self._h, ctypes.c_void_p(self.ghat_buf.data_ptr()),
                                          ctypes.c_void_p(self.work_buf.data_ptr())), "fsp_plan_bind")

    def precompute(self, stream=None) -> None:
        torch = _torch()
        with torch.cuda.device(self.device):
            check(self._lib.fsp_precompute(self._h, _stream_ptr(stream)), "fsp_precompute")

    def share_ghat(self, src: "Plan") -> None:
        """Read src's precomputed transform instead of computing one (equal plans only)."""
        check(self._lib.fsp_plan_share_ghat(self._h, src._h), "fsp_plan_share_ghat")
        self._shared_from = src  # keep src (and its buffer) alive

    def ghat_octant(self, component: int = 0):
        """A stored octant as a [n0+1][n1+1][n2+1] tensor (scaled by V/(8 n0 n1 n2)): component 0
        the transform of the Green's function, 1 + a the real T of a derivative table (transform -i T)."""
        torch = _torch()
        src = self._shared_from.ghat_octant(component) if self._shared_from is not None else None
        if src is not None:
            return src
        off = ctypes.c_size_t()
        check(self._lib.fsp_plan_octant_offset(self._h, int(component), ctypes.byref(off)), "fsp_plan_octant_offset")
        off = int(off.value)
        n0, n1, n2 = self.n
        esz = 8 if self.prec == "f64" else 4
        t = self.octant_tile
        tiles = (n2 + 1 + t - 1) // t
        nb = (n1 + 1) * tiles * (n0 + 1) * t * esz
        raw = self.ghat_buf[off:off + nb].view(self.dtype)
        blocked = raw.view(n1 + 1, tiles, n0 + 1, t)            # [k1][tile][k0][c]
        full = blocked.permute(2, 0, 1, 3).reshape(n0 + 1, n1 + 1, tiles * t)
        return full[:, :, : n2 + 1]

    # ------------------------------------------------------------ solves
    def _check_field(self, t, name: str) -> None:
        if t.dtype != self.dtype:
            raise TypeError(f"{name} must be {self.dtype}, got {t.dtype}")
        if tuple(t.shape) != self.n:
            raise ValueError(f"{name} must have shape {self.n}, got {tuple(t.shape)}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be C-contiguous")
        if t.device != self.device:
            raise ValueError(f"{name} must be on {self.device}")

    def solve(self, rho, out=None, stream=None):
        """phi for rho (CUDA tensor of the plan's shape and dtype); out may be rho (in place)."""
        torch = _torch()
        self._check_field(rho, "rho")
        if out is None:
            out = torch.empty_like(rho)
        self._check_field(out, "out")
        with torch.cuda.device(self.device):
            check(self._lib.fsp_solve(self._h, ctypes.c_void_p(rho.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                      _stream_ptr(stream)), "fsp_solve")
        return out

    def solve_static(self, rho, out=None, stream=None):
        """As ``solve`` but on the library's static per-GPU workspace (fsp_solve_static):
        the call allocates no device memory.  ``out`` must be given when the caller
        cannot allocate; calls that overlap on one GPU race (serialise them)."""
        torch = _torch()
        self._check_field(rho, "rho")
        if out is None:
            out = torch.empty_like(rho)
        self._check_field(out, "out")
        with torch.cuda.device(self.device):
            check(self._lib.fsp_solve_static(self._h, ctypes.c_void_p(rho.data_ptr()),
                                             ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)),
                  "fsp_solve_static")
        return out

    def solve_grad(self, rho, grad=None, phi=None, want_phi: bool = False, stream=None):
        """grad = (d phi/dx0, d phi/dx1, d phi/dx2) as a [3][n0][n1][n2] tensor, and phi when
        ``phi`` is given or ``want_phi``; returns (grad, phi or None).  See fsp_solve_grad."""
        torch = _torch()
        if not self.grad:
            raise ValueError("create the plan with grad=True")
        self._check_field(rho, "rho")
        if grad is None:
            grad = torch.empty((3,) + self.n, dtype=self.dtype, device=self.device)
        if tuple(grad.shape) != (3,) + self.n or grad.dtype != self.dtype or not grad.is_contiguous() \
                or grad.device != self.device:
            raise ValueError(f"grad must be a contiguous {self.dtype} tensor of shape {(3,) + self.n}")
        if phi is None and want_phi:
            phi = torch.empty_like(rho)
        if phi is not None:
            self._check_field(phi, "phi")
        with torch.cuda.device(self.device):
            check(self._lib.fsp_solve_grad(self._h, ctypes.c_void_p(rho.data_ptr()),
                                           ctypes.c_void_p(phi.data_ptr() if phi is not None else 0),
                                           ctypes.c_void_p(grad.data_ptr()), _stream_ptr(stream)),
                  "fsp_solve_grad")
        return grad, phi

    def solve_passes(self, rho, out, first: int, last: int, stream=None):
        """Run passes first..last (0..4) of a solve; see fsp_solve_passes."""
        torch = _torch()
        rp = ctypes.c_void_p(rho.data_ptr() if rho is not None else 0)
        op = ctypes.c_void_p(out.data_ptr() if out is not None else 0)
        with torch.cuda.device(self.device):
            check(self._lib.fsp_solve_passes(self._h, rp, op, int(first), int(last), _stream_ptr(stream)),
                  "fsp_solve_passes")
        return out

    @property
    def schedule(self):
        """Variant of each of the five passes."""
        arr = (ctypes.c_int * 5)()
        check(self._lib.fsp_plan_get_schedule(self._h, arr), "fsp_plan_get_schedule")
        return list(arr)

    @schedule.setter
    def schedule(self, variants):
        arr = (ctypes.c_int * 5)(*[int(v) for v in variants])
        check(self._lib.fsp_plan_set_schedule(self._h, arr), "fsp_plan_set_schedule")

    def autotune(self, rho, out=None, reps: int = 4, stream=None):
        """Time every pass variant on rho (see fsp_autotune); returns {pass: [ms per variant]} and the
        whole-solve times of the schedules built from them (solve_separate, solve_fused, solve_plane,
        solve_plane_fwd, solve_plane_inv)."""
        torch = _torch()
        self._check_field(rho, "rho")
        if out is None:
            out = torch.empty_like(rho)
        self._check_field(out, "out")
        times = (ctypes.c_float * (5 * _lib.NUM_VARIANTS + 5))()
        with torch.cuda.device(self.device):
            check(self._lib.fsp_autotune(self._h, ctypes.c_void_p(rho.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                         int(reps), _stream_ptr(stream), times), "fsp_autotune")
        nv = _lib.NUM_VARIANTS
        out = {p: [times[p * nv + v] for v in range(nv)] for p in range(5)}
        # whole solves with schedules built from the best variants (0: not supported)
        for i, key in enumerate(("solve_fused", "solve_separate", "solve_plane", "solve_plane_fwd",
                                 "solve_plane_inv")):
            out[key] = times[5 * nv + i]
        return out

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.fsp_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __repr__(self):
        return (f"Plan(n={self.n}, lo={self.lo}, hi={self.hi}, greens={self.greens!r}, prec={self.prec!r}, "
                f"alpha={self.alpha})")


def solve_batched(plans: Sequence[Plan], rhos: Sequence, outs: Optional[Sequence] = None, stream=None) -> List:
    """One call for many independent solves, each with its own plan (and so its own workspace)."""
    torch = _torch()
    count = len(plans)
    if len(rhos) != count:
        raise ValueError("need one rho per plan")
    if outs is None:
        outs = [torch.empty_like(r) for r in rhos]
    if len(outs) != count:
        raise ValueError("need one output per plan")
    for p, r, o in zip(plans, rhos, outs):
        p._check_field(r, "rho")
        p._check_field(o, "out")
    if count == 0:
        return list(outs)
    arr = ctypes.c_void_p * count
    hp = arr(*[p.handle.value for p in plans])
    rp = arr(*[r.data_ptr() for r in rhos])
    op = arr(*[o.data_ptr() for o in outs])
    lib = _lib.load()
    with torch.cuda.device(plans[0].device):
        check(lib.fsp_solve_batched(count, hp, rp, op, _stream_ptr(stream)), "fsp_solve_batched")
    return list(outs)


def autotune_batch(plans: Sequence[Plan], rhos: Sequence, outs: Optional[Sequence] = None, reps: int = 4,
                   stream=None) -> None:
    """Choose each equal-shape group's schedule with the group's solves timed together
    (fsp_autotune_batch); the plans keep the chosen schedules."""
    torch = _torch()
    count = len(plans)
    if len(rhos) != count:
        raise ValueError("need one rho per plan")
    if outs is None:
        outs = [torch.empty_like(r) for r in rhos]
    if len(outs) != count:
        raise ValueError("need one output per plan")
    for p, r, o in zip(plans, rhos, outs):
        p._check_field(r, "rho")
        p._check_field(o, "out")
    if count == 0:
        return
    arr = ctypes.c_void_p * count
    hp = arr(*[p.handle.value for p in plans])
    rp = arr(*[r.data_ptr() for r in rhos])
    op = arr(*[o.data_ptr() for o in outs])
    lib = _lib.load()
    with torch.cuda.device(plans[0].device):
        check(lib.fsp_autotune_batch(count, hp, rp, op, int(reps), _stream_ptr(stream)), "fsp_autotune_batch")


class Batch:
    """A set of solves replayed as one captured HIP graph (fsp_batch_*).

    The plans and the current rho / out tensors are held by the batch; the first
    launch captures the graph, later launches replay it.  ``set_io`` swaps in new
    rho / out tensors (the kernels read them from a device table), with no new
    capture.
    """

    def __init__(self, plans: Sequence[Plan], rhos: Sequence, outs: Optional[Sequence] = None):
        torch = _torch()
        count = len(plans)
        if count == 0 or len(rhos) != count:
            raise ValueError("need one rho per plan and at least one solve")
        if outs is None:
            outs = [torch.empty_like(r) for r in rhos]
        for p, r, o in zip(plans, rhos, outs):
            p._check_field(r, "rho")
            p._check_field(o, "out")
        self.plans, self.rhos, self.outs = list(plans), list(rhos), list(outs)
        self.device = self.plans[0].device
        arr = ctypes.c_void_p * count
        hp = arr(*[p.handle.value for p in self.plans])
        rp = arr(*[r.data_ptr() for r in self.rhos])
        op = arr(*[o.data_ptr() for o in self.outs])
        self._lib = _lib.load()
        h = ctypes.c_void_p()
        check(self._lib.fsp_batch_create(count, hp, rp, op, ctypes.byref(h)), "fsp_batch_create")
        self._h = h

    def set_io(self, rhos: Sequence, outs: Optional[Sequence] = None, stream=None):
        """New rho (and out) tensors for every solve, in the batch's order (fsp_batch_set_io);
        launches enqueued after this on the same stream use them."""
        torch = _torch()
        if len(rhos) != len(self.plans):
            raise ValueError("need one rho per solve")
        if outs is None:
            outs = [torch.empty_like(r) for r in rhos]
        if len(outs) != len(self.plans):
            raise ValueError("need one output per solve")
        for p, r, o in zip(self.plans, rhos, outs):
            p._check_field(r, "rho")
            p._check_field(o, "out")
        arr = ctypes.c_void_p * len(self.plans)
        rp = arr(*[r.data_ptr() for r in rhos])
        op = arr(*[o.data_ptr() for o in outs])
        with torch.cuda.device(self.device):
            check(self._lib.fsp_batch_set_io(self._h, rp, op, _stream_ptr(stream)), "fsp_batch_set_io")
        self.rhos, self.outs = list(rhos), list(outs)
        return self.outs

    def launch(self, stream=None):
        torch = _torch()
        with torch.cuda.device(self.device):
            check(self._lib.fsp_batch_launch(self._h, _stream_ptr(stream)), "fsp_batch_launch")
        return self.outs

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.fsp_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
