"""C ABI checks that need no GPU: the library loads, exports every declared
symbol, and validates plans on the host (plan creation touches no device)."""
import ctypes
import math
import os
import re

import pytest

from paper_2405_02603_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "fsp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fsp_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def _desc(n=32, lo=-0.5, hi=0.5, greens=2, prec=0, alpha=1.1, g0=float("nan")):
    d = _lib.PlanDesc()
    d.n[:] = list(n) if isinstance(n, tuple) else [n] * 3
    d.lo[:] = list(lo) if isinstance(lo, tuple) else [lo] * 3
    d.hi[:] = list(hi) if isinstance(hi, tuple) else [hi] * 3
    d.greens, d.prec, d.alpha, d.g0, d.flags = greens, prec, alpha, g0, 0
    return d


def _create(lib, d):
    h = ctypes.c_void_p()
    st = lib.fsp_plan_create(ctypes.byref(d), ctypes.byref(h))
    return st, h


def test_exports_every_declared_symbol(lib):
    decl = _declared_symbols()
    assert len(decl) >= 14
    for name in decl:
        assert hasattr(lib, name), name
    assert sorted(_lib.EXPORTS) == decl


def test_version(lib):
    assert lib.fsp_version().decode().startswith("fsp ")


@pytest.mark.parametrize("n", [8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512])
def test_supported_sizes_create(lib, n):
    st, h = _create(lib, _desc(n=(n, 8, 12), greens=0))
    assert st == _lib.FSP_OK
    assert lib.fsp_plan_destroy(h) == _lib.FSP_OK


@pytest.mark.parametrize("n", [0, 4, 7, 10, 20, 40, 100, 640, 768, 1024])
def test_unsupported_sizes_rejected(lib, n):
    st, h = _create(lib, _desc(n=(32, n, 32)))
    assert st == _lib.FSP_ERR_UNSUPPORTED_SIZE
    assert not h.value
    assert b"n[1]" in lib.fsp_last_error()


def test_invalid_arguments(lib):
    assert _create(lib, _desc(lo=(0, 0, 0), hi=(1, 0, 1)))[0] == _lib.FSP_ERR_INVALID_ARG
    assert _create(lib, _desc(hi=float("inf")))[0] == _lib.FSP_ERR_INVALID_ARG
    assert _create(lib, _desc(greens=3))[0] == _lib.FSP_ERR_INVALID_ARG
    assert _create(lib, _desc(prec=2))[0] == _lib.FSP_ERR_INVALID_ARG
    assert _create(lib, _desc(alpha=0.9))[0] == _lib.FSP_ERR_INVALID_ARG
    assert lib.fsp_plan_create(None, None) == _lib.FSP_ERR_INVALID_ARG
    assert lib.fsp_solve(None, None, None, None) == _lib.FSP_ERR_INVALID_ARG
    assert lib.fsp_plan_destroy(None) == _lib.FSP_ERR_INVALID_ARG
    assert lib.fsp_solve_batched(-1, None, None, None, None) == _lib.FSP_ERR_INVALID_ARG
    assert lib.fsp_solve_batched(0, None, None, None, None) == _lib.FSP_OK


def test_box_aspect_limit(lib):
    # cube: alpha |diag| = 1.1 sqrt(3) L < 3 L
    assert _create(lib, _desc(greens=2))[0] == _lib.FSP_OK
    # 2 x 2 x 4 box passes (5.39 <= 6)
    assert _create(lib, _desc(lo=(-1, -1, -2), hi=(1, 1, 2), greens=2))[0] == _lib.FSP_OK
    # a thin slab fails for Vico-Greengard but not for Hockney-Eastwood
    assert _create(lib, _desc(lo=(0, 0, 0), hi=(1, 1, 0.2), greens=2))[0] == _lib.FSP_ERR_BOX_ASPECT
    assert _create(lib, _desc(lo=(0, 0, 0), hi=(1, 1, 0.2), greens=0))[0] == _lib.FSP_OK


def test_original_vico_route_size_limit(lib):
    assert _create(lib, _desc(n=256, greens=1))[0] == _lib.FSP_OK
    assert _create(lib, _desc(n=512, greens=1))[0] == _lib.FSP_ERR_UNSUPPORTED_SIZE


def test_solve_before_bind_is_not_ready(lib):
    st, h = _create(lib, _desc())
    assert st == _lib.FSP_OK
    dummy = ctypes.c_void_p(256)
    assert lib.fsp_solve(h, dummy, dummy, None) == _lib.FSP_ERR_NOT_READY
    assert lib.fsp_precompute(h, None) == _lib.FSP_ERR_NOT_READY
    assert lib.fsp_solve_passes(h, dummy, dummy, 0, 5, None) == _lib.FSP_ERR_INVALID_ARG
    assert lib.fsp_solve_passes(h, dummy, dummy, 2, 1, None) == _lib.FSP_ERR_INVALID_ARG
    assert lib.fsp_plan_bind(h, ctypes.c_void_p(1), ctypes.c_void_p(256)) == _lib.FSP_ERR_INVALID_ARG
    lib.fsp_plan_destroy(h)


@pytest.mark.parametrize("prec,rb", [(0, 4), (1, 8)])
@pytest.mark.parametrize("n", [(32, 32, 32), (256, 256, 256), (16, 24, 48)])
def test_buffer_sizes_and_model_bytes(lib, prec, rb, n):
    st, h = _create(lib, _desc(n=n, prec=prec))
    assert st == _lib.FSP_OK
    g, w = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.fsp_plan_bytes(h, ctypes.byref(g), ctypes.byref(w)) == _lib.FSP_OK
    off, tile = ctypes.c_size_t(), ctypes.c_int()
    assert lib.fsp_plan_ghat_layout(h, ctypes.byref(off), ctypes.byref(tile)) == _lib.FSP_OK
    n0, n1, n2 = n
    t = tile.value
    assert t >= 1 and (t & (t - 1)) == 0
    assert off.value % 256 == 0
    tiles = (n2 + 1 + t - 1) // t
    assert g.value >= off.value + (n1 + 1) * tiles * (n0 + 1) * t * rb
    pitch = n2 + 1 + (-(n2 + 1)) % (128 // (2 * rb))
    assert w.value >= n0 * 2 * n1 * pitch * 2 * rb
    mb = ctypes.c_double()
    assert lib.fsp_plan_model_bytes(h, ctypes.byref(mb)) == _lib.FSP_OK
    # five passes: 2 N^3 + 24 (N2+1) N0 N1 + (N0+1)(N1+1)(N2+1) reals
    want = (2 * n0 * n1 * n2 + 24 * (n2 + 1) * n0 * n1 + (n0 + 1) * (n1 + 1) * (n2 + 1)) * rb
    assert math.isclose(mb.value, want, rel_tol=1e-12)
    pb = ctypes.c_size_t()
    assert lib.fsp_plan_precompute_bytes(h, ctypes.byref(pb)) == _lib.FSP_OK
    assert pb.value > 0
    lib.fsp_plan_destroy(h)


def test_status_strings(lib):
    for code in range(7):
        assert lib.fsp_status_str(code).decode().startswith("FSP_")


def test_schedule_validation(lib):
    st, h = _create(lib, _desc(n=32))
    assert st == _lib.FSP_OK
    arr = (ctypes.c_int * 5)()
    assert lib.fsp_plan_get_schedule(h, arr) == _lib.FSP_OK
    assert list(arr) == [0, 0, 0, 0, 0]
    ok = (ctypes.c_int * 5)(2, 1, 0, 2, 1)
    assert lib.fsp_plan_set_schedule(h, ok) == _lib.FSP_OK
    fused = (ctypes.c_int * 5)(0, 3, 3, 3, 0)
    assert lib.fsp_plan_set_schedule(h, fused) == _lib.FSP_OK
    # with the fused schedule a pass range holds all of passes 1-3 or none of them
    dummy = ctypes.c_void_p(256)
    for first, last in ((1, 1), (2, 2), (2, 4), (0, 2), (3, 4)):
        assert lib.fsp_solve_passes(h, dummy, dummy, first, last, None) == _lib.FSP_ERR_INVALID_ARG, (first, last)
    for first, last in ((0, 0), (4, 4), (1, 3), (0, 4)):
        assert lib.fsp_solve_passes(h, dummy, dummy, first, last, None) == _lib.FSP_ERR_NOT_READY, (first, last)
    for bad in ((0, 3, 0, 3, 0), (3, 0, 0, 0, 0), (0, 0, 0, 0, 4), (-1, 0, 0, 0, 0)):
        assert lib.fsp_plan_set_schedule(h, (ctypes.c_int * 5)(*bad)) == _lib.FSP_ERR_INVALID_ARG
    lib.fsp_plan_destroy(h)
    # the fused schedule needs n0 == n1 and a slab that fits in LDS
    st, h = _create(lib, _desc(n=(32, 64, 32)))
    assert lib.fsp_plan_set_schedule(h, fused) == _lib.FSP_ERR_INVALID_ARG
    lib.fsp_plan_destroy(h)
    st, h = _create(lib, _desc(n=256))
    assert lib.fsp_plan_set_schedule(h, fused) == _lib.FSP_ERR_INVALID_ARG
    lib.fsp_plan_destroy(h)


@pytest.mark.parametrize("prec,n,supported", [(0, 32, True), (0, (16, 96, 96), True),
                                              (0, 128, True), (0, 256, False),
                                              (0, (32, 32, 64), False), (0, 24, False),
                                              (1, 64, True), (1, 96, False)])
def test_plane_schedule_validation(lib, prec, n, supported):
    """The plane pairs: passes 0 and 1 (or 3 and 4) both set to 4, on grids with n1 == n2 whose
    plane fits in LDS; a pass range holds both passes of a pair or neither; the pairs exclude the
    fused slab schedule."""
    st, h = _create(lib, _desc(n=n, prec=prec, greens=0))
    assert st == _lib.FSP_OK
    P, F = _lib.PLANE, _lib.FUSED
    want = _lib.FSP_OK if supported else _lib.FSP_ERR_INVALID_ARG
    for sched in ((P, P, 0, P, P), (P, P, 2, 1, 0), (1, 2, 0, P, P)):
        assert lib.fsp_plan_set_schedule(h, (ctypes.c_int * 5)(*sched)) == want, sched
    for bad in ((P, 0, 0, 0, 0), (0, P, 0, 0, 0), (0, 0, 0, P, 0), (0, 0, 0, 0, P), (0, 0, P, 0, 0),
                (P, P, F, F, F), (0, F, F, F, P), (P, P, 3, P, P)):
        assert lib.fsp_plan_set_schedule(h, (ctypes.c_int * 5)(*bad)) == _lib.FSP_ERR_INVALID_ARG, bad
    if supported:
        # model bytes follow the schedule: each plane pair saves a write and a read of the
        # (n2+1) n1 n0 axis-2 spectrum
        n3 = n if isinstance(n, tuple) else (n,) * 3
        rb = 4 if prec == 0 else 8
        half1 = n3[0] * n3[1] * (n3[2] + 1) * 2 * rb
        mb = ctypes.c_double()
        assert lib.fsp_plan_set_schedule(h, (ctypes.c_int * 5)(0, 0, 0, 0, 0)) == _lib.FSP_OK
        assert lib.fsp_plan_model_bytes(h, ctypes.byref(mb)) == _lib.FSP_OK
        sep = mb.value
        assert lib.fsp_plan_set_schedule(h, (ctypes.c_int * 5)(P, P, 0, 0, 0)) == _lib.FSP_OK
        assert lib.fsp_plan_model_bytes(h, ctypes.byref(mb)) == _lib.FSP_OK
        assert mb.value == sep - 2 * half1
        assert lib.fsp_plan_set_schedule(h, (ctypes.c_int * 5)(P, P, 0, P, P)) == _lib.FSP_OK
        assert lib.fsp_plan_model_bytes(h, ctypes.byref(mb)) == _lib.FSP_OK
        assert mb.value == sep - 4 * half1
        dummy = ctypes.c_void_p(256)
        for first, last in ((0, 0), (1, 1), (1, 2), (3, 3), (4, 4), (2, 3), (1, 4)):
            assert lib.fsp_solve_passes(h, dummy, dummy, first, last, None) == _lib.FSP_ERR_INVALID_ARG, (first, last)
        for first, last in ((0, 1), (2, 2), (3, 4), (0, 4), (0, 2), (2, 4)):
            assert lib.fsp_solve_passes(h, dummy, dummy, first, last, None) == _lib.FSP_ERR_NOT_READY, (first, last)
    lib.fsp_plan_destroy(h)


def test_gradient_plan_sizes_offsets_and_errors(lib):
    # unknown flag bits are rejected (bits 1-3 are the periodic axes)
    d = _desc(n=32)
    d.flags = 16
    assert _create(lib, d)[0] == _lib.FSP_ERR_INVALID_ARG
    # a plan without FSP_WANT_GRAD: one octant, one workspace, no derivative tables
    st, h0 = _create(lib, _desc(n=(16, 24, 32)))
    g0, w0 = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.fsp_plan_bytes(h0, ctypes.byref(g0), ctypes.byref(w0)) == _lib.FSP_OK
    off = ctypes.c_size_t()
    assert lib.fsp_plan_octant_offset(h0, 1, ctypes.byref(off)) == _lib.FSP_ERR_INVALID_ARG
    dummy = ctypes.c_void_p(256)
    assert lib.fsp_solve_grad(h0, dummy, None, dummy, None) == _lib.FSP_ERR_INVALID_ARG
    # with it: three more octants in the Green's buffer and three more spectra in the workspace
    d = _desc(n=(16, 24, 32))
    d.flags = _lib.FSP_WANT_GRAD
    st, h = _create(lib, d)
    assert st == _lib.FSP_OK
    g, w = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.fsp_plan_bytes(h, ctypes.byref(g), ctypes.byref(w)) == _lib.FSP_OK
    assert w.value == 4 * w0.value
    layout_off = ctypes.c_size_t()
    assert lib.fsp_plan_ghat_layout(h, ctypes.byref(layout_off), None) == _lib.FSP_OK
    offs = []
    for c in range(4):
        assert lib.fsp_plan_octant_offset(h, c, ctypes.byref(off)) == _lib.FSP_OK
        offs.append(off.value)
    assert offs[0] == layout_off.value
    step = offs[1] - offs[0]
    assert step > 0 and step % 256 == 0 and offs[2] - offs[1] == step and offs[3] - offs[2] == step
    assert g.value == offs[3] + step and g0.value == offs[0] + step
    for bad in (-1, 4):
        assert lib.fsp_plan_octant_offset(h, bad, ctypes.byref(off)) == _lib.FSP_ERR_INVALID_ARG
    assert lib.fsp_solve_grad(h, None, None, dummy, None) == _lib.FSP_ERR_INVALID_ARG
    assert lib.fsp_solve_grad(h, dummy, None, None, None) == _lib.FSP_ERR_INVALID_ARG
    assert lib.fsp_solve_grad(h, dummy, None, dummy, None) == _lib.FSP_ERR_NOT_READY
    lib.fsp_plan_destroy(h)
    lib.fsp_plan_destroy(h0)


@pytest.mark.parametrize("n", [64, 128, 256, 512])
def test_footprint_against_the_paper_accounting(lib, n):
    """Device bytes of one float64 solve here (Green's buffer, workspace, rho and phi) beside the
    field memory of Section 3.3 (five float64 fields on the doubled grid and more): the fused
    pad/crop and the real octant keep it below a third of the paper's smallest (modified
    Vico-Greengard) figure, and the transient precompute of the Vico-Greengard tables stays
    below the (2N+1)^3 field the paper keeps."""
    from oracle import memory
    for greens, paper in ((0, memory.hockney_bytes(n)), (2, memory.vico_dct_bytes(n))):
        st, h = _create(lib, _desc(n=n, greens=greens, prec=1, lo=-1.0, hi=1.0))
        assert st == _lib.FSP_OK
        g, w = ctypes.c_size_t(), ctypes.c_size_t()
        assert lib.fsp_plan_bytes(h, ctypes.byref(g), ctypes.byref(w)) == _lib.FSP_OK
        ours = g.value + w.value + 2 * n ** 3 * 8
        assert ours < paper / 3, (greens, ours, paper)
        pb = ctypes.c_size_t()
        assert lib.fsp_plan_precompute_bytes(h, ctypes.byref(pb)) == _lib.FSP_OK
        if greens == 2:
            assert pb.value < 2 * (2 * n + 1) ** 3 * 8
        lib.fsp_plan_destroy(h)


def test_static_solve_rejects_oversize_on_the_host(lib):
    """fsp_solve_static checks the plan's workspace against its static scratch before
    anything touches a device: a 256^2 x 128 float32 plan is too big, 128^3 float64 fits
    (and is then only 'not ready', since it was never bound)."""
    dummy = ctypes.c_void_p(256)
    st, h = _create(lib, _desc(n=(256, 256, 128), greens=0, prec=0))
    assert st == _lib.FSP_OK
    assert lib.fsp_solve_static(h, dummy, dummy, None) == _lib.FSP_ERR_UNSUPPORTED_SIZE
    assert b"scratch" in lib.fsp_last_error()
    lib.fsp_plan_destroy(h)
    st, h = _create(lib, _desc(n=128, greens=0, prec=1))
    wb = ctypes.c_size_t()
    assert lib.fsp_plan_bytes(h, None, ctypes.byref(wb)) == _lib.FSP_OK
    assert wb.value <= _lib.STATIC_SCRATCH_BYTES
    assert lib.fsp_solve_static(h, dummy, dummy, None) == _lib.FSP_ERR_NOT_READY
    lib.fsp_plan_destroy(h)
    assert lib.fsp_solve_static(None, dummy, dummy, None) == _lib.FSP_ERR_INVALID_ARG


def test_static_scratch_size_matches_header():
    text = open(os.path.join(ROOT, "include", "fsp.h")).read()
    m = re.search(r"#define FSP_STATIC_SCRATCH_BYTES \((\d+)u \* 1024u \* 1024u\)", text)
    assert m and int(m.group(1)) * 1024 * 1024 == _lib.STATIC_SCRATCH_BYTES


def test_autotune_batch_arguments(lib):
    arr = ctypes.c_void_p * 1
    assert lib.fsp_autotune_batch(0, None, None, None, 2, None) == _lib.FSP_OK
    assert lib.fsp_autotune_batch(-1, None, None, None, 2, None) == _lib.FSP_ERR_INVALID_ARG
    assert lib.fsp_autotune_batch(1, None, None, None, 2, None) == _lib.FSP_ERR_INVALID_ARG
    st, h = _create(lib, _desc(n=32))
    d = ctypes.c_void_p(256)
    # an unbound plan is not ready (the check precedes any device work)
    assert lib.fsp_autotune_batch(1, arr(h.value), arr(d.value), arr(d.value), 2, None) == _lib.FSP_ERR_NOT_READY
    lib.fsp_plan_destroy(h)


def test_autotune_rejects_aliased_rho_phi(lib):
    """The tuning solves write phi many times, so phi may not overlap rho; checked on
    the host before the plan's state."""
    st, h = _create(lib, _desc(n=16))
    assert st == _lib.FSP_OK
    base = 1 << 20
    field = 16 ** 3 * 4
    for off in (0, 4, field - 4):
        r = lib.fsp_autotune(h, ctypes.c_void_p(base), ctypes.c_void_p(base + off), 2, None, None)
        assert r == _lib.FSP_ERR_INVALID_ARG, off
        assert b"overlaps" in lib.fsp_last_error()
    # disjoint buffers get past the alias check (and stop at the unbound plan)
    r = lib.fsp_autotune(h, ctypes.c_void_p(base), ctypes.c_void_p(base + field), 2, None, None)
    assert r == _lib.FSP_ERR_NOT_READY
    lib.fsp_plan_destroy(h)


def test_periodic_flags(lib):
    """Periodic-axis flags are accepted on every axis and Green's function; they cannot be
    combined with FSP_WANT_GRAD."""
    for greens in (0, 1, 2):
        for bit in (2, 4, 8, 14):
            d = _desc(n=16, greens=greens)
            d.flags = bit
            st, h = _create(lib, d)
            assert st == _lib.FSP_OK, (greens, bit)
            lib.fsp_plan_destroy(h)
    d = _desc(n=16)
    d.flags = 1 | 4
    assert _create(lib, d)[0] == _lib.FSP_ERR_INVALID_ARG
    assert b"FSP_WANT_GRAD" in lib.fsp_last_error()
    d.flags = 16
    assert _create(lib, d)[0] == _lib.FSP_ERR_INVALID_ARG
