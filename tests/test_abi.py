"""The C ABI of libbms.so without a GPU: every symbol include/bms.h declares is
exported, the Python binding names the same set, and the host-side argument
checks reject bad calls before any device work (none of these calls reaches
the HIP runtime)."""
import ctypes
import os
import re

import pytest

from paper_1808_01829_amd import bms

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bms.h")


def header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    src = re.sub(r"#[^\n]*", " ", src)
    names = re.findall(r"(?:^|[;}\n])\s*(?:const\s+)?(?:int|void|char|double)\s*\**\s*(bms_\w+)\s*\(",
                       src)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(bms.LIB_PATH):
        from paper_1808_01829_amd import build
        build.build()
    return bms._lib()


def test_header_parse_finds_the_entry_points():
    names = header_functions()
    for must in ("bms_create", "bms_solve", "bms_force", "bms_action", "bms_apply_hop"):
        assert must in names
    assert len(names) >= 14


def test_every_declared_symbol_is_exported(lib):
    raw = ctypes.CDLL(bms.LIB_PATH)
    missing = [n for n in header_functions() if not hasattr(raw, n)]
    assert not missing, missing


def test_binding_names_match_header():
    assert sorted(bms.EXPORTS) == header_functions()


def test_default_opts_and_error_strings(lib):
    o = bms.bms_opts()
    lib.bms_default_opts(ctypes.byref(o))
    assert o.precision == bms.BMS_PREC_F64
    assert o.check_interval >= 1 and o.qr_passes == 1 and o.reliable_interval >= 1
    for code in range(0, -8, -1):
        s = lib.bms_error_string(code).decode()
        assert s and "unknown" not in s
    assert "unknown" in lib.bms_error_string(-99).decode()


def _create(lib, dims, bc=(1, 1, 1, -1)):
    ctx = ctypes.c_void_p()
    rc = lib.bms_create(ctypes.byref(ctx), (ctypes.c_int * 4)(*dims), (ctypes.c_int * 4)(*bc), None)
    return rc, ctx


@pytest.mark.parametrize("dims,bc", [((3, 4, 4, 4), (1, 1, 1, -1)), ((4, 4, 4, 0), (1, 1, 1, 1)),
                                     ((4, 4, 4, 4), (1, 1, 1, 0)), ((64, 64, 64, 256), (1,) * 4)])
def test_create_rejects(lib, dims, bc):
    rc, ctx = _create(lib, dims, bc)
    assert rc == bms.BMS_EINVAL and not ctx.value


def test_calls_without_gauge_fail_on_the_host(lib):
    rc, ctx = _create(lib, (4, 4, 4, 4))
    assert rc == bms.BMS_OK and ctx.value
    try:
        dummy = ctypes.c_void_p(0x1000)
        other = ctypes.c_void_p(0x2000)
        sh = (ctypes.c_double * 2)(0.1, 0.2)
        # argument errors come first
        assert lib.bms_apply_hop(ctx, 2, 1, dummy, other, 0) == bms.BMS_EINVAL
        assert lib.bms_apply_hop(ctx, 1, 33, dummy, other, 0) == bms.BMS_EINVAL
        assert lib.bms_apply_hop(ctx, 1, 1, dummy, dummy, 0) == bms.BMS_EINVAL
        assert lib.bms_apply_mdagm(ctx, 0.1, 0.0, 1, dummy, other, 2) == bms.BMS_EINVAL
        assert "precision" in lib.bms_last_error(ctx).decode()
        assert lib.bms_solve(ctx, 0.1, 0, 2, sh, 1e-8, 100, None, dummy, other, None) == bms.BMS_EINVAL
        assert lib.bms_solve(ctx, 0.1, 1, 2, sh, 1.5, 100, None, dummy, other, None) == bms.BMS_EINVAL
        assert lib.bms_solve(ctx, 0.1, 1, 2, sh, 1e-8, 100, None, dummy, dummy, None) == bms.BMS_EINVAL
        neg = (ctypes.c_double * 2)(0.1, -0.2)
        assert lib.bms_solve(ctx, 0.1, 1, 2, neg, 1e-8, 100, None, dummy, other, None) == bms.BMS_EINVAL
        o = bms.bms_opts()
        lib.bms_default_opts(ctypes.byref(o))
        o.qr_passes = 3
        assert lib.bms_solve(ctx, 0.1, 1, 2, sh, 1e-8, 100, ctypes.byref(o), dummy, other,
                             None) == bms.BMS_EINVAL
        lib.bms_default_opts(ctypes.byref(o))
        assert o.mixed_switch == 3e-4
        o.mixed_switch = float("nan")
        assert lib.bms_solve(ctx, 0.1, 1, 2, sh, 1e-8, 100, ctypes.byref(o), dummy, other,
                             None) == bms.BMS_EINVAL
        assert "mixed_switch" in lib.bms_last_error(ctx).decode()
        assert lib.bms_force(ctx, 1, 2, sh, dummy, other, 7) == bms.BMS_EINVAL
        assert lib.bms_set_gauge(ctx, None) == bms.BMS_EINVAL
        assert lib.bms_set_variant(ctx, bms.BMS_KERNEL_UPDATE, 9) == bms.BMS_EINVAL
        # well-formed calls need a gauge field first
        assert lib.bms_apply_hop(ctx, 1, 1, dummy, other, 0) == bms.BMS_ESTATE
        assert lib.bms_solve(ctx, 0.1, 1, 2, sh, 1e-8, 100, None, dummy, other, None) == bms.BMS_ESTATE
        assert lib.bms_force(ctx, 1, 2, sh, dummy, other, 0) == bms.BMS_ESTATE
        S = (ctypes.c_double * 1)()
        assert lib.bms_action(ctx, 1, 2, 1.0, sh, dummy, other, S) == bms.BMS_ESTATE
        assert "gauge" in lib.bms_last_error(ctx).decode()
        # host-only bookkeeping
        assert lib.bms_timing_enable(ctx, 1) == bms.BMS_OK
        ms, nl, by = ctypes.c_double(-1), ctypes.c_longlong(-1), ctypes.c_double(-1)
        assert lib.bms_timing_read(ctx, bms.BMS_KERNEL_HOP, ctypes.byref(ms), ctypes.byref(nl),
                                   ctypes.byref(by)) == bms.BMS_OK
        assert (ms.value, nl.value, by.value) == (0.0, 0, 0.0)
        assert lib.bms_timing_read(ctx, 99, None, None, None) == bms.BMS_EINVAL
        fl = ctypes.c_double(-1)
        assert lib.bms_timing_floor(ctx, bms.BMS_KERNEL_UPDATE, 8e12, 78.6e12, 157.3e12,
                                    ctypes.byref(fl)) == bms.BMS_OK
        assert fl.value == 0.0
        assert lib.bms_timing_floor(ctx, bms.BMS_KERNEL_UPDATE, 0.0, 1.0, 1.0,
                                    ctypes.byref(fl)) == bms.BMS_EINVAL
        assert lib.bms_timing_floor(ctx, 99, 1.0, 1.0, 1.0, ctypes.byref(fl)) == bms.BMS_EINVAL
        assert lib.bms_timing_floor(ctx, 0, 1.0, 1.0, 1.0, None) == bms.BMS_EINVAL
        rows = ctypes.c_int(0)
        dev = ctypes.c_double(0)
        assert lib.bms_get_link_rows(ctx, ctypes.byref(rows), ctypes.byref(dev)) == bms.BMS_OK
        assert rows.value == 3 and dev.value == -1.0
        assert lib.bms_get_link_rows(ctx, None, None) == bms.BMS_EINVAL
        assert lib.bms_set_link_rows(ctx, 4) == bms.BMS_EINVAL
        assert lib.bms_set_link_rows(ctx, 3) == bms.BMS_OK
        assert lib.bms_set_link_rows(ctx, 2) == bms.BMS_OK
        assert lib.bms_set_variant(ctx, bms.BMS_KERNEL_UPDATE, 1) == bms.BMS_OK
    finally:
        assert lib.bms_destroy(ctx) == bms.BMS_OK


def test_null_context(lib):
    assert lib.bms_destroy(None) == bms.BMS_EINVAL
    assert lib.bms_set_gauge(None, None) == bms.BMS_EINVAL
    assert lib.bms_last_error(None) == b""


def test_driver_entry_points_reject_bad_calls(lib):
    rc, ctx = _create(lib, (4, 4, 4, 4))
    rc2, ctx2 = _create(lib, (2, 2, 2, 2))
    assert rc == bms.BMS_OK and rc2 == bms.BMS_OK
    try:
        v = ctypes.c_int(-5)
        assert lib.bms_get_variant(ctx, bms.BMS_KERNEL_UPDATE, ctypes.byref(v)) == bms.BMS_OK
        assert v.value == -1
        assert lib.bms_get_variant(ctx, bms.BMS_KERNEL_SMALL, ctypes.byref(v)) == bms.BMS_EINVAL
        assert lib.bms_get_variant(None, 0, ctypes.byref(v)) == bms.BMS_EINVAL
        sh = (ctypes.c_double * 2)(0.1, 0.2)
        dummy, other = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000)
        assert lib.bms_autotune(ctx, 0.1, 1, 2, sh, bms.BMS_PREC_F32, 8, dummy, other) == bms.BMS_EINVAL
        assert lib.bms_autotune(ctx, 0.1, 1, 2, sh, bms.BMS_PREC_F64, 0, dummy, other) == bms.BMS_EINVAL
        # well-formed but no gauge field: the solve it runs fails on the host
        assert lib.bms_autotune(ctx, 0.1, 1, 2, sh, bms.BMS_PREC_F64, 8, dummy, other) == bms.BMS_ESTATE
        # batch: argument checks, then per-problem status
        k = 2
        vp = ctypes.c_void_p
        ctxs = (vp * k)(ctx.value, ctx2.value)
        mass = (ctypes.c_double * k)(0.1, 0.1)
        n = (ctypes.c_int * k)(1, 1)
        nsh = (ctypes.c_int * k)(2, 2)
        shp = (ctypes.POINTER(ctypes.c_double) * k)(ctypes.cast(sh, ctypes.POINTER(ctypes.c_double)),
                                                     ctypes.cast(sh, ctypes.POINTER(ctypes.c_double)))
        tol = (ctypes.c_double * k)(1e-8, 1e-8)
        mi = (ctypes.c_int * k)(100, 100)
        Bp = (vp * k)(0x1000, 0x3000)
        Xp = (vp * k)(0x2000, 0x4000)
        status = (ctypes.c_int * k)(7, 7)
        args = [mass, n, nsh, shp, tol, mi, None, Bp, Xp, None, status]
        assert lib.bms_solve_batch(0, ctxs, *args) == bms.BMS_EINVAL
        same = (vp * k)(ctx.value, ctx.value)
        assert lib.bms_solve_batch(k, same, *args) == bms.BMS_EINVAL
        assert lib.bms_solve_batch(k, ctxs, *args) == bms.BMS_ESTATE
        assert list(status) == [bms.BMS_ESTATE, bms.BMS_ESTATE]
    finally:
        assert lib.bms_destroy(ctx) == bms.BMS_OK
        assert lib.bms_destroy(ctx2) == bms.BMS_OK
