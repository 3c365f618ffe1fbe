"""Host-only checks of the C ABI: the library loads, exports every entry point
declared in include/vp4d.h, and rejects bad arguments before touching the
device (no kernel is launched here)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vp4d.h")


def _lib():
    from paper_1803_02143_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        from paper_1803_02143_amd import build
        build.build()
    return L, L.load()


def declared_functions():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^VP4D_API\s+[\w\s\*]*?\b(\w+)\s*\(", src, re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("sldg_advect", "spline_advect", "vp_density", "vp_poisson",
              "vp_strang_step", "vp_moments", "vp_init", "vp_create", "vp_destroy",
              "vp_last_error"):
        assert n in names


def test_every_declared_symbol_is_exported():
    L, lib = _lib()
    for n in declared_functions():
        assert hasattr(lib, n), n
        assert n in L.SIGNATURES, f"binding lacks {n}"


def test_version_and_empty_error():
    _, lib = _lib()
    assert lib.vp_version().decode().startswith("vp4d")


def _fake(n=4096):
    # host buffers stand in for device pointers: validation fails before any use
    return ctypes.create_string_buffer(n)


def test_sldg_argument_errors():
    L, lib = _lib()
    dims = L.i64x4((6, 6, 6, 6))
    st = L.i64x4((0, 0, 1, 0))
    a, b, s = _fake(), _fake(), _fake()
    pa, pb, ps = (ctypes.cast(x, ctypes.c_void_p) for x in (a, b, s))
    assert lib.sldg_advect(4, 2, L.VP_F64, dims, pa, pb, ps, st, None) == L.VP_ERR_ARG
    assert "axis" in lib.vp_last_error().decode()
    assert lib.sldg_advect(0, 7, L.VP_F64, dims, pa, pb, ps, st, None) == L.VP_ERR_UNSUPPORTED
    assert lib.sldg_advect(0, 3, L.VP_F64, dims, pa, pb, ps, st, None) == L.VP_ERR_ARG  # 6 % 4
    assert lib.sldg_advect(0, 2, 5, dims, pa, pb, ps, st, None) == L.VP_ERR_ARG
    assert lib.sldg_advect(0, 2, L.VP_F64, dims, None, pb, ps, st, None) == L.VP_ERR_ARG
    assert lib.sldg_advect(0, 2, L.VP_F64, dims, pa, pa, ps, st, None) == L.VP_ERR_ALIAS
    bad = L.i64x4((1, 0, 0, 0))      # stride along the swept axis
    assert lib.sldg_advect(0, 2, L.VP_F64, dims, pa, pb, ps, bad, None) == L.VP_ERR_ARG
    neg = L.i64x4((0, -1, 0, 0))
    assert lib.sldg_advect(0, 2, L.VP_F64, dims, pa, pb, ps, neg, None) == L.VP_ERR_ARG
    zero = L.i64x4((6, 0, 6, 6))
    assert lib.sldg_advect(0, 2, L.VP_F64, zero, pa, pb, ps, st, None) == L.VP_ERR_ARG


def test_spline_and_field_argument_errors():
    L, lib = _lib()
    dims = L.i64x4((6, 6, 6, 6))
    st = L.i64x4((0, 0, 1, 0))
    a, b = _fake(), _fake()
    pa, pb = (ctypes.cast(x, ctypes.c_void_p) for x in (a, b))
    assert lib.spline_advect(-1, 3, L.VP_F32, dims, pa, pb, pa, st, None) == L.VP_ERR_ARG
    assert lib.spline_advect(0, 3, L.VP_F32, dims, pa, pa, pb, st, None) == L.VP_ERR_ALIAS
    for deg in (2, 1, 5, -1):
        assert lib.spline_advect(0, deg, L.VP_F32, dims, pa, pb, pa, st, None) == \
            L.VP_ERR_UNSUPPORTED
        assert "cubic" in lib.vp_last_error().decode()
        assert lib.spline_advect_adjoint(0, deg, L.VP_F32, dims, pa, pb, pa, st, None) == \
            L.VP_ERR_UNSUPPORTED
        assert lib.spline_advect_dshift(0, deg, L.VP_F32, dims, pa, pb, pa, st, pb, None) == \
            L.VP_ERR_UNSUPPORTED
    assert lib.vp_density(-2, L.VP_F64, dims, pa, 1.0, 1.0, pb, None) == L.VP_ERR_UNSUPPORTED
    assert lib.vp_density(2, L.VP_F64, dims, pa, -1.0, 1.0, pb, None) == L.VP_ERR_ARG
    ws = lib.vp_poisson_workspace(2, 6, 6)
    assert ws >= 3 * 16 * 36
    assert lib.vp_poisson(2, 6, 6, 1.0, 1.0, pa, pb, pb, None, pa, ws, None) == L.VP_ERR_ALIAS
    c = _fake()
    pc = ctypes.cast(c, ctypes.c_void_p)
    d = _fake()
    pd = ctypes.cast(d, ctypes.c_void_p)
    assert lib.vp_poisson(2, 6, 6, 1.0, 1.0, pa, pb, pc, None, pd, ws - 1, None) == L.VP_ERR_WORKSPACE
    assert lib.vp_poisson(2, 7, 6, 1.0, 1.0, pa, pb, pc, None, pd, ws, None) == L.VP_ERR_ARG
    mws = lib.vp_moments_workspace(dims)
    assert mws == 4 * 8 * 36
    lo, ln = L.dblx4((0, 0, -1, -1)), L.dblx4((1, 1, 2, 2))
    assert lib.vp_moments(2, L.VP_F64, dims, pa, lo, ln, pb, pc, mws - 8, None) == L.VP_ERR_WORKSPACE
    assert lib.vp_init(9, 0.1, 0.5, 0.0, 2, L.VP_F64, dims, lo, ln, pa, None) == L.VP_ERR_ARG
    h = ctypes.c_void_p()
    assert lib.vp_create(ctypes.byref(h), 5, 2, L.VP_F64, dims, lo, ln) == L.VP_ERR_ARG
    assert lib.vp_create(ctypes.byref(h), 0, 9, L.VP_F64, dims, lo, ln) == L.VP_ERR_UNSUPPORTED
    assert lib.vp_strang_step(None, pa, pb, 1, 0.1, None, None, None) == L.VP_ERR_ARG


def test_adjoint_and_run_argument_errors():
    L, lib = _lib()
    dims = L.i64x4((6, 6, 6, 6))
    st = L.i64x4((0, 0, 1, 0))
    a, b, s, g = _fake(), _fake(), _fake(), _fake()
    pa, pb, ps, pg = (ctypes.cast(x, ctypes.c_void_p) for x in (a, b, s, g))
    assert lib.sldg_advect_adjoint(5, 2, L.VP_F64, dims, pa, pb, ps, st, None) == L.VP_ERR_ARG
    assert lib.sldg_advect_adjoint(0, 2, L.VP_F64, dims, pa, pa, ps, st, None) == L.VP_ERR_ALIAS
    assert lib.sldg_advect_dshift(0, 2, L.VP_F64, dims, pa, pb, ps, st, None, None) == L.VP_ERR_ARG
    assert lib.spline_advect_adjoint(0, 3, L.VP_F64, dims, pa, pa, ps, st, None) == L.VP_ERR_ALIAS
    assert lib.spline_advect_dshift(0, 3, 7, dims, pa, pb, ps, st, pg, None) == L.VP_ERR_ARG
    assert lib.vp_density_adjoint(2, L.VP_F64, dims, None, 1.0, 1.0, pa, 0, None) == L.VP_ERR_ARG
    assert lib.vp_density_adjoint(2, L.VP_F64, dims, pb, 0.0, 1.0, pa, 0, None) == L.VP_ERR_ARG
    ws = lib.vp_poisson_workspace(2, 6, 6)
    assert lib.vp_poisson_adjoint(2, 6, 6, 1.0, 1.0, pa, pb, pa, pg, ws, None) == L.VP_ERR_ALIAS
    assert lib.vp_strang_adjoint(None, pa, pb, 0.1, pg, 1 << 20, None) == L.VP_ERR_ARG
    assert lib.vp_energy_gradient(None, pa, pb, None, None) == L.VP_ERR_ARG
    assert lib.vp_strang_run(None, pa, pb, 4, 0.1, 2, None, None, None) == L.VP_ERR_ARG
    assert lib.vp_timing_select(None, 1) == L.VP_ERR_ARG


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_1803_02143_amd import _lib as L
    saved = L._LIB
    L._LIB = None
    try:
        with pytest.raises(OSError):
            L.load(str(tmp_path / "missing.so"))
    finally:
        L._LIB = saved


def test_noalloc_poisson_rejects_before_touching_the_device():
    # the allocation-free Poisson solve validates like vp_poisson and refuses
    # grids beyond its static scratch before any HIP call
    L, lib = _lib()
    a, b, c = _fake(), _fake(), _fake()
    pa, pb, pc = (ctypes.cast(x, ctypes.c_void_p) for x in (a, b, c))
    assert L.VP_POISSON_NOALLOC_MAX_POINTS == 512 * 512
    # (addresses far apart that are never dereferenced: the check fails first)
    far = [ctypes.c_void_p(k << 32) for k in (1, 2, 3)]
    assert lib.vp_poisson_noalloc(2, 516, 516, 1.0, 1.0, *far, None, None) == \
        L.VP_ERR_WORKSPACE
    assert "at most" in lib.vp_last_error().decode()
    assert lib.vp_poisson_noalloc(2, 7, 6, 1.0, 1.0, pa, pb, pc, None, None) == L.VP_ERR_ARG
    assert lib.vp_poisson_noalloc(2, 6, 6, 1.0, 1.0, pa, pb, pb, None, None) == L.VP_ERR_ALIAS
    assert lib.vp_poisson_noalloc(9, 6, 6, 1.0, 1.0, pa, pb, pc, None, None) == \
        L.VP_ERR_UNSUPPORTED



def test_copy_pattern_argument_errors():
    L, lib = _lib()
    dims = L.i64x4((6, 6, 6, 6))
    far = [ctypes.c_void_p(k << 32) for k in (1, 2)]
    assert lib.vp_copy_pattern(7, L.VP_F64, dims, 0, *far, None) == L.VP_ERR_ARG
    assert lib.vp_copy_pattern(L.VP_PATTERN_TILES, L.VP_F64, dims, 3, *far, None) == L.VP_ERR_ARG
    assert lib.vp_copy_pattern(L.VP_PATTERN_LINES, L.VP_F64, dims, 0, far[0], far[0], None) == \
        L.VP_ERR_ALIAS
    odd = ctypes.c_void_p((2 << 32) + 8)
    assert lib.vp_copy_pattern(L.VP_PATTERN_CONTIGUOUS, L.VP_F64, dims, 0, far[0], odd, None) == \
        L.VP_ERR_ARG
    long_lines = L.i64x4((400, 2, 2, 2))
    assert lib.vp_copy_pattern(L.VP_PATTERN_TILES, L.VP_F32, long_lines, 0, *far, None) == \
        L.VP_ERR_UNSUPPORTED
