"""ctypes view of libvp4d.so (the C ABI declared in include/vp4d.h).

Loading never falls back to anything: if the shared library is missing the
import of the binding raises, and every call goes to the HIP library.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvp4d.so")

VP_OK = 0
VP_ERR_ARG = -1
VP_ERR_UNSUPPORTED = -2
VP_ERR_ALIAS = -3
VP_ERR_HIP = -4
VP_ERR_WORKSPACE = -5
STATUS_NAMES = {0: "VP_OK", -1: "VP_ERR_ARG", -2: "VP_ERR_UNSUPPORTED",
                -3: "VP_ERR_ALIAS", -4: "VP_ERR_HIP", -5: "VP_ERR_WORKSPACE"}

VP_F32 = 0
VP_F64 = 1
VP_TIMER_COUNT = 7
VP_POISSON_NOALLOC_MAX_POINTS = 512 * 512
VP_PATTERN_CONTIGUOUS = 0
VP_PATTERN_TILES = 1
VP_PATTERN_SEGMENTS = 2
VP_PATTERN_LINES = 3
TIMER_NAMES = ("sweep_x1", "sweep_x2", "sweep_v1", "sweep_v2", "field", "diag",
               "sweep_x2_rho")

_i64x4 = ctypes.c_int64 * 4
_dblx4 = ctypes.c_double * 4
_vp = ctypes.c_void_p
_dp = ctypes.c_void_p          # device double*, passed as an address

# name -> (restype, argtypes)
SIGNATURES = {
    "sldg_advect": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, _i64x4,
                                   _vp, _vp, _dp, _i64x4, _vp]),
    "spline_advect": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, _i64x4,
                                     _vp, _vp, _dp, _i64x4, _vp]),
    "vp_density": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _i64x4, _vp,
                                  ctypes.c_double, ctypes.c_double, _dp, _vp]),
    "vp_poisson": (ctypes.c_int, [ctypes.c_int, ctypes.c_int64, ctypes.c_int64,
                                  ctypes.c_double, ctypes.c_double, _dp, _dp, _dp, _dp,
                                  _vp, ctypes.c_size_t, _vp]),
    "vp_poisson_workspace": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_int64,
                                               ctypes.c_int64]),
    "vp_poisson_noalloc": (ctypes.c_int, [ctypes.c_int, ctypes.c_int64, ctypes.c_int64,
                                          ctypes.c_double, ctypes.c_double, _dp, _dp, _dp,
                                          _dp, _vp]),
    "vp_moments": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _i64x4, _vp, _dblx4,
                                  _dblx4, _dp, _vp, ctypes.c_size_t, _vp]),
    "vp_moments_workspace": (ctypes.c_size_t, [_i64x4]),
    "vp_init": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, ctypes.c_int, ctypes.c_int, _i64x4,
                               _dblx4, _dblx4, _vp, _vp]),
    "vp_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
                                 ctypes.c_int, ctypes.c_int, _i64x4, _dblx4, _dblx4]),
    "vp_destroy": (None, [_vp]),
    "vp_strang_step": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, ctypes.c_double,
                                      _dp, _dp, _vp]),
    "vp_strang_run": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, ctypes.c_double,
                                     ctypes.c_int, _dp, _dp, _vp]),
    "sldg_advect_adjoint": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, _i64x4,
                                           _vp, _vp, _dp, _i64x4, _vp]),
    "sldg_advect_dshift": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, _i64x4,
                                          _vp, _vp, _dp, _i64x4, _dp, _vp]),
    "spline_advect_adjoint": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                             _i64x4, _vp, _vp, _dp, _i64x4, _vp]),
    "spline_advect_dshift": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                            _i64x4, _vp, _vp, _dp, _i64x4, _dp, _vp]),
    "vp_density_adjoint": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _i64x4, _dp,
                                          ctypes.c_double, ctypes.c_double, _vp, ctypes.c_int,
                                          _vp]),
    "vp_poisson_adjoint": (ctypes.c_int, [ctypes.c_int, ctypes.c_int64, ctypes.c_int64,
                                          ctypes.c_double, ctypes.c_double, _dp, _dp, _dp,
                                          _vp, ctypes.c_size_t, _vp]),
    "vp_energy_gradient": (ctypes.c_int, [_vp, _vp, _vp, _dp, _vp]),
    "vp_strang_adjoint_workspace": (ctypes.c_size_t, [_vp]),
    "vp_strang_adjoint": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_double, _vp, ctypes.c_size_t,
                                         _vp]),
    "vp_timing_enable": (ctypes.c_int, [_vp, ctypes.c_int]),
    "vp_timing_select": (ctypes.c_int, [_vp, ctypes.c_uint]),
    "vp_timing_read": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_int64)]),
    "vp_copy_pattern": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _i64x4, ctypes.c_int, _vp,
                                       _vp, _vp]),
    "vp_last_error": (ctypes.c_char_p, []),
    "vp_version": (ctypes.c_char_p, []),
}

_LIB = None


def load(path=LIB_PATH):
    """The loaded library (raises OSError if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(path):
            raise OSError(f"{path} not found: build it with "
                          "`python -m paper_1803_02143_amd.build`")
        lib = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB


def i64x4(v):
    return _i64x4(*[int(x) for x in v])


def dblx4(v):
    return _dblx4(*[float(x) for x in v])
