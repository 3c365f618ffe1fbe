"""MI355X (gfx950) split-step semi-Lagrangian Vlasov-Poisson sweeps.

Thin Python binding of libvp4d.so: the functions below marshal torch
tensors (device memory) and the current HIP stream into the C ABI of
include/vp4d.h, with the same names.  Every step of the computation runs in
the library's HIP kernels; nothing here computes.

Method: L. Einkemmer, "A comparison of semi-Lagrangian discontinuous
Galerkin and spline based Vlasov solvers in four dimensions",
arXiv:1803.02143 (SLDG translate-and-project, Sec. 2-3; periodic cubic
spline, Sec. 3; Strang splitting, Sec. 2).
"""

import ctypes

import torch

from . import _lib
from ._lib import (VP_OK, VP_ERR_ARG, VP_ERR_UNSUPPORTED, VP_ERR_ALIAS,  # noqa: F401
                   VP_ERR_HIP, VP_ERR_WORKSPACE, VP_F32, VP_F64, TIMER_NAMES)

METHOD_SLDG = 0
METHOD_SPLINE = 1
IC_LANDAU = 0
IC_TWO_STREAM_SUM = 1
IC_TWO_STREAM_PRODUCT = 2


class VPError(RuntimeError):
    def __init__(self, func, status, message):
        self.status = status
        super().__init__(f"{func}: {_lib.STATUS_NAMES.get(status, status)}: {message}")


def lib():
    return _lib.load()


def _check(func, status):
    if status != VP_OK:
        msg = lib().vp_last_error()
        raise VPError(func, status, msg.decode() if msg else "")


def _dtype(t):
    if t.dtype == torch.float64:
        return VP_F64
    if t.dtype == torch.float32:
        return VP_F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _dev(t, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _f64(t, name, numel=None):
    p = _dev(t, name)
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} needs {numel} elements")
    return p


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dims(f):
    if f.dim() != 4:
        raise ValueError("f must be 4-dimensional (x1, x2, v1, v2)")
    return _lib.i64x4(f.shape)


def broadcast_strides(shift, axis):
    """Element strides of a 4D shift tensor, 0 along broadcast (size-1) axes."""
    if shift.dim() != 4:
        raise ValueError("pass shift_stride for a shift that is not 4-dimensional")
    st = [0 if shift.shape[d] == 1 else shift.stride(d) for d in range(4)]
    st[axis] = 0
    return st


def _check_shift(shift, dims, axis, shift_stride):
    need = 1 + sum((int(dims[d]) - 1) * int(shift_stride[d]) for d in range(4) if d != axis)
    if shift.numel() < need:
        raise ValueError(f"shift has {shift.numel()} elements, the strides need {need}")


def sldg_advect(axis, degree, f_in, f_out, shift, shift_stride=None, stream=None):
    """One SLDG sweep (C ABI ``sldg_advect``); shift in cells, float64."""
    if shift_stride is None:
        shift_stride = broadcast_strides(shift, axis)
    if f_in.dtype != f_out.dtype or f_in.shape != f_out.shape:
        raise ValueError("f_in and f_out must match in shape and dtype")
    _check_shift(shift, f_in.shape, axis, shift_stride)
    _check("sldg_advect", lib().sldg_advect(
        int(axis), int(degree), _dtype(f_in), _dims(f_in), _dev(f_in, "f_in"),
        _dev(f_out, "f_out"), _f64(shift, "shift"), _lib.i64x4(shift_stride),
        _stream(stream)))


def spline_advect(axis, f_in, f_out, shift, shift_stride=None, stream=None, degree=3):
    """One periodic cubic-spline sweep (C ABI ``spline_advect``; degree 3 only)."""
    if shift_stride is None:
        shift_stride = broadcast_strides(shift, axis)
    if f_in.dtype != f_out.dtype or f_in.shape != f_out.shape:
        raise ValueError("f_in and f_out must match in shape and dtype")
    _check_shift(shift, f_in.shape, axis, shift_stride)
    _check("spline_advect", lib().spline_advect(
        int(axis), int(degree), _dtype(f_in), _dims(f_in), _dev(f_in, "f_in"), _dev(f_out, "f_out"),
        _f64(shift, "shift"), _lib.i64x4(shift_stride), _stream(stream)))


def _lines_numel(f, axis):
    return f.numel() // f.shape[axis]


def sldg_advect_adjoint(axis, degree, lam_out, lam_in, shift, shift_stride=None, stream=None):
    """Transpose of the SLDG sweep for fixed shifts (C ABI ``sldg_advect_adjoint``)."""
    if shift_stride is None:
        shift_stride = broadcast_strides(shift, axis)
    if lam_out.dtype != lam_in.dtype or lam_out.shape != lam_in.shape:
        raise ValueError("lam_out and lam_in must match in shape and dtype")
    _check_shift(shift, lam_out.shape, axis, shift_stride)
    _check("sldg_advect_adjoint", lib().sldg_advect_adjoint(
        int(axis), int(degree), _dtype(lam_out), _dims(lam_out), _dev(lam_out, "lam_out"),
        _dev(lam_in, "lam_in"), _f64(shift, "shift"), _lib.i64x4(shift_stride),
        _stream(stream)))


def sldg_advect_dshift(axis, degree, f_in, lam_out, shift, g_line, shift_stride=None,
                       stream=None):
    """Per-line d<lam_out, sweep(f_in)>/d shift (C ABI ``sldg_advect_dshift``)."""
    if shift_stride is None:
        shift_stride = broadcast_strides(shift, axis)
    if f_in.dtype != lam_out.dtype or f_in.shape != lam_out.shape:
        raise ValueError("f_in and lam_out must match in shape and dtype")
    _check_shift(shift, f_in.shape, axis, shift_stride)
    _check("sldg_advect_dshift", lib().sldg_advect_dshift(
        int(axis), int(degree), _dtype(f_in), _dims(f_in), _dev(f_in, "f_in"),
        _dev(lam_out, "lam_out"), _f64(shift, "shift"), _lib.i64x4(shift_stride),
        _f64(g_line, "g_line", _lines_numel(f_in, axis)), _stream(stream)))


def spline_advect_adjoint(axis, lam_out, lam_in, shift, shift_stride=None, stream=None,
                          degree=3):
    """Transpose of the spline sweep for fixed shifts (C ABI ``spline_advect_adjoint``)."""
    if shift_stride is None:
        shift_stride = broadcast_strides(shift, axis)
    if lam_out.dtype != lam_in.dtype or lam_out.shape != lam_in.shape:
        raise ValueError("lam_out and lam_in must match in shape and dtype")
    _check_shift(shift, lam_out.shape, axis, shift_stride)
    _check("spline_advect_adjoint", lib().spline_advect_adjoint(
        int(axis), int(degree), _dtype(lam_out), _dims(lam_out), _dev(lam_out, "lam_out"),
        _dev(lam_in, "lam_in"), _f64(shift, "shift"), _lib.i64x4(shift_stride),
        _stream(stream)))


def spline_advect_dshift(axis, f_in, lam_out, shift, g_line, shift_stride=None, stream=None,
                         degree=3):
    """Per-line d<lam_out, spline sweep(f_in)>/d shift (C ABI ``spline_advect_dshift``)."""
    if shift_stride is None:
        shift_stride = broadcast_strides(shift, axis)
    if f_in.dtype != lam_out.dtype or f_in.shape != lam_out.shape:
        raise ValueError("f_in and lam_out must match in shape and dtype")
    _check_shift(shift, f_in.shape, axis, shift_stride)
    _check("spline_advect_dshift", lib().spline_advect_dshift(
        int(axis), int(degree), _dtype(f_in), _dims(f_in), _dev(f_in, "f_in"), _dev(lam_out, "lam_out"),
        _f64(shift, "shift"), _lib.i64x4(shift_stride),
        _f64(g_line, "g_line", _lines_numel(f_in, axis)), _stream(stream)))


def vp_density_adjoint(degree, rho_bar, len_v1, len_v2, lam, accumulate=False, stream=None):
    """lam (+)= rho_bar W3 W4 (C ABI ``vp_density_adjoint``)."""
    if rho_bar.numel() < lam.shape[0] * lam.shape[1]:
        raise ValueError("rho_bar too small")
    _check("vp_density_adjoint", lib().vp_density_adjoint(
        int(degree), _dtype(lam), _dims(lam), _f64(rho_bar, "rho_bar"), float(len_v1),
        float(len_v2), _dev(lam, "lam"), 1 if accumulate else 0, _stream(stream)))


def vp_poisson_adjoint(degree, L1, L2, G1, G2, rho_bar, workspace=None, stream=None):
    """rho_bar = P_1^T G1 + P_2^T G2 (C ABI ``vp_poisson_adjoint``)."""
    n1, n2 = G1.shape
    ws_bytes = vp_poisson_workspace(degree, n1, n2)
    if workspace is None:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=G1.device)
    _check("vp_poisson_adjoint", lib().vp_poisson_adjoint(
        int(degree), int(n1), int(n2), float(L1), float(L2), _f64(G1, "G1", n1 * n2),
        _f64(G2, "G2", n1 * n2), _f64(rho_bar, "rho_bar", n1 * n2),
        _dev(workspace, "workspace"), workspace.numel() * workspace.element_size(),
        _stream(stream)))


def vp_density(degree, f, len_v1, len_v2, rho, stream=None):
    """rho[x1][x2] = int f dv (C ABI ``vp_density``); degree -1 = spline grid."""
    _check("vp_density", lib().vp_density(
        int(degree), _dtype(f), _dims(f), _dev(f, "f"), float(len_v1), float(len_v2),
        _f64(rho, "rho", f.shape[0] * f.shape[1]), _stream(stream)))


def vp_poisson_workspace(degree, n1, n2):
    return int(lib().vp_poisson_workspace(int(degree), int(n1), int(n2)))


def vp_poisson(degree, L1, L2, rho, E1, E2, W_el=None, workspace=None, stream=None):
    """E and W = 1/2 int |E|^2 from rho (C ABI ``vp_poisson``)."""
    n1, n2 = rho.shape
    ws_bytes = vp_poisson_workspace(degree, n1, n2)
    if workspace is None:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=rho.device)
    _check("vp_poisson", lib().vp_poisson(
        int(degree), int(n1), int(n2), float(L1), float(L2), _f64(rho, "rho"),
        _f64(E1, "E1", n1 * n2), _f64(E2, "E2", n1 * n2),
        None if W_el is None else _f64(W_el, "W_el", 1),
        _dev(workspace, "workspace"), workspace.numel() * workspace.element_size(),
        _stream(stream)))


def vp_poisson_noalloc(degree, L1, L2, rho, E1, E2, W_el=None, stream=None):
    """vp_poisson without a workspace (C ABI ``vp_poisson_noalloc``): the
    library's static device scratch, at most 512 x 512 points."""
    n1, n2 = rho.shape
    _check("vp_poisson_noalloc", lib().vp_poisson_noalloc(
        int(degree), int(n1), int(n2), float(L1), float(L2), _f64(rho, "rho"),
        _f64(E1, "E1", n1 * n2), _f64(E2, "E2", n1 * n2),
        None if W_el is None else _f64(W_el, "W_el", 1), _stream(stream)))


def vp_moments_workspace(dims):
    return int(lib().vp_moments_workspace(_lib.i64x4(dims)))


def vp_moments(degree, f, lo, length, out4, workspace=None, stream=None):
    """mass, L1, L2, kinetic energy (C ABI ``vp_moments``)."""
    ws_bytes = vp_moments_workspace(f.shape)
    if workspace is None:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=f.device)
    _check("vp_moments", lib().vp_moments(
        int(degree), _dtype(f), _dims(f), _dev(f, "f"), _lib.dblx4(lo),
        _lib.dblx4(length), _f64(out4, "out4", 4), _dev(workspace, "workspace"),
        workspace.numel() * workspace.element_size(), _stream(stream)))


def vp_init(kind, eps, k, v0, degree, f, lo, length, stream=None):
    """Sample an initial condition at the nodes (C ABI ``vp_init``)."""
    _check("vp_init", lib().vp_init(
        int(kind), float(eps), float(k), float(v0), int(degree), _dtype(f), _dims(f),
        _lib.dblx4(lo), _lib.dblx4(length), _dev(f, "f"), _stream(stream)))


class VPState:
    """A solver instance (C ABI ``vp_create`` / ``vp_strang_step``)."""

    def __init__(self, method, degree, dtype, dims, lo, length):
        self._h = ctypes.c_void_p()
        dt = VP_F64 if dtype in (torch.float64, "f64") else VP_F32
        _check("vp_create", lib().vp_create(
            ctypes.byref(self._h), int(method), int(degree), dt, _lib.i64x4(dims),
            _lib.dblx4(lo), _lib.dblx4(length)))
        self.method, self.degree, self.dims = method, degree, tuple(int(d) for d in dims)
        self.dtype = torch.float64 if dt == VP_F64 else torch.float32

    def close(self):
        if self._h:
            lib().vp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, f, f_tmp, nsteps, tau, W_trace=None, moments=None, stream=None):
        for t, n in ((f, "f"), (f_tmp, "f_tmp")):
            if tuple(t.shape) != self.dims or t.dtype != self.dtype:
                raise ValueError(f"{n} must be {self.dtype} of shape {self.dims}")
        _check("vp_strang_step", lib().vp_strang_step(
            self._h, _dev(f, "f"), _dev(f_tmp, "f_tmp"), int(nsteps), float(tau),
            None if W_trace is None else _f64(W_trace, "W_trace", nsteps + 1),
            None if moments is None else _f64(moments, "moments", 4 * (nsteps + 1)),
            _stream(stream)))

    def run(self, f, f_tmp, nsteps, tau, diag_every, W_trace=None, moments=None, stream=None):
        """``nsteps`` Strang steps with merged x half-steps between the states
        f^0, f^{diag_every}, ... (``vp_strang_run``)."""
        for t, n in ((f, "f"), (f_tmp, "f_tmp")):
            if tuple(t.shape) != self.dims or t.dtype != self.dtype:
                raise ValueError(f"{n} must be {self.dtype} of shape {self.dims}")
        nd = nsteps // diag_every + 1 if diag_every > 0 else 1
        _check("vp_strang_run", lib().vp_strang_run(
            self._h, _dev(f, "f"), _dev(f_tmp, "f_tmp"), int(nsteps), float(tau),
            int(diag_every),
            None if W_trace is None else _f64(W_trace, "W_trace", nd),
            None if moments is None else _f64(moments, "moments", 4 * nd),
            _stream(stream)))

    def _check_f(self, t, name):
        if tuple(t.shape) != self.dims or t.dtype != self.dtype:
            raise ValueError(f"{name} must be {self.dtype} of shape {self.dims}")

    def adjoint_workspace_bytes(self):
        return int(lib().vp_strang_adjoint_workspace(self._h))

    def adjoint_workspace(self, device="cuda"):
        return torch.empty(self.adjoint_workspace_bytes(), dtype=torch.uint8, device=device)

    def adjoint_step(self, f, lam, tau, work, stream=None):
        """lam: dJ/df^{m+1} in, dJ/df^m out, for the step from f = f^m."""
        self._check_f(f, "f")
        self._check_f(lam, "lam")
        _check("vp_strang_adjoint", lib().vp_strang_adjoint(
            self._h, _dev(f, "f"), _dev(lam, "lam"), float(tau), _dev(work, "work"),
            work.numel() * work.element_size(), _stream(stream)))

    def energy_gradient(self, f, lam, W=None, stream=None):
        """lam = dW/df (and W) for W = 1/2 int |E(f)|^2."""
        self._check_f(f, "f")
        self._check_f(lam, "lam")
        _check("vp_energy_gradient", lib().vp_energy_gradient(
            self._h, _dev(f, "f"), _dev(lam, "lam"),
            None if W is None else _f64(W, "W", 1), _stream(stream)))

    def timing_enable(self, on=True):
        _check("vp_timing_enable", lib().vp_timing_enable(self._h, 1 if on else 0))

    def timing_select(self, names):
        """Time only the named categories (keys of ``timing_read``)."""
        mask = 0
        for n in names:
            if n not in TIMER_NAMES:
                raise ValueError(f"unknown timer {n!r}; known: {TIMER_NAMES}")
            mask |= 1 << TIMER_NAMES.index(n)
        _check("vp_timing_select", lib().vp_timing_select(self._h, mask))

    def timing_read(self):
        """{timer name: (total ms, launches)} since the last read."""
        ms = (ctypes.c_double * _lib.VP_TIMER_COUNT)()
        cnt = (ctypes.c_int64 * _lib.VP_TIMER_COUNT)()
        _check("vp_timing_read", lib().vp_timing_read(self._h, ms, cnt))
        return {TIMER_NAMES[i]: (ms[i], cnt[i]) for i in range(_lib.VP_TIMER_COUNT)}


PATTERN_CONTIGUOUS = _lib.VP_PATTERN_CONTIGUOUS
PATTERN_TILES = _lib.VP_PATTERN_TILES
PATTERN_SEGMENTS = _lib.VP_PATTERN_SEGMENTS
PATTERN_LINES = _lib.VP_PATTERN_LINES


def vp_copy_pattern(pattern, f_in, f_out, axis=0, stream=None):
    """f_out = f_in with the access pattern of a sweep family (C ABI
    ``vp_copy_pattern``): a bandwidth reference for the sweeps."""
    if f_in.dtype != f_out.dtype or f_in.shape != f_out.shape:
        raise ValueError("f_in and f_out must match in shape and dtype")
    _check("vp_copy_pattern", lib().vp_copy_pattern(
        int(pattern), _dtype(f_in), _dims(f_in), int(axis), _dev(f_in, "f_in"),
        _dev(f_out, "f_out"), _stream(stream)))


def version():
    return lib().vp_version().decode()
