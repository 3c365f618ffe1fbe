"""The allocation-free Poisson entry point against vp_poisson.

vp_poisson_noalloc runs the same kernels as vp_poisson with the library's
static device scratch in place of a caller workspace; two calls in a row,
the second on a smaller grid (and another degree), must give vp_poisson's
results, and a grid beyond the static maximum is refused."""

import ctypes
import math

import numpy as np
import pytest

from gpu_common import announce, require_gpu, to_dev, to_host, torch
from vp_inputs import random_field

pytestmark = pytest.mark.gpu


def _both(vp, degree, n1, n2, L1, L2, seed):
    rho = to_dev(1.0 + 0.3 * random_field((n1, n2), seed=seed))
    out = {}
    for name in ("vp_poisson", "vp_poisson_noalloc"):
        E1 = torch.full((n1, n2), float("nan"), dtype=torch.float64, device="cuda")
        E2 = torch.full((n1, n2), float("nan"), dtype=torch.float64, device="cuda")
        W = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        getattr(vp, name)(degree, L1, L2, rho, E1, E2, W)
        out[name] = (to_host(E1), to_host(E2), to_host(W))
    return out


def test_noalloc_poisson_matches_vp_poisson_on_two_calls():
    vp = require_gpu()
    L1, L2 = 4 * math.pi, 10 * math.pi
    cases = [(2, 288, 192, 11), (-1, 96, 80, 12)]      # second call smaller
    for degree, n1, n2, seed in cases:
        announce(f"vp_poisson_noalloc degree={degree} {n1}x{n2}")
        out = _both(vp, degree, n1, n2, L1, L2, seed)
        ref, got = out["vp_poisson"], out["vp_poisson_noalloc"]
        for a, b in zip(got, ref):
            assert np.all(np.isfinite(a))
            # the same kernels in the same order: identical results
            assert np.array_equal(a, b)
        assert np.max(np.abs(ref[0])) > 0.0


def test_noalloc_poisson_refuses_grids_beyond_its_scratch():
    vp = require_gpu()
    n1 = n2 = 516              # 516^2 > 512^2 points
    rho = torch.ones(n1, n2, dtype=torch.float64, device="cuda")
    E1 = torch.empty_like(rho)
    E2 = torch.empty_like(rho)
    announce("vp_poisson_noalloc beyond the static maximum")
    with pytest.raises(vp.VPError) as exc:
        vp.vp_poisson_noalloc(2, 1.0, 1.0, rho, E1, E2)
    assert exc.value.status == vp.VP_ERR_WORKSPACE
    assert "at most" in str(exc.value)
    # the largest grid it takes (spline grid: any n), through the C ABI
    announce("vp_poisson_noalloc at the static maximum, 512 x 512")
    lib = vp.lib()
    rho = 1.0 + 0.1 * torch.rand(512, 512, dtype=torch.float64, device="cuda")
    E1 = torch.empty_like(rho)
    E2 = torch.empty_like(rho)
    st = lib.vp_poisson_noalloc(-1, 512, 512, 1.0, 1.0, ctypes.c_void_p(rho.data_ptr()),
                                ctypes.c_void_p(E1.data_ptr()), ctypes.c_void_p(E2.data_ptr()),
                                None, None)
    assert st == vp.VP_OK, lib.vp_last_error()
    F1 = torch.empty_like(rho)
    F2 = torch.empty_like(rho)
    vp.vp_poisson(-1, 1.0, 1.0, rho, F1, F2)
    assert torch.equal(E1, F1) and torch.equal(E2, F2)
