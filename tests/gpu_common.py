"""Helpers for the GPU parity tests (imported by tests marked ``gpu``)."""

import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")


def require_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    import paper_1803_02143_amd as vp
    vp.lib()              # raises if libvp4d.so is missing: no fallback
    return vp


def announce(msg):
    sys.stdout.write(f"\n[case] {msg}\n")
    sys.stdout.flush()


TORCH_DTYPE = {"f64": torch.float64, "f32": torch.float32}
NP_DTYPE = {"f64": np.float64, "f32": np.float32}


def to_dev(a, dt="f64"):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=NP_DTYPE[dt])).cuda()


def to_host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def rel_l2(a, b):
    d = np.linalg.norm((a - b).ravel())
    n = np.linalg.norm(b.ravel())
    return d / n if n > 0 else d


def rel_max(a, b):
    m = np.max(np.abs(b))
    return np.max(np.abs(a - b)) / m if m > 0 else np.max(np.abs(a - b))


def assert_close(gpu, ref, dt, what=""):
    """FP64: 1e-12 relative in max and L2 norms; FP32: 1e-5 relative L2."""
    if dt == "f64":
        e1, e2 = rel_max(gpu, ref), rel_l2(gpu, ref)
        assert e1 <= 1e-12 and e2 <= 1e-12, f"{what}: rel max {e1:.3e}, rel L2 {e2:.3e}"
    else:
        e = rel_l2(gpu, ref)
        assert e <= 1e-5, f"{what}: rel L2 {e:.3e}"
