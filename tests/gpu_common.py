"""Shared helpers of the GPU parity tests (imported by test modules only)."""
import numpy as np
import pytest

SIGMA_FLOOR = np.array([2.0, 0.5, 0.5, 0.3])

# u*_0 tolerance: per-channel relative error floored by the noise scale,
# e = max_c |u_gpu - u_ref| / max(|u_ref|, sigma_c), gated at 1e-4 for the
# float32 path against the float64 oracle.
U0_TOL = 1e-4


def u0_error(u_gpu, u_ref):
    return float(np.max(np.abs(np.asarray(u_gpu) - u_ref) / np.maximum(np.abs(u_ref), SIGMA_FLOOR)))


def seq_error(U_gpu, U_ref):
    return float(np.max(np.abs(U_gpu - U_ref) / np.maximum(np.abs(U_ref), SIGMA_FLOOR[None, :])))


def require_gpu():
    try:
        import torch
    except Exception:
        pytest.skip("torch missing")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_07199_amd import mppi as M
    M.load_library()      # raises if the HIP library is missing: no fallback
    return M


def say(*a):
    print(*a, flush=True)
