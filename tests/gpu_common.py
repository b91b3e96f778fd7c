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


def adjudicate(prob, ref, sdf_gpu, tol):
    """Parity under a rounding contract (``bf16``, ``fp8``) where several
    results are correct.  ``ref`` is ``oracle.solve(..., near_ties=True)``:
    at a position whose activations hold near ties (``near_tie`` > 0) each
    value in ``sdf_alts`` comes from a legitimate rounding, else the field is
    unique.  Checks that every device field value is legitimate (within
    ``tol`` of one of those values) and returns the oracle's own update for
    the device's choice of roundings: at each near-tie position the oracle
    value closest to the device's.

    Returns (update dict, info): info["ties"] positions with near ties,
    info["flipped"] positions where the device took another rounding than
    the oracle's own, info["bad"] positions whose device value matches no
    legitimate value within tol, info["worst"] the largest |device - chosen|
    and info["noisy"] the positions where it exceeds a quarter of tol."""
    from oracle.mppi import costs_and_update

    s_gpu = np.asarray(sdf_gpu, dtype=np.float64)
    s = ref["sdf"]
    T = s.shape[1]
    tol = np.broadcast_to(tol, s.shape)
    s_adj = s.copy()
    for q, vals in ref["sdf_alts"].items():
        k, t = divmod(q, T)
        s_adj[k, t] = vals[np.argmin(np.abs(vals - s_gpu[k, t]))]
    d = np.abs(s_gpu - s_adj)
    info = {"ties": int(np.count_nonzero(ref["near_tie"])), "flipped": int(np.sum(np.abs(s_adj - s) > tol)),
            "bad": int(np.sum(d > tol)), "worst": float(d.max()), "noisy": int(np.sum(d > 0.25 * tol))}
    adj = costs_and_update(prob, ref["samples"], ref["p_rel"], ref["q"], s_adj, prob.get("U_nom"))
    return adj, info


def float32_floor(ref, prob, scale, ulps=4):
    """How far float32 cost arithmetic alone can move u*_0, to first order,
    in the metric of u0_error: every rollout cost J_k may carry an error of
    ``ulps`` float32 units of its magnitude ``scale[k]`` (eps_k = ulps 2^-24
    scale_k), and dU*_0 / dJ_k = -(w_k / lambda) (u_k,0 - U*_0), so
    |dU*_0,c| <= sum_k (w_k / lambda) |u_k,0,c - U*_0,c| eps_k.  Computed from
    the oracle's own weights and samples."""
    w = ref["w"]
    du = np.abs(ref["samples"][:, 0, :] - ref["u0"][None, :])
    eps = ulps * 2.0 ** -24 * np.asarray(scale, dtype=np.float64)
    bound = np.sum((w * eps / prob["lam"])[:, None] * du, axis=0)
    return float(np.max(bound / np.maximum(np.abs(ref["u0"]), SIGMA_FLOOR)))
