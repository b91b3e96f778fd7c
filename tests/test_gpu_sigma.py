"""Full (non-diagonal) noise covariance through the C ABI.

Section IV-A draws the control perturbations from N(0, Sigma); the library
samples L n with L L^T = Sigma (host Cholesky factor in float64, rounded to
float32 once).  Every other parity test uses a diagonal Sigma, so this file
covers the off-diagonal part of the factor and of the sampling:

* plain FP32 path: the sampled controls element by element against the
  oracle's (its own factor of Sigma), positions, field values, costs and
  u*_0 at the float32 tolerance;
* fused BF16X3 and F16X2 on the two-hidden-layer decoder: u*_0, per-rollout
  costs and the per-query field values against the ``bf16w`` contract;
* a singular positive semi-definite Sigma (rank 3 and rank 2): both sides
  accept it and factor it the same way (a zero pivot leaves its column
  zero), which the element-wise sample check pins.
"""
import numpy as np
import pytest

import oracle
import scenarios as sc
from gpu_common import U0_TOL, require_gpu, say, u0_error

pytestmark = pytest.mark.gpu


def _within(name, got, want, tol):
    d = np.abs(np.asarray(got, dtype=np.float64) - want)
    bad = ~(d <= tol)
    assert not bad.any(), f"{name}: {int(bad.sum())} of {d.size} out of tolerance, max |diff| {d.max():.3e}"


@pytest.mark.parametrize("rank", [4, 3, 2])
def test_plain_full_sigma_elementwise(rank):
    M = require_gpu()
    layers = (67, 128, 128, 1)
    W, b = sc.xavier_weights(layers, seed=0)
    eng = M.Engine((W, b), sc.MODEL, K_max=512, T_max=24, G_max=2, hidden=128, n_hidden=2,
                   precision="fp32", path="plain", budget=256 << 20)
    errs = []
    for seed in (1, 2):
        Sig = sc.correlated_sigma(10 * rank + seed, rank=rank)
        prob = sc.make_problem(512, 24, 2, rot="haar", start="moving", seed=seed, d_safe=1.0,
                               Sigma=Sig, instance_id=100 * rank + seed)
        ref = oracle.solve(prob, (W, b), sc.MODEL)
        out = eng.step(prob, exports=True)
        assert out["rc"] == 0, out["rc"]
        _within("samples", out["samples"], ref["samples"], 2e-6 * (np.abs(ref["samples"]) + 1.0))
        _within("positions", out["p_rel"], ref["p_rel"], 2e-5 + 2e-6 * np.abs(ref["p_rel"]))
        _within("sdf", out["sdf"], ref["sdf"], 2e-5 * (1.0 + np.abs(ref["sdf"])))
        _within("J", out["J"], ref["J"], 2e-6 * (np.abs(ref["J"]) + prob["Q_sdf"] * prob["T"] + 1.0))
        # the sampled noise carries the correlations of Sigma (a coarse check
        # that the off-diagonal entries reach the samples at all)
        dev = (ref["samples"] - ref["samples"].mean(axis=(0, 1))).reshape(-1, 4)
        emp = dev.T @ dev / dev.shape[0]
        if rank == 4:
            assert np.abs(emp[0, 1] / np.sqrt(emp[0, 0] * emp[1, 1]) - Sig[0, 1] / np.sqrt(Sig[0, 0] * Sig[1, 1])) < 0.1
        errs.append(u0_error(out["u0"], ref["u0"]))
    say(f"plain full Sigma rank {rank}: u0 errors {['%.2e' % e for e in errs]}")
    assert max(errs) <= U0_TOL
    eng.close()


@pytest.mark.parametrize("precision", ["bf16x3", "f16x2"])
def test_fused_full_sigma(precision):
    M = require_gpu()
    layers = (67, 256, 256, 256, 1)
    W, b = sc.xavier_weights(layers, seed=2, bias_scale=0.2)
    eng = M.Engine((W, b), sc.MODEL, K_max=1024, T_max=30, G_max=4, hidden=256, n_hidden=3,
                   precision=precision, path="fused", budget=256 << 20)
    for rank, seed in ((4, 1), (3, 2)):
        Sig = sc.correlated_sigma(50 + seed, rank=rank)
        prob = sc.make_problem(1000, 30, 4, rot="yaw", start="moving", seed=seed, d_safe=1.0,
                               Sigma=Sig, instance_id=900 + seed)
        ref = oracle.solve(prob, (W, b), sc.MODEL, contract="bf16w")
        out = eng.step(prob, exports=True)
        assert out["rc"] == 0, out["rc"]
        e = u0_error(out["u0"], ref["u0"])
        ds = np.abs(out["sdf"] - ref["sdf"])
        say(f"fused {precision} full Sigma rank {rank}: u0 err {e:.2e}, max |ds| {ds.max():.2e}")
        _within("sdf", out["sdf"], ref["sdf"], 2e-5 * (1.0 + np.abs(ref["sdf"])))
        _within("J", out["J"], ref["J"], 2e-5 * (np.abs(ref["J"]) + prob["Q_sdf"] * prob["T"] + 1.0))
        assert e <= U0_TOL
    eng.close()


def test_sigma_not_psd_rejected_by_both():
    """A symmetric Sigma with a negative eigenvalue: the oracle raises and
    the library returns EINVAL."""
    M = require_gpu()
    Sig = np.diag([4.0, 0.25, 0.25, 0.09])
    Sig[0, 1] = Sig[1, 0] = 1.5        # correlation 1.5: not positive semi-definite
    with pytest.raises(ValueError):
        oracle.mppi.noise_factor(Sig)
    W, b = sc.xavier_weights((67, 128, 128, 1), seed=0)
    with M.Engine((W, b), sc.MODEL, K_max=64, T_max=8, G_max=1, hidden=128, n_hidden=2,
                  precision="fp32", path="plain", budget=64 << 20) as eng:
        prob = sc.make_problem(64, 8, 1, seed=1, Sigma=Sig)
        assert eng.step(prob)["rc"] == M.MPPI_EINVAL
