"""Maximum sizes and the full fleet shape.

* The largest solve the engine accepts on the served decoder shape
  (K = 16384 rollouts, T = 64, G = 8, 67-256-256-256-1, BF16X3 and F16X2): the oracle
  cannot afford all of it in a test, so the per-rollout costs of the first
  64 rollouts are compared with an oracle run of a K = 64 problem (rollout k
  draws its noise from counter (k, t, instance, tick), so its samples and
  cost do not depend on K), and the rest is checked through properties that
  hold at any size: weights sum to one, the update is a convex combination
  of clipped samples, reruns of the same request (explicit tick and nominal
  sequence) are bitwise equal.
* One full solve of the fleet shape (K = 2048, T = 40, G = 8,
  67-512-512-512-1, BF16X3 and F16X2) against the complete oracle, and large lambda
  giving uniform weights (the softmax's degenerate limit) on the same shape.
"""
import numpy as np
import pytest

import oracle
import scenarios as sc
from gpu_common import U0_TOL, require_gpu, say, u0_error

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["bf16x3", "f16x2"])
def test_largest_solve_on_the_served_shape(precision):
    M = require_gpu()
    layers = (67, 256, 256, 256, 1)
    W, b = sc.xavier_weights(layers, seed=0)
    eng = M.Engine((W, b), sc.MODEL, K_max=16384, T_max=64, G_max=8, hidden=256, n_hidden=3,
                   precision=precision, path="fused", budget=1 << 30)
    U = oracle.hover_sequence(64, sc.MODEL["mass"], sc.MODEL["gravity"])
    prob = sc.make_problem(16384, 64, 8, rot="yaw", start="moving", seed=77, d_safe=1.0, instance_id=5, tick=2,
                           U_nom=U)
    out = eng.step(prob)
    assert out["rc"] == 0
    assert abs(out["w"].sum() - 1.0) < 1e-12 and np.all(out["w"] >= 0.0)
    assert 1.0 <= out["ess"] <= 16384.0
    assert np.all(out["U_star"] >= sc.MODEL["u_lo"] - 1e-12) and np.all(out["U_star"] <= sc.MODEL["u_hi"] + 1e-12)
    sub = dict(prob, K=64)
    ref = oracle.solve(sub, (W, b), sc.MODEL, contract="bf16w")
    rel = np.abs(out["J"][:64] - ref["J"]) / (np.abs(ref["J"]) + prob["Q_sdf"] * prob["T"] + 1.0)
    say(f"{precision} K=16384 T=64 G=8: first 64 costs max rel err {rel.max():.1e}, ess {out['ess']:.1f}")
    assert rel.max() <= 2e-5
    again = eng.step(prob)
    assert np.array_equal(again["U_star"], out["U_star"]) and np.array_equal(again["J"], out["J"])
    eng.close()


@pytest.mark.parametrize("precision", ["bf16x3", "f16x2"])
def test_full_fleet_shape_solve_and_uniform_limit(precision):
    M = require_gpu()
    layers = (67, 512, 512, 512, 1)
    W, b = sc.xavier_weights(layers, seed=0)
    eng = M.Engine((W, b), sc.MODEL, K_max=2048, T_max=40, G_max=8, hidden=512, n_hidden=3,
                   precision=precision, path="fused", budget=1 << 30)
    prob = sc.config_problem("S2", 3, d_safe=1.0, instance_id=11)
    ref = oracle.solve(prob, (W, b), sc.MODEL, contract="bf16w")
    out = eng.step(prob)
    assert out["rc"] == 0
    e = u0_error(out["u0"], ref["u0"])
    dJ = np.abs(out["J"] - ref["J"]) / (np.abs(ref["J"]) + prob["Q_sdf"] * prob["T"] + 1.0)
    say(f"{precision} fleet shape K=2048 T=40 G=8 H=512: u0 err {e:.2e}, max rel dJ {dJ.max():.1e}")
    assert e <= U0_TOL and dJ.max() <= 2e-5
    # lambda -> infinity: every weight 1/K and U* the plain mean of the
    # samples, which the device holds in float32 (half an ulp of the largest
    # sample per term bounds the difference from the FP64 oracle's samples)
    flat = eng.step(dict(prob, lam=1e12, instance_id=12))
    assert np.allclose(flat["w"], 1.0 / 2048, rtol=1e-9, atol=0)
    ref_flat = oracle.solve(dict(prob, lam=1e12, instance_id=12), (W, b), sc.MODEL, contract="bf16w")
    samples = ref_flat["samples"]
    bound = np.abs(samples).max() * 2.0 ** -24 + 1e-12
    assert np.max(np.abs(flat["U_star"] - samples.mean(axis=0))) <= bound
    eng.close()
