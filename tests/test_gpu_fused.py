"""Parity of the fused low-precision path with the FP64 oracle under the
matching precision contract (the oracle rounds exactly what the kernel's
matrix cores consume):

* BF16X3 (bfloat16 weights, activations split into three bfloat16 terms)
  against ``bf16w``: residual activation error ~2^-24 relative, float32 level,
  so u*_0 is gated at the float32 tolerance 1e-4;
* F16X2 (the bfloat16-rounded weights held exactly in FP16 under a
  power-of-two scale, activations split into two FP16 terms) against
  ``bf16w``: residual ~2^-22 relative, gated like BF16X3;
* BF16X2 (two terms) against ``bf16w``: residual ~2^-16 relative; a float32
  emulation of its arithmetic gives u*_0 errors up to 3.6e-4 on P1, so it is
  gated at 1e-3 and reported;
* BF16 against ``bf16`` and FP8 against ``fp8``: activations rounded to 8 / 4
  significant bits flip where the float32 and float64 values straddle a
  rounding boundary; each flip moves a cost by a discrete step that the
  softmax (lambda = 1) can amplify, so the worst scenario is reported and the
  gate is on the median u*_0 error and on the bulk of the per-rollout costs.
"""
import numpy as np
import pytest

import oracle
import scenarios as sc
from gpu_common import SIGMA_FLOOR, U0_TOL, require_gpu, say, u0_error
from oracle.mppi import sample_controls
from oracle.sdf import hidden_input_amax

pytestmark = pytest.mark.gpu

CONTRACT = {"bf16x2": "bf16w", "bf16x3": "bf16w", "f16x2": "bf16w", "bf16": "bf16", "fp8": "fp8"}
U0_GATE = {"bf16x2": 1e-3, "bf16x3": U0_TOL, "f16x2": U0_TOL, "bf16": 2e-2}
FP32_LEVEL = ("bf16x3", "f16x2")   # gated at the float32 tolerance
U0_MEDIAN_GATE = {"fp8": 2e-3}


def _act_scales(layers, W, b, probs):
    """Static FP8 activation scales from oracle queries of the given problems."""
    amax = np.zeros(len(layers) - 3)
    for p in probs:
        u = sample_controls(p, sc.MODEL, oracle.hover_sequence(p["T"], 0.37, 9.81))
        pr, _, _ = oracle.rollout(p["x0"], u, p["dt"], 0.37, 9.81)
        pts = (pr[:, 1:] + p["x0"][0:3]).reshape(-1, 3)
        for g in range(p["G"]):
            pg = (pts - p["gate_t"][g]) @ p["gate_R"][g]
            amax = np.maximum(amax, hidden_input_amax(pg, p["gate_z"][g].astype(np.float64),
                                                      [w.astype(np.float64) for w in W],
                                                      [v.astype(np.float64) for v in b]))
    return amax / 448.0


def _engine(M, layers, precision, K_max, T_max, G_max, act_scale=None, wseed=0, bias=0.0):
    W, b = sc.xavier_weights(layers, seed=wseed, bias_scale=bias)
    wts = (W, b, act_scale) if act_scale is not None else (W, b)
    eng = M.Engine(wts, sc.MODEL, K_max=K_max, T_max=T_max, G_max=G_max, hidden=layers[1],
                   n_hidden=len(layers) - 2, precision=precision, path="fused", budget=512 << 20)
    return eng, (W, b)


@pytest.mark.parametrize("precision", ["bf16x2", "bf16x3", "f16x2", "bf16", "fp8"])
def test_p1_fused_precision_variants(precision):
    M = require_gpu()
    layers = (67, 128, 128, 1)
    W, b = sc.xavier_weights(layers, seed=0)
    scales = None
    if precision == "fp8":
        scales = _act_scales(layers, W, b, [sc.config_problem("P1", 0, K=256)])
    eng, w = _engine(M, layers, precision, 256, 20, 1, act_scale=scales)
    for d_safe in (0.3, 1.0):
        errs, errs32, jrel = [], [], []
        for seed in range(1, 9):
            prob = sc.config_problem("P1", seed, d_safe=d_safe, instance_id=int(d_safe * 10) * 100 + seed)
            ref = oracle.solve(prob, w, sc.MODEL, contract=CONTRACT[precision], act_scales=scales)
            ref32 = oracle.solve(prob, w, sc.MODEL, contract="fp32")
            out = eng.step(prob)
            assert out["rc"] == 0, out["rc"]
            assert abs(out["w"].sum() - 1.0) < 1e-12
            errs.append(u0_error(out["u0"], ref["u0"]))
            errs32.append(u0_error(out["u0"], ref32["u0"]))
            dJ = np.abs(out["J"] - ref["J"])
            jrel.append(dJ / (np.abs(ref["J"]) + prob["Q_sdf"] * prob["T"] + 1.0))
            if precision in FP32_LEVEL:
                assert np.all(dJ <= 2e-5 * (np.abs(ref["J"]) + prob["Q_sdf"] * prob["T"] + 1.0)), dJ.max()
        jr = np.concatenate(jrel)
        say(f"P1 fused {precision} d_safe={d_safe}: u0 err vs {CONTRACT[precision]} max {max(errs):.2e} "
            f"median {np.median(errs):.2e}; vs fp32 max {max(errs32):.2e}; relative cost error "
            f"p50 {np.percentile(jr, 50):.1e} p99 {np.percentile(jr, 99):.1e} max {jr.max():.1e}")
        if precision in U0_GATE:
            assert max(errs) <= U0_GATE[precision]
        else:
            assert np.median(errs) <= U0_MEDIAN_GATE[precision]
            assert np.percentile(jr, 90) <= 1e-3
    eng.close()


@pytest.mark.parametrize("precision", ["bf16x3", "f16x2", "bf16x2"])
def test_p2_fused_full_size_and_determinism(precision):
    M = require_gpu()
    layers = (67, 256, 256, 256, 1)
    eng, w = _engine(M, layers, precision, 4096, 50, 4)
    for seed in (1, 2):
        prob = sc.config_problem("P2", seed, instance_id=seed)
        ref = oracle.solve(prob, w, sc.MODEL, contract="bf16w")
        out = eng.step(prob)
        assert out["rc"] == 0
        e = u0_error(out["u0"], ref["u0"])
        dJ = np.abs(out["J"] - ref["J"])
        say(f"P2 fused {precision} seed {seed}: u0 err {e:.2e}, max |dJ| {dJ.max():.2e}, ess {out['ess']:.1f}")
        assert e <= U0_GATE[precision]
        if precision in FP32_LEVEL:
            assert np.all(dJ <= 2e-5 * (np.abs(ref["J"]) + 50 * 50 + 1.0))
    # same request twice (same explicit tick and nominal): bitwise equal
    U = oracle.hover_sequence(50, 0.37, 9.81)
    prob = sc.config_problem("P2", 3, instance_id=77, tick=5, U_nom=U)
    a = eng.step(prob)
    c = eng.step(prob)
    assert np.array_equal(a["U_star"], c["U_star"]) and np.array_equal(a["J"], c["J"])
    eng.close()


@pytest.mark.parametrize("precision", FP32_LEVEL)
def test_fused_ragged_shapes_and_gates(precision):
    M = require_gpu()
    layers = (67, 256, 256, 1)
    eng, w = _engine(M, layers, precision, 1000, 37, 8, wseed=4, bias=0.3)
    for K, T, G, flags in ((1, 1, 1, 0), (17, 5, 3, 0), (999, 37, 8, 2), (250, 20, 5, 0)):
        prob = sc.make_problem(K, T, G, rot="haar", start="moving", seed=K + T, d_safe=1.0,
                               flags=flags, instance_id=K)
        ref = oracle.solve(prob, w, sc.MODEL, contract="bf16w")
        out = eng.step(prob)
        assert out["rc"] == 0
        e = u0_error(out["u0"], ref["u0"])
        say(f"fused ragged K={K} T={T} G={G}: u0 err {e:.2e}")
        assert e <= U0_TOL
    eng.close()


def test_fused_alignment_cost_two_hidden_layers():
    """Perception-alignment cost (eq. 6, Q_vis > 0) through the fused path's
    dynamics, on the P2 decoder shape at a reduced K."""
    M = require_gpu()
    layers = (67, 256, 256, 256, 1)
    eng, w = _engine(M, layers, "bf16x3", 512, 30, 4, wseed=2, bias=0.2)
    for seed in (5, 6):
        prob = sc.make_problem(512, 30, 4, rot="yaw", start="moving", seed=seed, d_safe=1.0, Q_vis=0.5,
                               instance_id=300 + seed)
        ref = oracle.solve(prob, w, sc.MODEL, contract="bf16w")
        out = eng.step(prob)
        assert out["rc"] == 0
        e = u0_error(out["u0"], ref["u0"])
        dJ = np.abs(out["J"] - ref["J"])
        say(f"fused Q_vis=0.5 seed {seed}: u0 err {e:.2e}, max |dJ| {dJ.max():.2e}")
        assert e <= U0_TOL
        assert np.all(dJ <= 2e-5 * (np.abs(ref["J"]) + prob["Q_sdf"] * prob["T"] + 1.0))
    eng.close()


@pytest.mark.parametrize("precision", ["bf16", "fp8"])
def test_fused_low_precision_two_hidden_layers(precision):
    """BF16 and FP8 on the two-hidden-layer decoder (the served shape), each
    against its own contract; reported like the P1 variants."""
    M = require_gpu()
    layers = (67, 256, 256, 256, 1)
    W, b = sc.xavier_weights(layers, seed=3)
    probs = [sc.make_problem(384, 24, 4, rot="yaw", start="moving", seed=s, d_safe=1.0, instance_id=400 + s)
             for s in (1, 2, 3)]
    scales = _act_scales(layers, W, b, probs) if precision == "fp8" else None
    eng, w = _engine(M, layers, precision, 384, 24, 4, act_scale=scales, wseed=3)
    errs, jrel = [], []
    for prob in probs:
        ref = oracle.solve(prob, w, sc.MODEL, contract=CONTRACT[precision], act_scales=scales)
        out = eng.step(prob)
        assert out["rc"] == 0
        errs.append(u0_error(out["u0"], ref["u0"]))
        jrel.append(np.abs(out["J"] - ref["J"]) / (np.abs(ref["J"]) + prob["Q_sdf"] * prob["T"] + 1.0))
    jr = np.concatenate(jrel)
    say(f"fused {precision} 67-256-256-256-1: u0 err vs {CONTRACT[precision]} max {max(errs):.2e} "
        f"median {np.median(errs):.2e}; relative cost error p50 {np.percentile(jr, 50):.1e} "
        f"p90 {np.percentile(jr, 90):.1e}")
    # observed: median 6.6e-4 (bf16), 2.9e-3 (fp8); cost p90 1.5e-6, 2.4e-5
    assert np.median(errs) <= {"bf16": 3e-3, "fp8": 1e-2}[precision]
    assert np.percentile(jr, 90) <= 1e-4
    eng.close()


@pytest.mark.parametrize("precision", FP32_LEVEL)
def test_fused_h128_two_hidden_layers(precision):
    """H = 128 with two hidden layers (each wave owns 32 neurons of one
    layer, layer-1 blocks split 1:1)."""
    M = require_gpu()
    layers = (67, 128, 128, 128, 1)
    eng, w = _engine(M, layers, precision, 600, 25, 3, wseed=5, bias=0.3)
    for K, T, G in ((600, 25, 3), (33, 7, 1)):
        prob = sc.make_problem(K, T, G, rot="haar", start="moving", seed=K, d_safe=1.0, instance_id=500 + K)
        ref = oracle.solve(prob, w, sc.MODEL, contract="bf16w")
        out = eng.step(prob)
        assert out["rc"] == 0
        e = u0_error(out["u0"], ref["u0"])
        say(f"fused {precision} H=128 x2 K={K} T={T} G={G}: u0 err {e:.2e}")
        assert e <= U0_TOL
    eng.close()


@pytest.mark.parametrize("precision", ["bf16x3", "f16x2", "bf16x2", "bf16", "fp8"])
def test_fused_h512_two_hidden_layers(precision):
    """H = 512 (the large-fleet decoder shape, weights streamed through LDS):
    BF16X3 at the float32 tolerance against bf16w, the others against their
    contracts as on the other shapes.  G = 3 leaves a padding row in every
    block of 16; K = 300 a ragged last tile."""
    M = require_gpu()
    layers = (67, 512, 512, 512, 1)
    W, b = sc.xavier_weights(layers, seed=6, bias_scale=0.2)
    probs = [sc.make_problem(300, 16, 3, rot="haar", start="moving", seed=s, d_safe=1.0, instance_id=600 + s)
             for s in (1, 2)]
    scales = _act_scales(layers, W, b, probs) if precision == "fp8" else None
    eng, w = _engine(M, layers, precision, 300, 16, 3, act_scale=scales, wseed=6, bias=0.2)
    errs, jrel = [], []
    for prob in probs:
        ref = oracle.solve(prob, w, sc.MODEL, contract=CONTRACT[precision], act_scales=scales)
        out = eng.step(prob)
        assert out["rc"] == 0
        errs.append(u0_error(out["u0"], ref["u0"]))
        jrel.append(np.abs(out["J"] - ref["J"]) / (np.abs(ref["J"]) + prob["Q_sdf"] * prob["T"] + 1.0))
    jr = np.concatenate(jrel)
    say(f"fused {precision} 67-512-512-512-1: u0 err vs {CONTRACT[precision]} max {max(errs):.2e} "
        f"median {np.median(errs):.2e}; relative cost error p50 {np.percentile(jr, 50):.1e} "
        f"p90 {np.percentile(jr, 90):.1e} max {jr.max():.1e}")
    if precision in FP32_LEVEL:
        assert max(errs) <= U0_TOL
        assert jr.max() <= 2e-5
    elif precision == "bf16x2":
        assert max(errs) <= U0_GATE["bf16x2"]
    else:
        # the bulk of the costs matches the contract closely; FP8 activation
        # flips across 512-wide layers move a few costs by discrete steps that
        # the softmax amplifies in u*_0 (observed: median 1.5e-2 for FP8,
        # 9e-4 for BF16)
        assert np.median(errs) <= {"bf16": 1e-2, "fp8": 5e-2}[precision]
        assert np.percentile(jr, 50) <= 1e-5
        assert np.percentile(jr, 90) <= 1e-4
    eng.close()


@pytest.mark.parametrize("precision", FP32_LEVEL)
def test_fused_h512_one_hidden_layer_and_edges(precision):
    """H = 512 with one hidden layer; single rollout, one step, one gate;
    and a full tile with G = 8 (two positions per block)."""
    M = require_gpu()
    layers = (67, 512, 512, 1)
    eng, w = _engine(M, layers, precision, 64, 12, 8, wseed=7, bias=0.3)
    for K, T, G in ((1, 1, 1), (64, 12, 8), (17, 5, 5)):
        prob = sc.make_problem(K, T, G, rot="haar", start="moving", seed=K + 7 * T, d_safe=1.0, instance_id=700 + K)
        ref = oracle.solve(prob, w, sc.MODEL, contract="bf16w")
        out = eng.step(prob)
        assert out["rc"] == 0
        e = u0_error(out["u0"], ref["u0"])
        say(f"fused {precision} H=512 x1 K={K} T={T} G={G}: u0 err {e:.2e}")
        assert e <= U0_TOL
    eng.close()


@pytest.mark.parametrize("H", [256, 512])
def test_f16x2_weight_scaling(H):
    """F16X2 holds the bfloat16 weights in FP16 under a per-layer power of
    two: hidden layers scaled by 2^-12 (every weight below the FP16 normal
    range without the scale) and by 2^6 (activations of tens to hundreds in
    the next layer) still match the bf16w contract at the float32
    tolerance."""
    M = require_gpu()
    layers = (67, H, H, H, 1)
    W, b = sc.xavier_weights(layers, seed=8, bias_scale=0.2)
    W = list(W)
    W[1] = (W[1] * 2.0 ** -12).astype(np.float32)
    W[2] = (W[2] * 2.0 ** 6).astype(np.float32)
    w = (W, b)
    eng = M.Engine(w, sc.MODEL, K_max=256, T_max=16, G_max=2, hidden=H, n_hidden=3,
                   precision="f16x2", path="fused", budget=512 << 20)
    for seed in (1, 2):
        # lambda = 10: with costs of several hundred, float32-level cost
        # errors alone move u*_0 by ~1e-4 at lambda = 1; the per-rollout
        # costs carry the check of the scaling
        prob = sc.make_problem(256, 16, 2, rot="haar", start="moving", seed=seed, d_safe=1.0,
                               instance_id=800 + seed, lam=10.0)
        ref = oracle.solve(prob, w, sc.MODEL, contract="bf16w")
        out = eng.step(prob)
        assert out["rc"] == 0
        e = u0_error(out["u0"], ref["u0"])
        jr = np.abs(out["J"] - ref["J"]) / (np.abs(ref["J"]) + prob["Q_sdf"] * prob["T"] + 1.0)
        say(f"f16x2 H={H} scaled layers seed {seed}: u0 err {e:.2e}, max rel dJ {jr.max():.1e}")
        assert e <= U0_TOL and jr.max() <= 2e-5
    eng.close()
