"""Parity of the plain FP32 path (one solve per launch sequence) with the FP64
oracle, element by element, through the C ABI.

Tolerances (derived from float32 arithmetic, checked against the oracle):
* samples: Box-Muller in float32 with ocml log/sqrt/sincospi, |du| <= 2e-6 (|u| + 1);
* positions: 50 float32 integration steps from the local frame, |dp| <= 2e-5 + 2e-6 |p|;
* SDF: float32 decoder (FP32 matrix cores, float32 accumulation), |ds| <= 2e-5 (1 + |s|);
* costs: |dJ| <= 2e-6 (|J| + Q_sdf T) (float32 sums of T terms);
* u*_0: the A.19-style metric above, gated at 1e-4.
"""
import numpy as np
import pytest

import oracle
import scenarios as sc
from oracle.mppi import sample_controls
from gpu_common import U0_TOL, require_gpu, say, seq_error, u0_error

pytestmark = pytest.mark.gpu


def _engine(M, layers, K_max, T_max, G_max, **kw):
    W, b = sc.xavier_weights(layers, seed=kw.pop("wseed", 0), bias_scale=kw.pop("bias_scale", 0.0))
    eng = M.Engine((W, b), sc.MODEL, K_max=K_max, T_max=T_max, G_max=G_max, hidden=layers[1],
                   n_hidden=len(layers) - 2, precision="fp32", path="plain",
                   budget=kw.pop("budget", 512 << 20), **kw)
    return eng, (W, b)


def _within(name, got, want, tol):
    d = np.abs(np.asarray(got, dtype=np.float64) - want)
    bad = ~(d <= tol)
    assert not bad.any(), f"{name}: {int(bad.sum())} elements out of tolerance, max |diff| {d.max():.3e}"


def _check_elementwise(out, ref, prob):
    K, T = prob["K"], prob["T"]
    _within("samples", out["samples"], ref["samples"], 2e-6 * (np.abs(ref["samples"]) + 1.0))
    _within("positions", out["p_rel"], ref["p_rel"], 2e-5 + 2e-6 * np.abs(ref["p_rel"]))
    _within("sdf", out["sdf"], ref["sdf"], 2e-5 * (1.0 + np.abs(ref["sdf"])))
    _within("J", out["J"], ref["J"], 2e-6 * (np.abs(ref["J"]) + prob["Q_sdf"] * T + 1.0))
    assert abs(out["w"].sum() - 1.0) < 1e-12


@pytest.fixture(scope="module")
def p1():
    M = require_gpu()
    eng, w = _engine(M, (67, 128, 128, 1), 256, 20, 1)
    yield M, eng, w
    eng.close()


@pytest.mark.parametrize("d_safe", [0.3, 1.0])
def test_p1_elementwise_and_u0(p1, d_safe):
    M, eng, w = p1
    errs = []
    for seed in (1, 2, 3):
        prob = sc.config_problem("P1", seed, d_safe=d_safe, instance_id=int(100 * d_safe) * 100 + seed)
        ref = oracle.solve(prob, w, sc.MODEL)
        out = eng.step(prob, exports=True)
        assert out["rc"] == 0
        _check_elementwise(out, ref, prob)
        errs.append(u0_error(out["u0"], ref["u0"]))
        assert seq_error(out["U_star"], ref["U_star"]) <= 1e-3
        assert abs(out["J_min"] - ref["rho"]) <= 1e-5 * (1 + abs(ref["rho"]))
        assert abs(out["ess"] - ref["ess"]) <= 1e-3 * ref["ess"]
    say(f"P1 d_safe={d_safe}: u0 errors {['%.2e' % e for e in errs]}")
    assert max(errs) <= U0_TOL


def test_noise_stream_at_scale():
    """The device's Philox4x64-10 stream and its Box-Muller transform against
    the oracle's over 1.47 M counters (K = 8192, T = 60, three ticks, with a
    64-bit key and an instance id and tick that set high counter bits): the
    samples use the top 24 bits of every Philox word, so any word that
    differs moves a sample far outside the float32 tolerance."""
    M = require_gpu()
    key = 0x9E3779B97F4A7C15          # the engine's Philox key (mppi_config.seed)
    eng, _ = _engine(M, (67, 128, 128, 1), 8192, 60, 1, budget=1 << 30, seed=key)
    U = oracle.hover_sequence(60, sc.MODEL["mass"], sc.MODEL["gravity"])
    for tick in (0, 1, 0xFFFFFFFE):
        prob = sc.make_problem(8192, 60, 1, seed=3, instance_id=(1 << 40) + 7, tick=tick, rng_seed=key,
                               U_nom=U)
        out = eng.step(prob, exports=True)
        assert out["rc"] == 0
        ref = sample_controls(prob, sc.MODEL, U)
        _within("samples", out["samples"], ref, 2e-6 * (np.abs(ref) + 1.0))
        say(f"noise stream tick {tick:#x}: {ref.size // 4} counters, max |du| "
            f"{np.abs(out['samples'] - ref).max():.1e}")
    eng.close()


def test_p1_32_scenarios_u0_error(p1):
    M, eng, w = p1
    for d_safe in (0.3, 1.0):
        errs = []
        for seed in range(1, 33):
            prob = sc.config_problem("P1", seed, d_safe=d_safe, instance_id=int(100 * d_safe) * 1000 + seed + 50000)
            ref = oracle.solve(prob, w, sc.MODEL)
            out = eng.step(prob, weights=False, costs=False)
            assert out["rc"] == 0
            errs.append(u0_error(out["u0"], ref["u0"]))
        say(f"P1 x32 d_safe={d_safe}: u0 err max {max(errs):.3e} median {np.median(errs):.3e}")
        assert max(errs) <= U0_TOL


def test_deterministic_rerun(p1):
    M, eng, w = p1
    # the same instance, tick and nominal twice: bitwise equal (fixed-order reductions)
    U = oracle.hover_sequence(20, sc.MODEL["mass"], sc.MODEL["gravity"])
    prob = sc.config_problem("P1", 5, d_safe=1.0, instance_id=7, tick=3, U_nom=U)
    a = eng.step(prob)
    c = eng.step(prob)
    assert a["rc"] == 0 and c["rc"] == 0
    assert np.array_equal(a["U_star"], c["U_star"]) and np.array_equal(a["J"], c["J"])


def test_edge_shapes_and_flags():
    M = require_gpu()
    cases = [
        dict(layers=(67, 64, 64, 64, 1), K=1, T=1, G=1),
        dict(layers=(67, 64, 64, 1), K=257, T=7, G=3),            # ragged K, G not dividing 64
        dict(layers=(67, 128, 128, 1), K=100, T=13, G=8, flags=2),  # SDF at p_0..p_{T-1}
        dict(layers=(67, 512, 512, 512, 1), K=64, T=5, G=2),
        dict(layers=(67, 256, 256, 256, 1), K=333, T=9, G=5, bias=0.4),
    ]
    for c in cases:
        eng, w = _engine(M, c["layers"], max(c["K"], 1), max(c["T"], 1), c["G"],
                         bias_scale=c.get("bias", 0.0), wseed=3)
        prob = sc.make_problem(c["K"], c["T"], c["G"], rot="haar", start="moving", seed=17,
                               d_safe=1.0, flags=c.get("flags", 0), instance_id=5)
        say("edge case", c)
        ref = oracle.solve(prob, w, sc.MODEL)
        out = eng.step(prob, exports=True)
        eng.close()
        assert out["rc"] == 0
        _check_elementwise(out, ref, prob)
        assert u0_error(out["u0"], ref["u0"]) <= U0_TOL


def test_analytic_sdf_path():
    M = require_gpu()
    eng = M.Engine(None, sc.MODEL, K_max=512, T_max=30, G_max=4, sdf_kind="analytic",
                   budget=256 << 20)
    for seed in (3, 4):
        prob = sc.make_problem(500, 30, 4, rot="haar", start="moving", seed=seed, d_safe=1.0,
                               instance_id=seed)
        ref = oracle.solve(prob, None, sc.MODEL, sdf_kind="analytic")
        out = eng.step(prob, exports=True)
        assert out["rc"] == 0
        _within("sdf", out["sdf"], ref["sdf"], 1e-5 * (1 + np.abs(ref["sdf"])))
        assert u0_error(out["u0"], ref["u0"]) <= U0_TOL
    eng.close()


def test_zero_noise_returns_nominal_and_alignment_cost():
    M = require_gpu()
    eng, w = _engine(M, (67, 64, 64, 1), 128, 12, 2)
    prob = sc.make_problem(128, 12, 2, seed=9, Sigma=np.zeros((4, 4)), instance_id=1,
                           U_nom=np.tile([4.0, 0.1, -0.2, 0.3], (12, 1)))
    out = eng.step(prob)
    assert out["rc"] == 0
    assert np.allclose(out["U_star"], prob["U_nom"], rtol=0, atol=1e-6)
    assert np.allclose(out["w"], 1.0 / 128)
    prob = sc.make_problem(128, 12, 2, rot="yaw", start="moving", seed=10, Q_vis=3.0,
                           instance_id=2, d_safe=1.0)
    ref = oracle.solve(prob, w, sc.MODEL)
    out = eng.step(prob)
    assert out["rc"] == 0
    _within("J", out["J"], ref["J"], 2e-6 * (np.abs(ref["J"]) + 600 + 1.0))
    assert u0_error(out["u0"], ref["u0"]) <= U0_TOL
    eng.close()


def test_errors_and_all_nonfinite():
    M = require_gpu()
    eng, w = _engine(M, (67, 64, 64, 1), 128, 12, 2)
    good = sc.make_problem(64, 12, 2, seed=9, instance_id=3)
    assert eng.step(good)["rc"] == 0
    bad = [dict(good, lam=0.0), dict(good, lam=float("nan")), dict(good, K=129),
           dict(good, T=13), dict(good, Sigma=-np.eye(4)),
           dict(good, Sigma=np.array([[1, 2, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0], [0, 0, 0, 1.0]])),
           dict(good, x0=np.r_[good["x0"][:3], [2, 0, 0, 0], good["x0"][7:]]),
           dict(good, x0=np.r_[np.nan, good["x0"][1:]])]
    for b in bad:
        assert eng.step(b)["rc"] == M.MPPI_EINVAL
    # every cost non-finite -> ENUMERIC, U* = nominal, warm start kept
    U = np.tile([3.0, 0.0, 0.0, 0.0], (12, 1))
    out = eng.step(dict(good, Q_gate=float("inf"), U_nom=U, instance_id=4))
    assert out["rc"] == M.MPPI_ENUMERIC
    assert np.array_equal(out["U_star"], U)
    ref = oracle.solve(dict(good, Q_gate=float("inf")), w, sc.MODEL, U_nom=U)
    assert ref["status"] == -5
    eng.close()


def _advance(x, u, dt):
    """The harness's plant: one float64 model step from x under u."""
    p, q, v = oracle.rollout(x, u[None, None, :], dt, sc.MODEL["mass"], sc.MODEL["gravity"])
    xn = x.copy()
    xn[0:3] = x[0:3] + p[0, 1]
    xn[3:7] = q[0, 1]
    xn[7:10] = v[0, 1]
    xn[10:13] = u[1:4]
    return xn


def test_p2_full_size_warm_started_ticks():
    """Paper-scale solve (K=4096, T=50, 4 gates, 67-256-256-256-1) over 10
    warm-started ticks; each tick's oracle starts from the GPU's state,
    resident nominal and tick, so errors do not compound."""
    M = require_gpu()
    eng, w = _engine(M, (67, 256, 256, 256, 1), 4096, 50, 4, budget=1 << 30)
    prob = sc.config_problem("P2", 1, instance_id=42)
    U_prev = None
    x = prob["x0"].copy()
    errs = []
    for tick in range(10):
        p = dict(prob, x0=x, tick=M.TICK_RESIDENT, U_nom=None)
        out = eng.step(p)
        assert out["rc"] == 0 and out["tick_used"] == tick
        ref = oracle.solve(dict(p, tick=tick), w, sc.MODEL,
                           U_nom=None if U_prev is None else oracle.shift_warm_start(U_prev))
        e = u0_error(out["u0"], ref["u0"])
        errs.append(e)
        dJ = np.abs(out["J"] - ref["J"])
        say(f"P2 tick {tick}: u0 err {e:.2e}, max |dJ| {dJ.max():.2e}, ess {out['ess']:.1f}")
        _within("J", out["J"], ref["J"], 2e-6 * (np.abs(ref["J"]) + 50 * 50 + 1.0))
        U_prev = out["U_star"]
        x = _advance(x, out["u0"], prob["dt"])
    assert max(errs) <= U0_TOL
    eng.close()


def test_torch_memory_and_stream():
    """The engine can take its per-solve pool and stream from torch."""
    M = require_gpu()
    import torch
    W, b = sc.xavier_weights((67, 128, 128, 1), seed=0)
    prob = sc.config_problem("P1", 2, instance_id=9)
    ref = oracle.solve(prob, (W, b), sc.MODEL)
    with M.Engine((W, b), sc.MODEL, use_torch_memory=True, K_max=256, T_max=20, G_max=1,
                  hidden=128, n_hidden=2, budget=64 << 20) as eng:
        out = eng.step(prob)
    torch.cuda.synchronize()
    assert out["rc"] == 0 and u0_error(out["u0"], ref["u0"]) <= U0_TOL
