"""Pins of the oracle's reduced-precision bookkeeping (CPU only).

* The two-term bfloat16 split of the ``bf16x2`` contract against PyTorch's
  own conversions, and its error bound.
* Near ties (``bf16`` / ``fp8`` contracts): an activation is flagged when a
  rounding boundary lies within the window w = 2^-20 |x| + 2^-22 of it.
  Pins: hand values at and around boundaries; soundness by brute force (any
  perturbation within the window that changes the rounding only happens at
  a flagged value); the flagged fraction of uniform values against its
  expectation.
* The range of the decoder output over every legitimate rounding
  (``mlp_alternatives``): a hand-built decoder with one activation on a
  bfloat16 midpoint, and, with a wide window, random float32-like
  evaluators (perturbation within the window before each rounding) whose
  outputs must all fall inside the range, cascades through two hidden
  layers included.
"""
import math

import numpy as np
import pytest
import torch

import scenarios as sc
from oracle import bf16_round, e4m3_round, solve
from oracle.precision import NEAR_TIE_ABS, NEAR_TIE_REL, bf16_split2, contract_weights, near_tie_mask
from oracle.sdf import mlp_alternatives, mlp_concat, _softplus_t, _t


def test_bf16_split2_matches_torch_and_bound():
    rng = np.random.default_rng(0)
    # float32 values (torch converts to bfloat16 from float32; the remainder
    # x - hi is exact in float32)
    x32 = np.concatenate([rng.uniform(0.0, 8.0, 100000), np.exp(rng.uniform(-20, 5, 100000))]).astype(np.float32)
    x = x32.astype(np.float64)
    hi, lo = bf16_split2(x)
    th = torch.from_numpy(x32).to(torch.bfloat16)
    tl = (torch.from_numpy(x32) - th.to(torch.float32)).to(torch.bfloat16)
    assert np.array_equal(hi, th.to(torch.float64).numpy()) and np.array_equal(lo, tl.to(torch.float64).numpy())
    assert np.all(np.abs(x - hi - lo) <= 2.0 ** -17 * np.abs(x))
    # values with at most 16 significant bits split exactly
    y = np.ldexp(rng.integers(1 << 15, 1 << 16, 1000).astype(np.float64), -15)
    yh, yl = bf16_split2(y)
    assert np.array_equal(yh + yl, y)


def test_near_tie_hand_values_bf16():
    mid = 1.0 + 2.0 ** -8                      # halfway between 1 and 1 + 2^-7
    w = NEAR_TIE_REL * mid + NEAR_TIE_ABS
    x = np.array([mid, mid + 0.9 * w, mid - 0.9 * w, mid + 1.1 * w, 1.0, 1.5, mid + 2.0 ** -12])
    assert near_tie_mask(x, "bf16").tolist() == [True, True, True, False, False, False, False]


def test_near_tie_hand_values_fp8():
    s = 0.25
    mid = (1.0 + 2.0 ** -4) * s                # halfway between 1 and 1.125 (scaled)
    w = NEAR_TIE_REL * mid + NEAR_TIE_ABS
    x = np.array([mid, mid + 0.9 * w, mid + 1.1 * w, 1.0 * s, 600.0 * s])
    # above the largest value plus half a step everything saturates to 448: no boundary
    assert near_tie_mask(x, "fp8", scale=s).tolist() == [True, True, False, False, False]


@pytest.mark.parametrize("contract,scale", [("bf16", 1.0), ("fp8", 0.05)])
def test_near_tie_soundness_brute_force(contract, scale):
    rng = np.random.default_rng(1)
    x = np.exp(rng.uniform(-12.0, 3.0, 400000))
    w = NEAR_TIE_REL * x + NEAR_TIE_ABS
    rnd = (lambda v: bf16_round(v)) if contract == "bf16" else (lambda v: e4m3_round(v / scale) * scale)
    flagged = near_tie_mask(x, contract, scale=scale)
    for f in (-1.0, 1.0, rng.uniform(-1, 1, x.size)):
        changed = rnd(x + f * w) != rnd(x)
        assert np.all(flagged[changed])


def test_near_tie_rate_of_uniform_values():
    """For x uniform in [1, 2) (bfloat16 spacing 2^-7) a value is flagged
    when it lies within w(x) of one of the 128 midpoints: expected fraction
    E[2 w(x)] / 2^-7."""
    rng = np.random.default_rng(2)
    n = 2_000_000
    x = rng.uniform(1.0, 2.0, n)
    p = np.mean(2.0 * (NEAR_TIE_REL * x + NEAR_TIE_ABS)) / 2.0 ** -7
    k = np.count_nonzero(near_tie_mask(x, "bf16"))
    assert abs(k - n * p) <= 5.0 * math.sqrt(n * p * (1 - p)) + 1


def _hand_decoder():
    """67 -> 2 -> 2 -> 1 decoder whose first activation is softplus(x*) =
    1 + 2^-8 (a bfloat16 midpoint) and second 0.75 (exact in bfloat16)."""
    W0 = np.zeros((2, 67))
    W0[0, 3] = 1.0
    W0[1, 4] = 1.0
    z = np.zeros(64)
    z[0] = math.log(math.expm1(1.0 + 2.0 ** -8))
    z[1] = math.log(math.expm1(0.75))
    W = [W0, np.eye(2), np.array([[1.0, 1.0]])]
    b = [np.zeros(2), np.zeros(2), np.zeros(1)]
    return W, b, z


def test_alternatives_hand_decoder():
    W, b, z = _hand_decoder()
    pg = np.zeros((1, 3))
    count, lo, hi, vals = mlp_alternatives(pg, z, W, b, "bf16", values=True)
    sp = lambda v: math.log1p(math.exp(v))
    assert count.tolist() == [1]
    assert abs(lo[0] - (sp(1.0) + sp(0.75))) <= 1e-15
    assert abs(hi[0] - (sp(1.0 + 2.0 ** -7) + sp(0.75))) <= 1e-15
    # exactly the two roundings of the tied activation
    assert list(vals) == [0] and vals[0].size == 2
    assert abs(vals[0][0] - lo[0]) <= 1e-15 and abs(vals[0][1] - hi[0]) <= 1e-15
    # the oracle's own rounding (ties to even: 1) is one end of the range
    assert abs(mlp_concat(pg, z, W, b, "bf16")[0] - lo[0]) <= 1e-15


def _perturbed_eval(x_rows, z, W, b, contract, act_scales, window, rng):
    """A float32-like evaluator: before each rounding the activation carries
    an arbitrary error within the window."""
    F0 = W[0].shape[1] - z.shape[-1]
    xin = np.concatenate([x_rows, np.broadcast_to(z, (x_rows.shape[0], z.shape[-1]))], axis=1)
    assert F0 == 3
    h = _softplus_t(_t(xin) @ _t(W[0]).T + _t(b[0])).numpy()
    n = len(W)
    for l in range(1, n - 1):
        w = window[0] * np.abs(h) + window[1]
        e = rng.choice([-1.0, 1.0], size=h.shape) * rng.uniform(0.0, 1.0, size=h.shape) ** 0.25
        hp = h + e * w
        a = bf16_round(hp) if contract == "bf16" else e4m3_round(hp / act_scales[l - 1]) * act_scales[l - 1]
        h = _softplus_t(_t(a) @ _t(W[l]).T + _t(b[l])).numpy()
    return h @ np.asarray(W[n - 1])[0] + b[n - 1][0]


@pytest.mark.parametrize("contract", ["bf16", "fp8"])
def test_alternatives_contain_every_perturbed_evaluation(contract):
    """Wide window (2^-9 relative) so that most rows have near ties and the
    second hidden layer's ties depend on the first's choices; 64 random
    evaluators per row, every output inside [lo, hi]."""
    W32, b32 = sc.xavier_weights((67, 12, 12, 12, 1), seed=3, bias_scale=0.3)
    scales = [0.01, 0.01] if contract == "fp8" else None
    W, b = contract_weights(W32, b32, contract)
    rng = np.random.default_rng(4)
    pg = rng.uniform(-2, 2, (40, 3))
    z = rng.standard_normal(64)
    window = (2.0 ** -9, 2.0 ** -14)
    count, lo, hi, vals = mlp_alternatives(pg, z, W, b, contract, scales, window=window, values=True)
    assert np.count_nonzero(count) >= 20
    assert np.all(lo <= hi)
    assert sorted(vals) == np.nonzero(count)[0].tolist()
    widen = 0
    for _ in range(64):
        s = _perturbed_eval(pg, z, W, b, contract, scales, window, rng)
        assert np.all(s >= lo - 1e-12) and np.all(s <= hi + 1e-12)
        # every evaluation is one of the enumerated values of its row
        for r, v in vals.items():
            assert np.min(np.abs(v - s[r])) <= 1e-12
        widen += np.count_nonzero(np.abs(s - mlp_concat(pg, z, W, b, contract, scales)) > 1e-12)
    assert widen > 0      # the evaluators do take other roundings


def test_solve_reports_ranges_and_counts():
    W, b = sc.xavier_weights((67, 32, 32, 1), seed=0)
    prob = sc.make_problem(64, 8, 2, rot="haar", start="moving", seed=6, d_safe=1.0)
    r = solve(prob, (W, b), sc.MODEL, contract="bf16", near_ties=True)
    assert r["near_tie"].shape == (64, 8)
    assert np.all(r["sdf_lo"] <= r["sdf"] + 1e-15) and np.all(r["sdf"] <= r["sdf_hi"] + 1e-15)
    assert np.all(r["sdf_lo"][r["near_tie"] == 0] == r["sdf_hi"][r["near_tie"] == 0])
    assert np.any(r["sdf_lo"] < r["sdf_hi"])
    # the value sets of the max over gates span exactly the reported ranges
    # and hold the oracle's own value
    assert sorted(r["sdf_alts"]) == np.flatnonzero(r["near_tie"]).tolist()
    for q, v in r["sdf_alts"].items():
        k, t = divmod(q, 8)
        assert abs(v[0] - r["sdf_lo"][k, t]) <= 1e-13 and abs(v[-1] - r["sdf_hi"][k, t]) <= 1e-13
        assert np.min(np.abs(v - r["sdf"][k, t])) <= 1e-13
    # zero window: no near ties, the range collapses to the contract's value
    r0 = solve(prob, (W, b), sc.MODEL, contract="bf16", near_ties=(0.0, 0.0))
    assert r0["near_tie"].sum() == 0 and np.allclose(r0["sdf_lo"], r0["sdf"], rtol=0, atol=1e-13)
