"""Pins of the oracle's Gate-SDF evaluation (CPU only).

* The analytic field of Section III-A eqs. 1-2 against hand-worked values
  (tests/golden/gate_sdf_eq2.txt) and its symmetries.
* The decoder MLP: literal concatenation form, latent-fold form and
  ``torch.nn.Sequential`` in float64 with the same weights (library routine).
* softplus against ``torch.nn.functional.softplus`` in float64.
"""
import os

import numpy as np
import pytest
import torch

import scenarios as sc
from oracle import softplus, mlp_concat, mlp_fold, gate_sdf_analytic

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "gate_sdf_eq2.txt")


def test_analytic_gate_sdf_hand_values():
    rows = np.loadtxt(GOLDEN, comments="#")
    s = gate_sdf_analytic(rows[:, :3])
    assert np.allclose(s, rows[:, 3], atol=1e-15)


def test_analytic_gate_sdf_symmetries():
    rng = np.random.default_rng(0)
    p = rng.uniform(-3, 3, size=(1000, 3))
    s = gate_sdf_analytic(p)
    assert np.array_equal(s, gate_sdf_analytic(p * [-1, 1, 1]))
    assert np.array_equal(s, gate_sdf_analytic(p[:, [0, 2, 1]]))
    assert np.array_equal(s, gate_sdf_analytic(p * [1, -1, -1]))
    # the safe funnel widens linearly with |x| (slope tan alpha = 0.5)
    q = p.copy(); q[:, 0] = np.abs(q[:, 0]) + 1.0
    assert np.allclose(gate_sdf_analytic(q) - gate_sdf_analytic(q - [1.0, 0, 0]), 0.5)


def test_softplus_matches_torch_float64():
    x = np.concatenate([np.linspace(-60, 60, 20001), [-745.0, -700.0, 0.0, 700.0, 1e-300]])
    ref = torch.nn.functional.softplus(torch.from_numpy(x), beta=1, threshold=1e9).numpy()
    assert np.allclose(softplus(x), ref, rtol=1e-15, atol=1e-300)
    assert softplus(np.array([800.0]))[0] == 800.0      # no overflow


def _torch_mlp(W, b):
    layers = []
    for l, (w, v) in enumerate(zip(W, b)):
        lin = torch.nn.Linear(w.shape[1], w.shape[0], dtype=torch.float64)
        with torch.no_grad():
            lin.weight.copy_(torch.from_numpy(np.asarray(w, dtype=np.float64)))
            lin.bias.copy_(torch.from_numpy(np.asarray(v, dtype=np.float64)))
        layers.append(lin)
        if l < len(W) - 1:
            layers.append(torch.nn.Softplus(beta=1.0, threshold=1e9))
    return torch.nn.Sequential(*layers)


@pytest.mark.parametrize("layers", [(67, 128, 128, 1), (67, 256, 256, 256, 1), (67, 32, 1)])
def test_mlp_fold_concat_and_torch_agree(layers):
    W, b = sc.xavier_weights(layers, seed=0, bias_scale=0.3)
    W64 = [w.astype(np.float64) for w in W]
    b64 = [v.astype(np.float64) for v in b]
    rng = np.random.default_rng(1)
    pg = rng.uniform(-8, 8, size=(512, 3))
    z = rng.standard_normal(64)
    s_cat = mlp_concat(pg, z, W64, b64)
    s_fold = mlp_fold(pg, z, W64, b64)
    x = np.concatenate([pg, np.broadcast_to(z, (512, 64))], axis=1)
    s_t = _torch_mlp(W, b)(torch.from_numpy(x)).detach().numpy()[:, 0]
    scale = 1.0 + np.abs(s_t).max()
    assert np.max(np.abs(s_cat - s_t)) <= 1e-12 * scale
    assert np.max(np.abs(s_fold - s_t)) <= 1e-12 * scale


def test_mlp_input_order_is_coordinates_then_latent():
    # only column 0 of layer 1 is non-zero -> output depends on x only
    W = [np.zeros((4, 67)), np.eye(4), np.ones((1, 4))]
    W[0][:, 0] = 1.0
    b = [np.zeros(4), np.zeros(4), np.zeros(1)]
    pg = np.array([[2.0, 5.0, -5.0]])
    s1 = mlp_concat(pg, np.zeros(64), W, b)
    s2 = mlp_concat(pg, np.full(64, 9.0), W, b)
    assert s1 == s2
    assert np.isclose(s1[0], 4 * np.log1p(np.exp(np.log1p(np.exp(2.0)))))


# ------------------------------------------------------ positional encoding
from oracle.sdf import positional_encoding, pe_freqs_of  # noqa: E402


def test_positional_encoding_hand_values():
    """Features at points where sin / cos of multiples of pi are known."""
    p = np.array([[0.25, 0.5, -1.0]])
    f = positional_encoding(p, 2)[0]
    r2 = np.sqrt(0.5)
    expect = [0.25, 0.5, -1.0,
              r2, 1.0, 0.0, r2, 0.0, -1.0,          # sin(pi p), cos(pi p)
              1.0, 0.0, 0.0, 0.0, -1.0, 1.0]        # sin(2 pi p), cos(2 pi p)
    assert np.allclose(f, expect, atol=1e-15)
    assert positional_encoding(p, 0).shape == (1, 3)


def test_encoded_decoder_is_periodic_without_raw_coordinates():
    """With the raw-coordinate columns zeroed the encoded decoder depends on
    p only through sin / cos(2^k pi p): period 2 in every coordinate, and not
    period 1 (the k = 0 band has period 2)."""
    F = 3
    W, b = sc.xavier_weights((3 + 6 * F + 64, 32, 32, 1), seed=2, bias_scale=0.1)
    W = [w.astype(np.float64) for w in W]
    b = [v.astype(np.float64) for v in b]
    W[0][:, 0:3] = 0.0
    z = np.random.default_rng(1).standard_normal(64)
    p = np.random.default_rng(2).uniform(-3, 3, size=(50, 3))
    s0 = mlp_concat(p, z, W, b)
    for shift in (np.array([2.0, 0, 0]), np.array([0, -2.0, 0]), np.array([0, 0, 4.0])):
        assert np.allclose(mlp_concat(p + shift, z, W, b), s0, atol=1e-12)
    assert not np.allclose(mlp_concat(p + np.array([1.0, 0, 0]), z, W, b), s0, atol=1e-6)


def test_encoded_decoder_fold_and_concat_agree_and_width():
    F = 2
    W, b = sc.xavier_weights((3 + 6 * F + 64, 24, 24, 24, 1), seed=5, bias_scale=0.2)
    W = [w.astype(np.float64) for w in W]
    b = [v.astype(np.float64) for v in b]
    assert pe_freqs_of(W[0], 64) == F
    z = np.random.default_rng(3).standard_normal(64)
    p = np.random.default_rng(4).uniform(-6, 6, size=(40, 3))
    assert np.allclose(mlp_fold(p, z, W, b), mlp_concat(p, z, W, b), rtol=1e-13, atol=1e-13)
    # the same network through torch in float64 on the explicit features
    x = np.concatenate([positional_encoding(p, F), np.broadcast_to(z, (40, 64))], axis=1)
    h = torch.tensor(x)
    for l in range(len(W)):
        h = h @ torch.tensor(W[l]).T + torch.tensor(b[l])
        if l + 1 < len(W):
            h = torch.nn.functional.softplus(h)
    assert np.allclose(mlp_concat(p, z, W, b), h[:, 0].numpy(), rtol=1e-13, atol=1e-13)
    with pytest.raises(ValueError):
        pe_freqs_of(np.zeros((4, 3 + 5 + 64)), 64)
