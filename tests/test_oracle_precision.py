"""Pins of the oracle's rounding for the precision contracts (CPU only):
bfloat16 and OCP FP8 E4M3 rounding against PyTorch's own conversions."""
import numpy as np
import torch

from oracle import bf16_round, e4m3_round, quantise_weights_fp8


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(0)
    x32 = np.concatenate([
        rng.standard_normal(200000).astype(np.float32) * np.float32(3.0),
        rng.uniform(-1e4, 1e4, 50000).astype(np.float32),
        # exact ties between two bfloat16 neighbours (even and odd)
        (np.arange(1, 2000, dtype=np.float32) * np.float32(2 ** -8) + np.float32(1.0)),
    ]).astype(np.float32)
    ref = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(bf16_round(x32.astype(np.float64)), ref)


def test_e4m3_round_matches_torch_in_range():
    rng = np.random.default_rng(1)
    x32 = np.concatenate([
        rng.uniform(-448, 448, 100000),
        rng.standard_normal(100000) * 0.05,          # subnormal region (< 2^-6)
        rng.standard_normal(100000) * 4.0,
    ]).astype(np.float32)
    ref = torch.from_numpy(x32).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(e4m3_round(x32.astype(np.float64)), ref)


def test_e4m3_grid_and_saturation():
    assert e4m3_round(np.array([448.0, 464.0, 1e6, -1e6]))[:4].tolist() == [448.0, 448.0, 448.0, -448.0]
    assert e4m3_round(np.array([2.0 ** -9, 2.0 ** -10, 1.5 * 2.0 ** -10])).tolist() == [2.0 ** -9, 0.0, 2.0 ** -9]
    # ties to even: 1 + 1/16 lies between 1 and 1.125 -> 1
    assert e4m3_round(np.array([1.0 + 1.0 / 16.0, 1.0 + 3.0 / 16.0])).tolist() == [1.0, 1.25]


def test_fp8_weight_quantisation_scale():
    rng = np.random.default_rng(3)
    W = rng.uniform(-0.1, 0.1, size=(64, 64)).astype(np.float32)
    codes, s = quantise_weights_fp8(W)
    assert np.max(np.abs(codes)) == 448.0
    assert np.max(np.abs(codes * s - W)) <= s * 16.0      # half an e4m3 step at the top binade
