"""Precision contracts for the SDF decoder's matrix layers (oracle side).

The paper does not discuss reduced precision; the contracts define what a
reduced-precision GPU variant is compared against.  Only the H x H hidden
layers (the ones a GPU runs on matrix cores) are affected; the first layer,
the output layer and all other arithmetic stay float64.

* ``fp32``  - weights as given (float32 values, exact in float64).
* ``bf16w`` - hidden-layer weights rounded float32 -> bfloat16,
  round-to-nearest-even; activations exact.
* ``bf16``  - ``bf16w`` plus every activation that feeds a hidden layer
  rounded to bfloat16 (round-to-nearest-even from its float64 value).
* ``fp8``   - hidden-layer weights quantised to OCP FP8 E4M3 (bias 7,
  largest finite 448, no infinities, saturating, round-to-nearest-even)
  with a per-layer scale s_W = max|W| / 448; activations feeding a hidden
  layer quantised to E4M3 with a static per-layer scale s_a given as input.
  The weight codes are decided in float32, as the library decides them
  when it packs the weights (a code is an integer decision: both sides take
  it in the same precision).
"""
from __future__ import annotations

import numpy as np

E4M3_MAX = 448.0


def bf16_round(x):
    """Round float64 values to the nearest bfloat16 (8 significant bits),
    ties to even.  Finite normal-range inputs only."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                       # x = m * 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.rint(m * 256.0), e - 8)


def e4m3_round(x):
    """Round float64 values to OCP FP8 E4M3 (saturating at +-448), ties to even.

    Normal numbers have 4 significant bits and exponents down to 2^-6;
    below 2^-6 the grid is uniform with spacing 2^-9 (subnormals)."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)
    normal = np.ldexp(np.rint(m * 16.0), e - 4)
    sub = np.rint(x * 512.0) / 512.0
    q = np.where(np.abs(x) < 2.0 ** -6, sub, normal)
    return np.clip(q, -E4M3_MAX, E4M3_MAX)


def quantise_weights_fp8(W32):
    """Per-layer FP8 E4M3 quantisation of one float32 weight matrix.

    Returns (codes_as_float64, scale) with W ~= codes * scale; the scale and
    the scaled values are formed in float32."""
    W32 = np.asarray(W32, dtype=np.float32)
    amax = np.float32(np.max(np.abs(W32)))
    scale = np.float32(amax / np.float32(E4M3_MAX)) if amax > 0 else np.float32(1.0)
    scaled = (W32 / scale).astype(np.float32)
    return e4m3_round(scaled.astype(np.float64)), float(scale)


def contract_weights(W32, b32, contract):
    """float64 layer lists under a precision contract (+ per-layer weight scales)."""
    W = [np.asarray(w, dtype=np.float64) for w in W32]
    b = [np.asarray(v, dtype=np.float64) for v in b32]
    n = len(W)
    if contract in ("bf16w", "bf16"):
        for l in range(1, n - 1):
            W[l] = bf16_round(W[l])
    elif contract == "fp8":
        for l in range(1, n - 1):
            codes, s = quantise_weights_fp8(W32[l])
            W[l] = codes * s
    elif contract != "fp32":
        raise ValueError(f"unknown precision contract {contract!r}")
    return W, b
