"""Precision contracts for the SDF decoder's matrix layers (oracle side).

The paper does not discuss reduced precision; the contracts define what a
reduced-precision GPU variant is compared against.  Only the H x H hidden
layers (the ones a GPU runs on matrix cores) are affected; the first layer,
the output layer and all other arithmetic stay float64.

* ``fp32``  - weights as given (float32 values, exact in float64).
* ``bf16w`` - hidden-layer weights rounded float32 -> bfloat16,
  round-to-nearest-even; activations exact.
* ``bf16x2`` - ``bf16w`` with every activation that feeds a hidden layer
  replaced by its two-term bfloat16 split hi + lo, hi the round-to-nearest-
  even bfloat16 of the activation and lo that of the remainder (16
  significant bits kept, the rest dropped).
* ``bf16``  - ``bf16w`` plus every activation that feeds a hidden layer
  rounded to bfloat16 (round-to-nearest-even from its float64 value).
* ``fp8``   - hidden-layer weights quantised to OCP FP8 E4M3 (bias 7,
  largest finite 448, no infinities, saturating, round-to-nearest-even)
  with a per-layer scale s_W = max|W| / 448; activations feeding a hidden
  layer quantised to E4M3 with a static per-layer scale s_a given as input.
  The weight codes are decided in float32, as the library decides them
  when it packs the weights (a code is an integer decision: both sides take
  it in the same precision).

Near ties (``near_tie_mask``).  Under ``bf16`` and ``fp8`` an activation is
rounded to a coarse grid; a float32 evaluation of the same network carries
its activations with a small error, so where the float64 activation lies
within that error of a rounding boundary either rounding is a correct
result.  The oracle flags such elements: x is a near tie when the interval
[x - w, x + w] holds a rounding boundary, i.e. when its ends round
differently (rounding is monotone), with the window w = 2^-20 |x| + 2^-22
(reading: the relative part covers float32 accumulation and rounding of
the pre-activation, the absolute part the ~1e-7 absolute error of a float32
softplus evaluated through base-2 exponential and logarithm).
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


def bf16_split2(x):
    """Two-term bfloat16 split of float64 values: (hi, lo) with hi the RNE
    bfloat16 of x and lo the RNE bfloat16 of the exact remainder x - hi."""
    hi = bf16_round(x)
    return hi, bf16_round(np.asarray(x, dtype=np.float64) - hi)


NEAR_TIE_REL = 2.0 ** -20
NEAR_TIE_ABS = 2.0 ** -22


def near_tie_mask(x, contract, scale=1.0, rel=NEAR_TIE_REL, abs_=NEAR_TIE_ABS):
    """Elements of the activations x (float64) that lie within the window
    w = rel |x| + abs_ of a rounding boundary of the contract's activation
    grid: bfloat16 for ``bf16``, E4M3 of x / scale for ``fp8`` (the window is
    taken on x, then scaled with it)."""
    x = np.asarray(x, dtype=np.float64)
    w = rel * np.abs(x) + abs_
    if contract == "bf16":
        return bf16_round(x - w) != bf16_round(x + w)
    if contract == "fp8":
        return e4m3_round((x - w) / scale) != e4m3_round((x + w) / scale)
    raise ValueError(f"near ties are defined for the bf16 and fp8 contracts, not {contract!r}")


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
    if contract in ("bf16w", "bf16", "bf16x2"):
        for l in range(1, n - 1):
            W[l] = bf16_round(W[l])
    elif contract == "fp8":
        for l in range(1, n - 1):
            codes, s = quantise_weights_fp8(W32[l])
            W[l] = codes * s
    elif contract != "fp32":
        raise ValueError(f"unknown precision contract {contract!r}")
    return W, b
