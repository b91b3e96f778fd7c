"""Counter-based Gaussian control noise for MPPI (oracle side).

Section IV-A draws the perturbations delta u_k^m ~ N(0, Sigma) but does not
say how.  Reading used here (shared by the GPU path through its own,
independently written code):

* generator: Philox4x64 with 10 rounds (Salmon, Moraes, Dror, Shaw,
  "Parallel random numbers: as easy as 1, 2, 3", SC'11);
* counter = (rollout k, step t, instance id, tick), key = (seed, 0);
* each of the four 64-bit output words gives one uniform from its top 23
  bits, u = (floor(r / 2^41) + 1/2) * 2^-23, which lies strictly inside
  (0, 1) and is exact in float32;
* Box-Muller (1958) turns (u0, u1) and (u2, u3) into four standard normals,
  channels 0..3 of the control.

Pinned against NumPy's own Philox4x64-10 bit generator and by moment /
Kolmogorov-Smirnov statistics of the normals (tests).
"""
from __future__ import annotations

import numpy as np

_M0 = np.uint64(0xD2E7470EE14C6C93)
_M1 = np.uint64(0xCA5A826395121157)
_W0 = np.uint64(0x9E3779B97F4A7C15)
_W1 = np.uint64(0xBB67AE8584CAA73B)
_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo64(a, b):
    """Full 64x64 -> 128-bit product of uint64 arrays, as (hi, lo)."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    a0, a1 = a & _LO32, a >> _S32
    b0, b1 = b & _LO32, b >> _S32
    p00 = a0 * b0
    p01 = a0 * b1
    p10 = a1 * b0
    p11 = a1 * b1
    mid = (p00 >> _S32) + (p01 & _LO32) + (p10 & _LO32)
    hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
    lo = a * b
    return hi, lo


def philox4x64_10(ctr, key):
    """Philox4x64-10 block function.

    ``ctr``: uint64 array (..., 4); ``key``: uint64 array (..., 2) or (2,).
    Returns uint64 array (..., 4).  Each round multiplies words 0 and 2 by
    the two Philox multipliers, swaps the word pairs and XORs the high
    halves with the other words and the round key; the key is advanced by
    the two Weyl constants between rounds.
    """
    with np.errstate(over="ignore"):
        c = np.array(ctr, dtype=np.uint64, copy=True)
        k = np.broadcast_to(np.asarray(key, dtype=np.uint64), c.shape[:-1] + (2,))
        k0 = k[..., 0].copy()
        k1 = k[..., 1].copy()
        x0, x1, x2, x3 = c[..., 0], c[..., 1], c[..., 2], c[..., 3]
        for r in range(10):
            if r > 0:
                k0 = k0 + _W0
                k1 = k1 + _W1
            hi0, lo0 = _mulhilo64(_M0, x0)
            hi1, lo1 = _mulhilo64(_M1, x2)
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
        return np.stack([x0, x1, x2, x3], axis=-1)


def uniforms_from_words(words):
    """Top 23 bits of each uint64 word -> float64 uniform in (0, 1)."""
    top = (np.asarray(words, dtype=np.uint64) >> np.uint64(41)).astype(np.float64)
    return (top + 0.5) * 2.0 ** -23


def box_muller(u):
    """Four uniforms (..., 4) -> four standard normals (..., 4), float64."""
    r01 = np.sqrt(-2.0 * np.log(u[..., 0]))
    r23 = np.sqrt(-2.0 * np.log(u[..., 2]))
    a01 = 2.0 * np.pi * u[..., 1]
    a23 = 2.0 * np.pi * u[..., 3]
    return np.stack([r01 * np.cos(a01), r01 * np.sin(a01),
                     r23 * np.cos(a23), r23 * np.sin(a23)], axis=-1)


def control_noise(seed, instance_id, tick, K, T):
    """Standard normals n[k, t, c] for every rollout k < K and step t < T."""
    kk, tt = np.meshgrid(np.arange(K, dtype=np.uint64), np.arange(T, dtype=np.uint64),
                         indexing="ij")
    ctr = np.stack([kk, tt,
                    np.full_like(kk, np.uint64(instance_id & (2**64 - 1))),
                    np.full_like(kk, np.uint64(tick & (2**64 - 1)))], axis=-1)
    key = np.array([seed & (2**64 - 1), 0], dtype=np.uint64)
    return box_muller(uniforms_from_words(philox4x64_10(ctr, key)))
