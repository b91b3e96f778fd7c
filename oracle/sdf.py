"""Gate-SDF evaluation (oracle side), float64.

* Analytic guidance field, Section III-A eqs. 1-2:
  r(p) = max(|y|, |z|) on the gate plane x = 0, and
  s_guide(p) = c + |x| tan(alpha) - r(p).  The paper leaves c and alpha
  open; with the 1.0 m inner opening of Section V, c = 0.5 m, and
  tan(alpha) = 0.5 is this library's reading.
* Learned decoder g_phi(z, PE(p)), Section III-B: an MLP on the
  concatenation of the encoded query point and the latent code z.  The
  measured workloads take PE as the identity (input width 3 + 64 = 67:
  coordinates in columns 0..2, the latent in 3..66).  The paper does not
  define PE; the encoded variant reads it as the usual Fourier features
  PE(p) = [p, sin(2^0 pi p), cos(2^0 pi p), ..., sin(2^(F-1) pi p),
  cos(2^(F-1) pi p)] (3 + 6F columns, each sin / cos block over x, y, z),
  followed by the latent; F is implied by the width of the first layer.
  Hidden layers use softplus (beta = 1) and the output layer is linear so
  the field can be negative.
  The paper's Fig. 2 duplicates z for every query and concatenates;
  ``mlp_concat`` does exactly that, ``mlp_fold`` applies the first layer's
  latent block once per gate (an exact re-association).
* Several gates per solve (the multi-gate workloads): the field at
  a point is the maximum over gates of each gate's field (union of the safe
  funnels); with one gate this is the paper's single-latent case.
"""
from __future__ import annotations

import numpy as np
import torch

from .precision import NEAR_TIE_ABS, NEAR_TIE_REL, bf16_round, bf16_split2, e4m3_round, near_tie_mask

C_HALF_WIDTH = 0.5
TAN_ALPHA = 0.5


def _softplus_t(x):
    """softplus on a float64 torch tensor (CPU, multithreaded elementwise ops)."""
    return torch.clamp_min(x, 0.0) + torch.log1p(torch.exp(-torch.abs(x)))


def softplus(x):
    """log(1 + exp(x)) in the overflow-free form max(x, 0) + log1p(exp(-|x|))."""
    return _softplus_t(torch.as_tensor(np.asarray(x, dtype=np.float64))).numpy()


def gate_sdf_analytic(pg, c=C_HALF_WIDTH, tan_alpha=TAN_ALPHA):
    """s_guide at gate-frame points pg (..., 3): eqs. 1-2."""
    r = np.maximum(np.abs(pg[..., 1]), np.abs(pg[..., 2]))
    return c + np.abs(pg[..., 0]) * tan_alpha - r


def _t(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float64))


def _hidden_input(h, layer, contract, act_scales):
    """Operand of hidden layer ``layer`` (1-based H x H layer) under a contract."""
    if contract == "bf16":
        return _t(bf16_round(h.numpy()))
    if contract == "bf16x2":
        hi, lo = bf16_split2(h.numpy())
        return _t(hi) + _t(lo)
    if contract == "fp8":
        s = act_scales[layer - 1]
        return _t(e4m3_round(h.numpy() / s) * s)
    return h


def _grid_round(x, contract, scale):
    """The contract's activation rounding (bf16, or E4M3 of x / scale)."""
    if contract == "fp8":
        return e4m3_round(x / scale) * scale
    return bf16_round(x)


def _mlp_tail(h, W, b, contract, act_scales):
    """Layers 2..L+1 of the decoder from the first hidden activation h."""
    n = len(W)
    for l in range(1, n - 1):
        a = _hidden_input(h, l, contract, act_scales)
        h = _softplus_t(a @ _t(W[l]).T + _t(b[l]))
    return h @ _t(W[n - 1]).T + _t(b[n - 1])


# Enumeration limit of the alternative roundings of one query row: at most
# MAX_TIE_BITS tied elements per layer.
MAX_TIE_BITS = 12


def _alt_values(x, l, W, b, contract, act_scales, window):
    """Every output value of the decoder over the legitimate roundings of the
    activation row x (float64, the input of hidden layer l, 1-based) and of
    the rows it leads to (sorted, distinct).  Elements within the near-tie
    window of a rounding boundary may round either way (both candidates: the
    roundings of x - w and x + w); each combination is carried through the
    next layer exactly, whose own near ties are enumerated in turn."""
    n = len(W)
    sc = act_scales[l - 1] if contract == "fp8" else 1.0
    rel, abs_ = window
    w = rel * np.abs(x) + abs_
    lo_c, hi_c = _grid_round(x - w, contract, sc), _grid_round(x + w, contract, sc)
    idx = np.nonzero(lo_c != hi_c)[0]
    if idx.size > MAX_TIE_BITS:
        raise ValueError(f"{idx.size} near ties in one activation row: too many to enumerate")
    base = _grid_round(x, contract, sc)
    # the candidates of a tied element: the roundings of x - w, x and x + w
    # (x's own differs from both only when the window spans two boundaries)
    cands = [np.unique([lo_c[i], base[i], hi_c[i]]) for i in idx]
    m = int(np.prod([c.size for c in cands])) if cands else 1
    A = np.broadcast_to(base, (m, x.size)).copy()
    rep = 1
    for c, i in zip(cands, idx):
        A[:, i] = c[(np.arange(m) // rep) % c.size]
        rep *= c.size
    H = np.logaddexp(0.0, A @ np.asarray(W[l], dtype=np.float64).T + np.asarray(b[l], dtype=np.float64))
    if l + 1 == n - 1:
        return np.unique(H @ np.asarray(W[n - 1], dtype=np.float64)[0] + float(b[n - 1][0]))
    return np.unique(np.concatenate([_alt_values(H[r], l + 1, W, b, contract, act_scales, window)
                                     for r in range(m)]))


def mlp_alternatives(pg, z, W, b, contract, act_scales=None, window=(NEAR_TIE_REL, NEAR_TIE_ABS),
                     values=False):
    """Near ties of the decoder under the ``bf16`` / ``fp8`` contracts for
    points pg (N, 3): per query row the number of activations feeding the
    hidden layers that lie within the near-tie window of a rounding boundary
    (precision.near_tie_mask), and the range [s_lo, s_hi] of the output over
    every combination of their legitimate roundings, cascades into later
    layers included (s_lo = s_hi = s for a row without near ties).  With
    ``values`` also a dict row -> array of every distinct output value over
    those roundings, for the rows with near ties.
    ``W``/``b`` as in mlp_concat (already under the contract)."""
    if contract not in ("bf16", "fp8"):
        raise ValueError(f"near ties are defined for the bf16 and fp8 contracts, not {contract!r}")
    F = pe_freqs_of(W[0], z.shape[-1])
    x = np.concatenate([positional_encoding(pg, F), np.broadcast_to(z, (pg.shape[0], z.shape[-1]))], axis=1)
    h1 = _softplus_t(_t(x) @ _t(W[0]).T + _t(b[0])).numpy()
    n = len(W)
    count = np.zeros(pg.shape[0], dtype=np.int64)
    # rows with a near tie in any hidden input: found along the contract's own pass
    h = h1
    for l in range(1, n - 1):
        sc = act_scales[l - 1] if contract == "fp8" else 1.0
        count += np.sum(near_tie_mask(h, contract, scale=sc, rel=window[0], abs_=window[1]), axis=1)
        a = _hidden_input(_t(h), l, contract, act_scales)
        h = _softplus_t(a @ _t(W[l]).T + _t(b[l])).numpy()
    s = h @ np.asarray(W[n - 1], dtype=np.float64)[0] + float(b[n - 1][0])
    s_lo, s_hi = s.copy(), s.copy()
    vals = {}
    for r in np.nonzero(count)[0]:
        v = _alt_values(h1[r], 1, W, b, contract, act_scales, window)
        s_lo[r], s_hi[r] = v[0], v[-1]
        if values:
            vals[int(r)] = v
    if values:
        return count, s_lo, s_hi, vals
    return count, s_lo, s_hi


def pe_freqs_of(W0, latent_dim):
    """F of a first layer of width 3 + 6F + latent_dim."""
    extra = W0.shape[1] - latent_dim - 3
    if extra < 0 or extra % 6:
        raise ValueError(f"first-layer width {W0.shape[1]} is not 3 + 6F + {latent_dim}")
    return extra // 6


def positional_encoding(pg, F):
    """[p, sin(2^k pi p), cos(2^k pi p) for k < F] of points pg (N, 3): (N, 3 + 6F)."""
    cols = [pg]
    for k in range(F):
        a = np.pi * (2.0 ** k) * pg
        cols += [np.sin(a), np.cos(a)]
    return np.concatenate(cols, axis=1)


def mlp_concat(pg, z, W, b, contract="fp32", act_scales=None):
    """Decoder on the literal concatenation [PE(p); z] for points pg (N, 3).

    ``W``/``b`` are float64 arrays of the (possibly quantised) layers,
    W[l] of shape (n_out, n_in); returns s of shape (N,).
    """
    F = pe_freqs_of(W[0], z.shape[-1])
    x = np.concatenate([positional_encoding(pg, F), np.broadcast_to(z, (pg.shape[0], z.shape[-1]))], axis=1)
    h = _softplus_t(_t(x) @ _t(W[0]).T + _t(b[0]))
    return _mlp_tail(h, W, b, contract, act_scales)[:, 0].numpy()


def mlp_fold(pg, z, W, b, contract="fp32", act_scales=None):
    """Same decoder with the latent block of layer 1 applied once:
    c = W1[:, n:] z + b1, h1 = softplus(W1[:, :n] PE(p) + c), n = 3 + 6F."""
    n = W[0].shape[1] - z.shape[-1]
    c = _t(W[0])[:, n:] @ _t(z) + _t(b[0])
    h = _softplus_t(_t(positional_encoding(pg, (n - 3) // 6)) @ _t(W[0])[:, :n].T + c)
    return _mlp_tail(h, W, b, contract, act_scales)[:, 0].numpy()


def hidden_input_amax(pg, z, W, b):
    """max |h_l| of every activation that feeds a hidden H x H layer (l = 1..L-1),
    float64, over query points pg: the calibration statistic of the FP8
    contract's static activation scales (scale = amax / 448)."""
    n = W[0].shape[1] - z.shape[-1]
    h = _softplus_t(_t(positional_encoding(pg, (n - 3) // 6)) @ _t(W[0])[:, :n].T +
                    (_t(W[0])[:, n:] @ _t(z) + _t(b[0])))
    out = []
    for l in range(1, len(W) - 1):
        out.append(float(torch.max(torch.abs(h))))
        h = _softplus_t(h @ _t(W[l]).T + _t(b[l]))
    return out
