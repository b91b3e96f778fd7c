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

from .precision import bf16_round, e4m3_round

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
    if contract == "fp8":
        s = act_scales[layer - 1]
        return _t(e4m3_round(h.numpy() / s) * s)
    return h


def _mlp_tail(h, W, b, contract, act_scales):
    """Layers 2..L+1 of the decoder from the first hidden activation h."""
    n = len(W)
    for l in range(1, n - 1):
        a = _hidden_input(h, l, contract, act_scales)
        h = _softplus_t(a @ _t(W[l]).T + _t(b[l]))
    return h @ _t(W[n - 1]).T + _t(b[n - 1])


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
