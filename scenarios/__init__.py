"""Seeded synthetic inputs for the MPPI + Gate-SDF hot path.

This module produces *inputs only*: network weights, latent codes, gate poses,
initial states, noise covariances and cost weights.  It contains none of the
method's arithmetic (no sampling of control noise, no dynamics, no SDF, no
cost and no update), so both the FP64 oracle and the GPU library can be fed
from it without sharing any computation.

The paper trains its Gate-SDF decoder on rendered depth data and ships no
weights, so seeded random weights stand in for the trained decoder
(Section III-B describes the decoder; its width and depth are not given).
Every generator draws from ``numpy.random.default_rng(seed)`` in a fixed
order, so a (config, seed) pair always yields the same problem.

Problem dictionaries use the field names of ``mppi_request`` in
``include/mppi.h``; rollouts are ``K``, horizon steps ``T`` and gates ``G``
(the paper writes M for rollouts and K for the horizon, Section IV-A).
"""
from __future__ import annotations

import numpy as np

# Vehicle and input bounds (Section V-B: 370 g vehicle; Table I: thrust in
# [0, 10] N, body rates in [-10, 10] rad/s).
MODEL = {
    "mass": 0.370,
    "gravity": 9.81,
    "u_lo": np.array([0.0, -10.0, -10.0, -10.0]),
    "u_hi": np.array([10.0, 10.0, 10.0, 10.0]),
}

# Noise covariance diag(sigma^2) for sigma = (2.0 N, 0.5, 0.5, 0.3 rad/s).
SIGMA_DIAG = np.array([4.0, 0.25, 0.25, 0.09])

# The paper's own input (Section IV-A): rates of the four rotor thrusts.
# Table I bounds the rates to [-10, 10] N/s, the thrusts to [0, 10] N and the
# body rate to [-10, 10] rad/s; the paper gives no inertia or geometry, so a
# 370 g racing quadrotor's are assumed (diagonal inertia, 0.09 m arms, yaw
# torque 0.016 N m per N of thrust).
ROTOR_MODEL = {
    "kind": "rotor",
    "mass": 0.370,
    "gravity": 9.81,
    "u_lo": np.array([-10.0, -10.0, -10.0, -10.0]),
    "u_hi": np.array([10.0, 10.0, 10.0, 10.0]),
    "inertia": np.array([1.5e-3, 1.5e-3, 2.6e-3]),
    "arm_length": 0.09,
    "yaw_coeff": 0.016,
    "thrust_max": 10.0,
    "rate_max": 10.0,
}
# Rotor-thrust-rate noise sigma = 4 N/s per rotor.
ROTOR_SIGMA_DIAG = np.array([16.0, 16.0, 16.0, 16.0])

LATENT_DIM = 64

# Named workloads.  Sizes follow the five benchmark configurations of this
# project (plain small solve, paper-scale solve, precision variants, served
# mix, served fleet).
CONFIGS = {
    "P1": dict(K=256, T=20, dt=0.02, G=1, layers=(67, 128, 128, 1), rot="haar",
               start="rest", n_scen=32),
    "P2": dict(K=4096, T=50, dt=0.02, G=4, layers=(67, 256, 256, 256, 1), rot="yaw",
               start="moving", n_scen=8, ticks=10),
    "S1": dict(layers=(67, 256, 256, 256, 1), G=1, dt=0.02, rot="yaw", start="moving",
               n_req=512, mean_gap_us=50.0, K_set=(1024, 2048, 4096, 8192),
               T_set=(20, 30, 40, 60)),
    "S2": dict(K=2048, T=40, dt=0.02, G=8, layers=(67, 512, 512, 512, 1), rot="yaw",
               start="moving", n_inst=1024, ticks=100),
}


def xavier_weights(layers, seed=0, bias_scale=0.0):
    """Glorot-uniform weights U(+-sqrt(6/(fan_in+fan_out))) for an MLP.

    ``layers`` lists the widths, e.g. (67, 256, 256, 256, 1).  Returns
    (W, b): W[l] has shape (n_out, n_in) row-major FP32, b[l] shape (n_out,).
    Biases are zero unless ``bias_scale`` > 0, in which case they are drawn
    U(-bias_scale, bias_scale) from a second stream so that W is unchanged.
    """
    rng = np.random.default_rng(seed)
    W, b = [], []
    for n_in, n_out in zip(layers[:-1], layers[1:]):
        lim = np.sqrt(6.0 / (n_in + n_out))
        W.append(rng.uniform(-lim, lim, size=(n_out, n_in)).astype(np.float32))
    brng = np.random.default_rng(seed + 1_000_003)
    for n_out in layers[1:]:
        if bias_scale > 0:
            b.append(brng.uniform(-bias_scale, bias_scale, size=n_out).astype(np.float32))
        else:
            b.append(np.zeros(n_out, dtype=np.float32))
    return W, b


def haar_rotation(rng):
    """Uniformly random rotation matrix (QR of a Gaussian matrix, sign-fixed)."""
    a = rng.standard_normal((3, 3))
    qm, rm = np.linalg.qr(a)
    qm = qm * np.sign(np.diag(rm))
    if np.linalg.det(qm) < 0:
        qm[:, 0] = -qm[:, 0]
    return qm


def yaw_rotation(psi):
    c, s = np.cos(psi), np.sin(psi)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def correlated_sigma(seed, rank=4, sigma=(2.0, 0.5, 0.5, 0.3)):
    """A full (non-diagonal) noise covariance with standard deviations
    ``sigma`` and seeded random correlations: Sigma = D C D with C the
    correlation matrix of B B^T, B a 4 x rank Gaussian matrix.  rank < 4
    gives a singular positive semi-definite Sigma (some channel an exact
    combination of the others)."""
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((4, rank))
    S = B @ B.T
    dinv = 1.0 / np.sqrt(np.diag(S))
    C = S * dinv[:, None] * dinv[None, :]
    D = np.asarray(sigma, dtype=np.float64)
    Sig = C * D[:, None] * D[None, :]
    return 0.5 * (Sig + Sig.T)


def _initial_state(rng, start):
    """State x0 = [p(3), q(w,x,y,z)(4), v(3), omega(3)]."""
    x0 = np.zeros(13)
    x0[3] = 1.0
    if start == "rest":
        return x0
    x0[0:3] = rng.uniform(-5.0, 5.0, size=3)
    psi = rng.uniform(-np.pi, np.pi)
    x0[3:7] = [np.cos(psi / 2), 0.0, 0.0, np.sin(psi / 2)]
    d = rng.standard_normal(3)
    d /= np.linalg.norm(d)
    x0[7:10] = rng.uniform(0.0, 15.0) * d
    return x0


def _gates(rng, G, rot):
    z = rng.standard_normal((G, LATENT_DIM)).astype(np.float32)
    t = rng.uniform(-5.0, 5.0, size=(G, 3))
    if rot == "haar":
        R = np.stack([haar_rotation(rng) for _ in range(G)])
    else:
        R = np.stack([yaw_rotation(rng.uniform(-np.pi, np.pi)) for _ in range(G)])
    return z, R, t


def make_problem(K, T, G, dt=0.02, rot="haar", start="rest", seed=1, instance_id=0,
                 tick=0, rng_seed=0, lam=1.0, Q_gate=1.0, Q_vis=0.0, Q_sdf=50.0,
                 d_safe=0.3, R_u=0.01, U_nom=None, Sigma=None, flags=0):
    """One MPPI solve request (field names follow ``mppi_request``)."""
    rng = np.random.default_rng(seed)
    z, R, t = _gates(rng, G, rot)
    x0 = _initial_state(rng, start)
    return {
        "K": int(K), "T": int(T), "G": int(G), "dt": float(dt),
        "instance_id": int(instance_id), "tick": int(tick), "seed": int(rng_seed),
        "x0": x0,
        "U_nom": None if U_nom is None else np.asarray(U_nom, dtype=np.float64),
        "Sigma": np.diag(SIGMA_DIAG) if Sigma is None else np.asarray(Sigma, dtype=np.float64),
        "lam": float(lam), "Q_gate": float(Q_gate), "Q_vis": float(Q_vis),
        "Q_sdf": float(Q_sdf), "d_safe": float(d_safe), "R_u": float(R_u),
        "wp": t[0].copy(),
        "gate_z": z, "gate_R": R, "gate_t": t,
        "flags": int(flags),
    }


def rotor_problem(K, T, G, seed=1, **kw):
    """A make_problem() request for the rotor-thrust-rate input: rate noise,
    rotor thrusts near hover (m g / 4 each, +-0.2 N) and, for a moving start,
    a body rate in [-1, 1] rad/s, drawn from a second stream so that the
    rest of the problem equals make_problem(K, T, G, seed, ...)."""
    kw.setdefault("Sigma", np.diag(ROTOR_SIGMA_DIAG))
    p = make_problem(K, T, G, seed=seed, **kw)
    rng = np.random.default_rng(seed + 1_000_003)
    m = ROTOR_MODEL
    p["thrust0"] = m["mass"] * m["gravity"] / 4.0 + rng.uniform(-0.2, 0.2, size=4)
    if kw.get("start", "rest") == "moving":
        p["x0"] = p["x0"].copy()
        p["x0"][10:13] = rng.uniform(-1.0, 1.0, size=3)
    return p


def config_problem(name, seed, **over):
    """Problem ``seed`` of a named configuration ("P1" or "P2")."""
    c = CONFIGS[name]
    kw = dict(K=c["K"], T=c["T"], G=c["G"], dt=c["dt"], rot=c["rot"], start=c["start"],
              seed=seed)
    kw.update(over)
    return make_problem(**kw)


def config_weights(name, seed=0, bias_scale=0.0):
    return xavier_weights(CONFIGS[name]["layers"], seed=seed, bias_scale=bias_scale)


def serving_requests(seed=4, n_req=None, K_set=None, T_set=None, mean_gap_us=None):
    """Served-mix request list: Poisson arrivals, uneven K and T, G = 1.

    Returns a list of (arrival_time_s, problem) sorted by arrival time; each
    request is its own drone instance (instance_id = request index).
    """
    c = CONFIGS["S1"]
    n_req = c["n_req"] if n_req is None else n_req
    K_set = c["K_set"] if K_set is None else K_set
    T_set = c["T_set"] if T_set is None else T_set
    gap = (c["mean_gap_us"] if mean_gap_us is None else mean_gap_us) * 1e-6
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(gap, size=n_req))
    Ks = rng.choice(np.asarray(K_set), size=n_req)
    Ts = rng.choice(np.asarray(T_set), size=n_req)
    out = []
    for i in range(n_req):
        p = make_problem(int(Ks[i]), int(Ts[i]), c["G"], dt=c["dt"], rot=c["rot"],
                         start=c["start"], seed=10_000 + seed * 100_000 + i, instance_id=i)
        out.append((float(arrivals[i]), p))
    return out
