"""One MPPI iteration with the Gate-SDF cost (oracle side), float64.

Steps, in the order of Section IV:

1. Perturbations (Section IV-A): delta u = L n with L L^T = Sigma and n the
   counter-based standard normals of ``philox.control_noise``; the sampled
   sequence is U* + delta U, clipped to the input bounds of Table I
   (reading: clipping happens before the rollout and the weighted average
   uses the clipped samples; every one of the K samples is perturbed).
2. Rollouts through the quadrotor model (``dynamics.rollout``).
3. Gate-SDF at the predicted positions (Section IV-B-3: the decoder is
   queried at every predicted position).  Reading: the T predicted positions
   p_1..p_T are queried (flag SDF_AT_P0 selects p_0..p_{T-1}, the literal
   index range of eq. 8).  A world point p maps into gate g's frame as
   R_g^T (p - t_g), R_g having the gate axes as columns, gate x = normal.
4. Costs (Section IV-B): gate progress eq. 5 with p_wp the target waypoint,
   perception alignment eq. 6, SDF stage cost eq. 7 summed over the horizon
   eq. 8, total eq. 9, plus the control-effort term R_u sum |u_t|^2 of this
   build's workloads.
5. Update, eq. mppi_update: w_m = exp(-J_m / lambda) / sum_i exp(-J_i /
   lambda) and U* = sum_m w_m U^m.  Evaluated with the minimum cost
   subtracted first (the same weights; the shift cancels in the ratio).
   Reading: a non-finite cost gets weight 0; if every cost is non-finite
   the update is refused and U* stays as it was.
6. Receding horizon (Section IV-A): the first action is applied and the
   sequence seeds the next cycle, shifted left by one step with the last
   action repeated (reading).
"""
from __future__ import annotations

import numpy as np

from .dynamics import rollout, rotor_rollout
from .philox import control_noise
from .precision import contract_weights
from .precision import NEAR_TIE_ABS, NEAR_TIE_REL
from .sdf import gate_sdf_analytic, mlp_alternatives, mlp_concat

FLAG_SDF_AT_P0 = 1 << 1

STATUS_OK = 0
STATUS_ENUMERIC = -5


def hover_sequence(T, mass, gravity, rotor=False):
    """Nominal sequence of a new instance: hover thrust m g, zero body rates
    (rotor-thrust rates: zero rates, the thrusts stay where they are)."""
    U = np.zeros((T, 4))
    if not rotor:
        U[:, 0] = mass * gravity
    return U


# A pivot of the Cholesky factorisation within PIVOT_TOL of the matrix scale
# max |Sigma_ij| counts as zero (a semi-definite direction); the rest of its
# column must then vanish to within OFFDIAG_TOL of the scale, else Sigma is
# not positive semi-definite.
PIVOT_TOL = 1e-12
OFFDIAG_TOL = 1e-9


def noise_factor(Sigma):
    """Lower-triangular L with L L^T = Sigma (Section IV-A: delta u ~ N(0,
    Sigma), sampled as L n with n standard normal).

    Diagonal Sigma -> sqrt(diag), which admits zero variances.  Otherwise the
    column-by-column Cholesky factorisation: L_jj = sqrt(Sigma_jj - sum_k<j
    L_jk^2), L_ij = (Sigma_ij - sum_k<j L_ik L_jk) / L_jj.  Reading for a
    semi-definite Sigma (the factor is then not unique): a zero pivot leaves
    its whole column zero, which is the factor of a positive definite Sigma
    in the limit and keeps L L^T = Sigma.  Raises ValueError when Sigma is not
    symmetric positive semi-definite."""
    S = np.asarray(Sigma, dtype=np.float64).reshape(4, 4)
    if not np.all(np.isfinite(S)):
        raise ValueError("Sigma has non-finite entries")
    scale = float(np.max(np.abs(S)))
    if np.max(np.abs(S - S.T)) > 1e-12 * max(scale, 1.0):
        raise ValueError("Sigma is not symmetric")
    if np.count_nonzero(S - np.diag(np.diag(S))) == 0:
        if np.any(np.diag(S) < 0):
            raise ValueError("Sigma has a negative variance")
        return np.diag(np.sqrt(np.diag(S)))
    L = np.zeros((4, 4))
    for j in range(4):
        d = S[j, j] - sum(L[j, k] ** 2 for k in range(j))
        if d < -PIVOT_TOL * scale:
            raise ValueError("Sigma is not positive semi-definite")
        zero_pivot = d <= PIVOT_TOL * scale
        L[j, j] = 0.0 if zero_pivot else np.sqrt(d)
        for i in range(j + 1, 4):
            r = S[i, j] - sum(L[i, k] * L[j, k] for k in range(j))
            if zero_pivot:
                if abs(r) > OFFDIAG_TOL * scale:
                    raise ValueError("Sigma is not positive semi-definite")
            else:
                L[i, j] = r / L[j, j]
    return L


def sample_controls(prob, model, U_nom):
    K, T = prob["K"], prob["T"]
    n = control_noise(prob["seed"], prob["instance_id"], prob["tick"], K, T)
    eps = n @ noise_factor(prob["Sigma"]).T
    return np.clip(U_nom[None, :, :] + eps, model["u_lo"], model["u_hi"])


def gate_frame_points(p_world, R, t):
    """R^T (p - t) for points (..., 3)."""
    return (p_world - t) @ R


def sdf_values(p_rel, prob, weights, contract, act_scales, sdf_kind, ties=None):
    """max over gates of the decoder at the query positions; shape (K, T).

    ``ties`` (optional dict) receives (K, T) arrays under the ``bf16`` /
    ``fp8`` contracts: "count", the near-tie activations of the position
    summed over the gates, and "lo" / "hi", the range of the max over gates
    when those roundings go either way (sdf.mlp_alternatives; the maximum of
    per-gate ranges is the range of the maximum); and "alts", a dict flat
    position index (k T + t) -> every distinct value of the max over gates
    over those roundings, for the positions with near ties."""
    K, T, G = prob["K"], prob["T"], prob["G"]
    sel = slice(0, T) if prob["flags"] & FLAG_SDF_AT_P0 else slice(1, T + 1)
    pts = (p_rel[:, sel, :] + prob["x0"][0:3]).reshape(-1, 3)
    best = np.full(pts.shape[0], -np.inf)
    if sdf_kind == "mlp":
        W, b = contract_weights(weights[0], weights[1], contract)
    if ties is not None:
        cnt = np.zeros(pts.shape[0], dtype=np.int64)
        lo = np.full(pts.shape[0], -np.inf)
        hi = np.full(pts.shape[0], -np.inf)
        per_gate, per_gate_alts = [], []
    for g in range(G):
        pg = gate_frame_points(pts, prob["gate_R"][g], prob["gate_t"][g])
        if sdf_kind == "analytic":
            s = gate_sdf_analytic(pg)
        else:
            z = prob["gate_z"][g].astype(np.float64)
            s = np.empty(pg.shape[0])
            galts = {}
            step = 1 << 15
            for i in range(0, pg.shape[0], step):
                s[i:i + step] = mlp_concat(pg[i:i + step], z, W, b, contract, act_scales)
                if ties is not None:
                    c, a, e, v = mlp_alternatives(pg[i:i + step], z, W, b, contract, act_scales,
                                                  ties.get("window", (NEAR_TIE_REL, NEAR_TIE_ABS)), values=True)
                    cnt[i:i + step] += c
                    lo[i:i + step] = np.maximum(lo[i:i + step], a)
                    hi[i:i + step] = np.maximum(hi[i:i + step], e)
                    galts.update({i + r: vv for r, vv in v.items()})
        best = np.maximum(best, s)
        if ties is not None:
            per_gate.append(s)
            per_gate_alts.append(galts)
    if ties is not None:
        # values of the max over gates: every combination of the gates' values
        alts = {}
        for q in np.nonzero(cnt)[0]:
            acc = np.array([-np.inf])
            for s_g, a_g in zip(per_gate, per_gate_alts):
                v = a_g.get(int(q), np.array([s_g[q]]))
                acc = np.unique(np.maximum.outer(acc, v).ravel())
            alts[int(q)] = acc
        ties["count"] = cnt.reshape(K, T)
        ties["lo"] = lo.reshape(K, T)
        ties["hi"] = hi.reshape(K, T)
        ties["alts"] = alts
    return best.reshape(K, T)


def progress_cost_literal(p_world, wp):
    """Eq. 5 as printed: sum_t |p_{t+1} - wp|^2 - |p_t - wp|^2."""
    d2 = np.sum((p_world - wp) ** 2, axis=-1)
    return np.sum(d2[:, 1:] - d2[:, :-1], axis=1)


def progress_cost_closed(p_rel, p0, wp):
    """Eq. 5 after telescoping: |d|^2 + 2 d.(p_0 - wp), d = p_T - p_0."""
    d = p_rel[:, -1, :]
    e = p0 - wp
    return np.sum(d * d, axis=1) + 2.0 * d @ e


def alignment_cost(p_rel, q, prob):
    """Eq. 6: sum over steps 0..T-1 of 1 - cos(psi_t - psi_gate,t), psi the yaw
    of the attitude and psi_gate the bearing from p_t to the target waypoint."""
    T = prob["T"]
    qq = q[:, :T]
    w, x, y, z = qq[..., 0], qq[..., 1], qq[..., 2], qq[..., 3]
    psi = np.arctan2(2.0 * (w * z + x * y), 1.0 - 2.0 * (y * y + z * z))
    pw = p_rel[:, :T, :] + prob["x0"][0:3]
    los = np.arctan2(prob["wp"][1] - pw[..., 1], prob["wp"][0] - pw[..., 0])
    return np.sum(1.0 - np.cos(psi - los), axis=1)


def mppi_update(J, u, lam):
    """Eq. mppi_update with the minimum cost subtracted; non-finite J -> w = 0.

    Returns (U_star, w, rho, log_eta, ess, ok)."""
    J = np.asarray(J, dtype=np.float64)
    finite = np.isfinite(J)
    if not finite.any():
        return None, np.zeros_like(J), np.nan, np.nan, 0.0, False
    rho = np.min(J[finite])
    wt = np.where(finite, np.exp(-(np.where(finite, J, rho) - rho) / lam), 0.0)
    eta = np.sum(wt)
    w = wt / eta
    U = np.tensordot(w, u, axes=(0, 0))
    return U, w, rho, np.log(eta) - rho / lam, 1.0 / np.sum(w * w), True


def shift_warm_start(U):
    """Next cycle's nominal: shift left one step, repeat the last action."""
    return np.concatenate([U[1:], U[-1:]], axis=0)


def solve(prob, weights, model, contract="fp32", sdf_kind="mlp", act_scales=None,
          U_nom=None, near_ties=False):
    """One MPPI iteration.  ``weights`` = (W list, b list) float32 as given
    to the library; ``model`` = dict(mass, gravity, u_lo, u_hi), plus for the
    rotor-thrust-rate input (kind "rotor") inertia, arm_length, yaw_coeff,
    thrust_max, rate_max, with the rotor thrusts in ``prob["thrust0"]``.

    Returns a dict with U_star (T, 4), u0 (4,), J (K,), w (K,), rho, log_eta,
    ess, status and the intermediates samples (K, T, 4), p_rel (K, T+1, 3),
    sdf (K, T).  With ``near_ties`` (``bf16`` / ``fp8`` contracts; True, or
    a (relative, absolute) near-tie window) also near_tie (K, T): per query
    position the number of activations feeding the hidden layers that lie
    within the near-tie window of a rounding boundary
    (precision.near_tie_mask), summed over the gates, sdf_lo / sdf_hi
    (K, T): the range of the field at that position over every legitimate
    rounding of those activations (sdf.mlp_alternatives), and sdf_alts: a
    dict flat position (k T + t) -> every distinct field value over those
    roundings, for the positions with near ties."""
    T = prob["T"]
    if U_nom is None:
        U_nom = prob["U_nom"]
    rotor = model.get("kind") == "rotor"
    if U_nom is None:
        U_nom = hover_sequence(T, model["mass"], model["gravity"], rotor=rotor)
    U_nom = np.asarray(U_nom, dtype=np.float64)
    u = sample_controls(prob, model, U_nom)
    if rotor:
        p_rel, q, _ = rotor_rollout(prob["x0"], prob["thrust0"], u, prob["dt"], model)
    else:
        p_rel, q, _ = rollout(prob["x0"], u, prob["dt"], model["mass"], model["gravity"])
    ties = None
    if near_ties:
        if contract not in ("bf16", "fp8") or sdf_kind != "mlp":
            raise ValueError("near ties are counted for the MLP under the bf16 and fp8 contracts")
        ties = {} if near_ties is True else {"window": tuple(near_ties)}
    s = sdf_values(p_rel, prob, weights, contract, act_scales, sdf_kind, ties)
    out = costs_and_update(prob, u, p_rel, q, s, U_nom)
    out.update({"samples": u, "p_rel": p_rel, "q": q, "sdf": s})
    if ties is not None:
        out.update({"near_tie": ties["count"], "sdf_lo": ties["lo"], "sdf_hi": ties["hi"],
                    "sdf_alts": ties["alts"]})
    return out


def costs_and_update(prob, u, p_rel, q, s, U_nom):
    """Costs (eqs. 5-9 with the control effort) of rollouts u (K, T, 4) with
    positions p_rel, attitudes q and field values s (K, T) at their query
    points, then the update (eq. mppi_update).  ``solve`` calls it with the
    field it evaluated; under the ``bf16`` / ``fp8`` contracts a caller may
    pass another of the legitimate fields (values from ``sdf_lo`` / ``sdf_hi``
    at near-tie positions) to get the update that goes with that rounding."""
    J_gate = progress_cost_closed(p_rel, prob["x0"][0:3], prob["wp"])
    J_sdf = np.sum(np.maximum(0.0, prob["d_safe"] - s), axis=1)
    J_u = np.sum(u * u, axis=(1, 2))
    J = prob["Q_gate"] * J_gate + prob["Q_sdf"] * J_sdf + prob["R_u"] * J_u
    if prob["Q_vis"] != 0.0:
        J = J + prob["Q_vis"] * alignment_cost(p_rel, q, prob)
    U_star, w, rho, log_eta, ess, ok = mppi_update(J, u, prob["lam"])
    if not ok:
        U_star = np.asarray(U_nom, dtype=np.float64).copy()
    return {
        "status": STATUS_OK if ok else STATUS_ENUMERIC,
        "U_star": U_star, "u0": U_star[0].copy(), "U_next": shift_warm_start(U_star),
        "J": J, "w": w, "rho": rho, "log_eta": log_eta, "ess": ess,
    }
