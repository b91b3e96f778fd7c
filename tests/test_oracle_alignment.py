"""Pins of the perception-alignment cost, eq. 6 of Section IV-B-2 (CPU only).

J_vis = sum over steps t = 0..T-1 of 1 - cos(psi_t - psi_gate,t): psi_t the
yaw of the attitude q_t, psi_gate,t the bearing of the target waypoint seen
from the position p_t.  Hand values fix which yaw (q_t, not q_{t+1}) and
which bearing (from p_t to the waypoint, not the reverse) the oracle uses;
a constant yaw rate gives a closed-form sum of sines.
"""
import math

import numpy as np
import pytest

import scenarios as sc
from oracle import rollout, solve
from oracle.mppi import alignment_cost

M, G = sc.MODEL["mass"], sc.MODEL["gravity"]


def _prob(T, wp, p0=(0.0, 0.0, 0.0)):
    x0 = np.zeros(13)
    x0[0:3] = p0
    x0[3] = 1.0
    return {"T": T, "x0": x0, "wp": np.asarray(wp, dtype=float)}


def _still(T, yaw=0.0):
    """One rollout at rest at p0 with constant yaw (K = 1)."""
    p_rel = np.zeros((1, T + 1, 3))
    q = np.zeros((1, T + 1, 4))
    q[..., 0] = math.cos(yaw / 2)
    q[..., 3] = math.sin(yaw / 2)
    return p_rel, q


@pytest.mark.parametrize("wp,per_step", [
    ((5.0, 0.0, 0.0), 0.0),                          # straight ahead
    ((0.0, 5.0, 0.0), 1.0),                          # 90 degrees to the left
    ((0.0, -5.0, 0.0), 1.0),                         # 90 degrees to the right
    ((-5.0, 0.0, 0.0), 2.0),                         # behind
    ((5.0, 5.0, 3.0), 1.0 - math.cos(math.pi / 4)),  # 45 degrees, height ignored
])
def test_hover_at_origin_facing_x(wp, per_step):
    T = 12
    p_rel, q = _still(T)
    J = alignment_cost(p_rel, q, _prob(T, wp))
    assert J.shape == (1,)
    assert abs(J[0] - T * per_step) <= 1e-13 * T


def test_yaw_of_attitude_counts():
    # facing +y (yaw 90 degrees): a waypoint on +y is aligned, one on +x is not
    T = 7
    p_rel, q = _still(T, yaw=math.pi / 2)
    assert abs(alignment_cost(p_rel, q, _prob(T, (0.0, 4.0, 0.0)))[0]) <= 1e-13
    assert abs(alignment_cost(p_rel, q, _prob(T, (4.0, 0.0, 0.0)))[0] - T) <= 1e-13


def test_constant_yaw_rate_closed_form():
    """Hover thrust, body rate (0, 0, w): psi_t = w t dt and the drone stays at
    the origin; with the waypoint on +y, psi_gate = pi/2 and
    J = sum_{t=0}^{T-1} 1 - cos(w t dt - pi/2) = T - sum_{t=0}^{T-1} sin(w t dt)
      = T - sin((T-1) a / 2) sin(T a / 2) / sin(a / 2),  a = w dt.
    Summing over t = 1..T instead (yaw of q_{t+1}) misses it by
    sin(T a) - sin(0)."""
    T, dt, w = 25, 0.02, 3.0
    u = np.zeros((1, T, 4))
    u[..., 0] = M * G
    u[..., 3] = w
    x0 = np.zeros(13)
    x0[3] = 1.0
    p_rel, q, _ = rollout(x0, u, dt, M, G)
    a = w * dt
    closed = T - math.sin((T - 1) * a / 2) * math.sin(T * a / 2) / math.sin(a / 2)
    J = alignment_cost(p_rel, q, _prob(T, (0.0, 5.0, 0.0)))
    assert abs(J[0] - closed) <= 1e-12
    assert abs(math.sin(T * a)) > 0.1          # the shifted range would fail


def test_bearing_from_position_to_waypoint():
    """Moving along +x at yaw 0 past a waypoint at (x_w, 1): the bearing from
    p_t is atan2(1, x_w - x_t), so each step adds 1 - (x_w - x_t) / r_t with
    r_t = sqrt((x_w - x_t)^2 + 1); the reversed bearing (waypoint to p_t)
    would add 1 + (x_w - x_t) / r_t."""
    T, dt, v = 30, 0.02, 4.0
    xs = v * dt * np.arange(T + 1)
    p_rel = np.zeros((1, T + 1, 3))
    p_rel[0, :, 0] = xs
    _, q = _still(T)
    x_w = 0.5 * xs[-1]
    J = alignment_cost(p_rel, q, _prob(T, (x_w, 1.0, 0.0)))
    dx = x_w - xs[:T]
    expect = np.sum(1.0 - dx / np.sqrt(dx * dx + 1.0))
    assert abs(J[0] - expect) <= 1e-12 * T


def test_solve_adds_q_vis_times_alignment():
    """Zero noise at hover, yaw 0, waypoint on +y: every rollout has J_vis = T,
    so J(Q_vis) - J(0) = Q_vis T exactly, and the update is unchanged."""
    K, T = 8, 10
    base = sc.make_problem(K, T, 1, seed=5, Sigma=np.zeros((4, 4)), U_nom=np.tile([M * G, 0, 0, 0], (T, 1)))
    base["x0"] = np.zeros(13)
    base["x0"][3] = 1.0
    base["wp"] = np.array([0.0, 3.0, 0.0])
    W, b = sc.xavier_weights((67, 16, 16, 1), seed=2)
    r0 = solve(base, (W, b), sc.MODEL)
    r1 = solve(dict(base, Q_vis=0.75), (W, b), sc.MODEL)
    assert np.allclose(r1["J"] - r0["J"], 0.75 * T, rtol=0, atol=1e-12)
    assert np.array_equal(r0["U_star"], r1["U_star"])
