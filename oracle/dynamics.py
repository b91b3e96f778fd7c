"""Quadrotor rollout f(x, u) for MPPI (oracle side), float64.

Section IV-A uses a standard quadrotor model with state [p, v, q, omega].
Two input forms: collective thrust + body rates (the form of the measured
workloads), and the paper's own four rotor-thrust rates (rotor_rollout
below), which turn the rotor thrusts and the body rate into state.
Readings where the paper is silent:

* state layout x = [p(3), q(4) as (w, x, y, z), v(3), omega(3)], world z up;
* Hamilton quaternions mapping body to world, thrust along body +z;
* input u = [collective thrust T (N), body rates omega_x, omega_y, omega_z];
  the body rate follows the command instantly (omega_{t+1} = u[1:4]);
* integrator over one step dt: the attitude is held at its start value for
  the acceleration a = (T / m) R(q_t) e3 - g e3 (zero-order hold), so
  p_{t+1} = p_t + v_t dt + a dt^2 / 2 and v_{t+1} = v_t + a dt; the
  attitude advances by the exact exponential of the constant body rate,
  q_{t+1} = q_t (x) [cos(|w| dt / 2), sin(|w| dt / 2) w / |w|];
* positions are reported relative to the start position p_0.
"""
from __future__ import annotations

import numpy as np


def quat_mul(a, b):
    """Hamilton product a (x) b of (..., 4) arrays in (w, x, y, z) order."""
    aw, ax, ay, az = a[..., 0], a[..., 1], a[..., 2], a[..., 3]
    bw, bx, by, bz = b[..., 0], b[..., 1], b[..., 2], b[..., 3]
    return np.stack([
        aw * bw - ax * bx - ay * by - az * bz,
        aw * bx + ax * bw + ay * bz - az * by,
        aw * by - ax * bz + ay * bw + az * bx,
        aw * bz + ax * by - ay * bx + az * bw,
    ], axis=-1)


def quat_to_matrix(q):
    """Rotation matrix (..., 3, 3) of unit quaternions (..., 4)."""
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    r = np.empty(q.shape[:-1] + (3, 3))
    r[..., 0, 0] = 1 - 2 * (y * y + z * z)
    r[..., 0, 1] = 2 * (x * y - w * z)
    r[..., 0, 2] = 2 * (x * z + w * y)
    r[..., 1, 0] = 2 * (x * y + w * z)
    r[..., 1, 1] = 1 - 2 * (x * x + z * z)
    r[..., 1, 2] = 2 * (y * z - w * x)
    r[..., 2, 0] = 2 * (x * z - w * y)
    r[..., 2, 1] = 2 * (y * z + w * x)
    r[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return r


def thrust_axis(q):
    """Body +z axis in the world frame, R(q) e3 (third column of R(q))."""
    return quat_to_matrix(q)[..., :, 2]


def rate_increment(omega, dt):
    """Unit quaternion exp(omega dt / 2) for a constant body rate omega."""
    n = np.linalg.norm(omega, axis=-1)
    half = 0.5 * n * dt
    # sin(half)/n, with its Taylor series where n is tiny (exact limit dt/2).
    small = half < 1e-4
    safe_n = np.where(small, 1.0, n)
    s_over_n = np.where(small, 0.5 * dt * (1.0 - half * half / 6.0), np.sin(half) / safe_n)
    return np.concatenate([np.cos(half)[..., None], s_over_n[..., None] * omega], axis=-1)


def rollout(x0, u, dt, mass, gravity):
    """Integrate rollouts from x0 under controls u (K, T, 4).

    Returns (p_rel, q, v): positions relative to p_0 with shape (K, T+1, 3),
    quaternions (K, T+1, 4) and velocities (K, T+1, 3) at steps 0..T.
    """
    K, T = u.shape[0], u.shape[1]
    p = np.zeros((K, T + 1, 3))
    q = np.zeros((K, T + 1, 4))
    v = np.zeros((K, T + 1, 3))
    q[:, 0] = x0[3:7]
    v[:, 0] = x0[7:10]
    e3 = np.array([0.0, 0.0, 1.0])
    for t in range(T):
        thrust = u[:, t, 0]
        rates = u[:, t, 1:4]
        a = (thrust / mass)[:, None] * thrust_axis(q[:, t]) - gravity * e3
        p[:, t + 1] = p[:, t] + v[:, t] * dt + 0.5 * a * dt * dt
        v[:, t + 1] = v[:, t] + a * dt
        q[:, t + 1] = quat_mul(q[:, t], rate_increment(rates, dt))
    return p, q, v


# ------------------------------------------------------------ rotor-thrust rates
#
# The paper's input (Section IV-A): u = (dT_1, dT_2, dT_3, dT_4)/dt, the
# rates of the four rotor thrusts (Table I bounds the rates to [-10, 10] N/s,
# the thrusts to [0, 10] N and the body rate to [-10, 10] rad/s).  The state
# grows by the four thrusts; the body rate becomes a state driven by the
# rotor torques.  Readings where the paper is silent (it gives no inertia,
# arm length or rotor layout):
#
# * "X" layout, rotor i at body (x_i, y_i) = a (s_x, s_y) with a = arm / sqrt 2
#   and (s_x, s_y) = (+,+), (-,-), (+,-), (-,+) for rotors 1..4; rotors 1, 2
#   and 3, 4 spin in opposite senses, the drag torque of rotor i is
#   kappa T_i about body z with sign +, +, -, -;
#   torque tau = sum_i (y_i T_i, -x_i T_i, +/- kappa T_i);
# * Euler's equations with a diagonal inertia J:
#   J domega/dt = tau - omega x (J omega);
# * one step dt, in this order: T_{t+1} = clip(T_t + u_t dt, 0, T_max);
#   omega_{t+1} = clip(omega_t + dt J^-1 (tau(T_{t+1}) - omega_t x J omega_t),
#   -omega_max, omega_max) (explicit Euler on the rate, clipped per axis);
#   then the collective-thrust step above with thrust sum_i T_{t+1,i} and
#   body rate omega_{t+1}.


def rotor_torque(thrusts, arm, kappa):
    """Body torque (..., 3) of rotor thrusts (..., 4) in the X layout."""
    a = arm / np.sqrt(2.0)
    t1, t2, t3, t4 = thrusts[..., 0], thrusts[..., 1], thrusts[..., 2], thrusts[..., 3]
    return np.stack([a * (t1 - t2 - t3 + t4), a * (-t1 + t2 - t3 + t4), kappa * (t1 + t2 - t3 - t4)], axis=-1)


def rotor_inputs(omega0, thrust0, u, dt, model):
    """Collective thrust and body rate per step (K, T, 4) that the rotor-rate
    controls u (K, T, 4) produce from body rate omega0 (3,) and rotor thrusts
    thrust0 (4,)."""
    K, T = u.shape[0], u.shape[1]
    J = np.asarray(model["inertia"], dtype=np.float64)
    thr = np.broadcast_to(np.asarray(thrust0, dtype=np.float64), (K, 4)).copy()
    w = np.broadcast_to(np.asarray(omega0, dtype=np.float64), (K, 3)).copy()
    out = np.zeros((K, T, 4))
    for t in range(T):
        thr = np.clip(thr + u[:, t] * dt, 0.0, model["thrust_max"])
        tau = rotor_torque(thr, model["arm_length"], model["yaw_coeff"])
        w = np.clip(w + dt * (tau - np.cross(w, J * w)) / J, -model["rate_max"], model["rate_max"])
        out[:, t, 0] = thr.sum(axis=1)
        out[:, t, 1:4] = w
    return out


def rotor_rollout(x0, thrust0, u, dt, model):
    """rollout() for rotor-thrust-rate controls u (K, T, 4); x0 carries the
    initial body rate in x0[10:13], thrust0 the four rotor thrusts."""
    return rollout(x0, rotor_inputs(x0[10:13], thrust0, u, dt, model), dt, model["mass"], model["gravity"])
