"""Quadrotor rollout f(x, u) for MPPI (oracle side), float64.

Section IV-A uses a standard quadrotor model with state [p, v, q, omega].
The paper's input is four rotor-thrust rates; here the input is collective
thrust + body rates, the form of the workloads the library is measured on.
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
