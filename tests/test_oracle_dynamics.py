"""Pins of the oracle's quadrotor rollout against closed forms (CPU only)."""
import numpy as np
import pytest

import scenarios as sc
from oracle import rollout, quat_mul, solve
from oracle.dynamics import rate_increment, quat_to_matrix

M, G = sc.MODEL["mass"], sc.MODEL["gravity"]


def _x0(p=(0, 0, 0), q=(1, 0, 0, 0), v=(0, 0, 0)):
    x = np.zeros(13)
    x[0:3], x[3:7], x[7:10] = p, q, v
    return x


def test_hover_thrust_gives_zero_acceleration():
    T, dt = 50, 0.02
    u = np.zeros((3, T, 4))
    u[..., 0] = M * G
    p, q, v = rollout(_x0(), u, dt, M, G)
    assert np.max(np.abs(p)) <= 1e-15 * T
    assert np.max(np.abs(v)) <= 1e-15 * T
    assert np.allclose(q, [1, 0, 0, 0], atol=0)


def test_free_fall_is_exact():
    T, dt = 60, 0.02
    v0 = np.array([3.0, -1.5, 7.0])
    u = np.zeros((1, T, 4))
    p, q, v = rollout(_x0(v=v0), u, dt, M, G)
    t = np.arange(T + 1) * dt
    exact = v0[None, :] * t[:, None] - 0.5 * G * (t ** 2)[:, None] * np.array([0, 0, 1.0])
    assert np.max(np.abs(p[0] - exact)) <= 1e-12
    assert np.max(np.abs(v[0] - (v0 - G * t[:, None] * np.array([0, 0, 1.0])))) <= 1e-12


def test_constant_yaw_rate_at_hover():
    T, dt, wz = 40, 0.02, 2.5
    u = np.zeros((1, T, 4))
    u[..., 0] = M * G
    u[..., 3] = wz
    p, q, v = rollout(_x0(), u, dt, M, G)
    ang = wz * np.arange(T + 1) * dt
    qe = np.stack([np.cos(ang / 2), 0 * ang, 0 * ang, np.sin(ang / 2)], axis=-1)
    assert np.max(np.abs(q[0] - qe)) <= 1e-13
    assert np.max(np.abs(p)) <= 1e-14 * T


def test_fixed_tilt_constant_thrust_parabola():
    T, dt, thrust = 30, 0.02, 6.0
    th = 0.3                                    # tilt about body x
    q0 = np.array([np.cos(th / 2), np.sin(th / 2), 0, 0])
    v0 = np.array([1.0, 2.0, -0.5])
    u = np.zeros((1, T, 4))
    u[..., 0] = thrust
    p, q, v = rollout(_x0(q=q0, v=v0), u, dt, M, G)
    # body z rotated by th about x: (0, -sin th, cos th)
    a = thrust / M * np.array([0.0, -np.sin(th), np.cos(th)]) - np.array([0, 0, G])
    t = np.arange(T + 1) * dt
    exact = v0[None] * t[:, None] + 0.5 * a[None] * (t ** 2)[:, None]
    assert np.max(np.abs(p[0] - exact)) <= 1e-12


def test_quaternion_norm_preserved_without_renormalisation():
    rng = np.random.default_rng(5)
    T = 200
    u = np.zeros((16, T, 4))
    u[..., 0] = rng.uniform(0, 10, size=(16, T))
    u[..., 1:] = rng.uniform(-10, 10, size=(16, T, 3))
    q0 = rng.standard_normal(4)
    q0 /= np.linalg.norm(q0)
    _, q, _ = rollout(_x0(q=q0), u, 0.02, M, G)
    assert np.max(np.abs(np.linalg.norm(q, axis=-1) - 1.0)) <= 1e-13


def test_rate_increment_small_angle_branch_is_continuous():
    dt = 0.02
    for n in [1e-3, 5e-3, 1e-2, 1e-1]:
        w = np.array([[n, 0.0, 0.0]])
        dq = rate_increment(w, dt)[0]
        exact = [np.cos(n * dt / 2), np.sin(n * dt / 2), 0, 0]
        assert np.allclose(dq, exact, rtol=0, atol=1e-16)
    assert np.array_equal(rate_increment(np.zeros((1, 3)), dt)[0], [1, 0, 0, 0])


def test_quaternion_product_matches_rotation_composition():
    rng = np.random.default_rng(2)
    a = rng.standard_normal(4); a /= np.linalg.norm(a)
    b = rng.standard_normal(4); b /= np.linalg.norm(b)
    Ra, Rb, Rab = quat_to_matrix(a), quat_to_matrix(b), quat_to_matrix(quat_mul(a, b))
    assert np.allclose(Ra @ Rb, Rab, atol=1e-14)
    assert np.allclose(Ra @ Ra.T, np.eye(3), atol=1e-14)


def _scene(seed, **over):
    return sc.make_problem(K=64, T=12, G=3, rot="haar", start="moving", seed=seed,
                           d_safe=1.0, **over)


def _rotz(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1.0]])


@pytest.mark.parametrize("sdf_kind", ["analytic", "mlp"])
def test_scene_translation_leaves_update_unchanged(sdf_kind):
    W, b = sc.xavier_weights((67, 16, 16, 1), seed=3, bias_scale=0.5)
    p = _scene(11)
    r1 = solve(p, (W, b), sc.MODEL, sdf_kind=sdf_kind)
    shift = np.array([12.5, -7.25, 3.0])
    p2 = dict(p)
    p2["x0"] = p["x0"].copy(); p2["x0"][0:3] += shift
    p2["wp"] = p["wp"] + shift
    p2["gate_t"] = p["gate_t"] + shift
    r2 = solve(p2, (W, b), sc.MODEL, sdf_kind=sdf_kind)
    assert np.allclose(r1["J"], r2["J"], rtol=0, atol=1e-9 * (1 + np.abs(r1["J"]).max()))
    assert np.allclose(r1["U_star"], r2["U_star"], rtol=0, atol=1e-12)


@pytest.mark.parametrize("sdf_kind", ["analytic", "mlp"])
def test_scene_yaw_rotation_leaves_update_unchanged(sdf_kind):
    W, b = sc.xavier_weights((67, 16, 16, 1), seed=3, bias_scale=0.5)
    p = _scene(12)
    r1 = solve(p, (W, b), sc.MODEL, sdf_kind=sdf_kind)
    a = 0.7
    Rz = _rotz(a)
    p2 = dict(p)
    x0 = p["x0"].copy()
    x0[0:3] = Rz @ x0[0:3]
    x0[3:7] = quat_mul(np.array([np.cos(a / 2), 0, 0, np.sin(a / 2)]), x0[3:7])
    x0[7:10] = Rz @ x0[7:10]
    p2["x0"] = x0
    p2["wp"] = Rz @ p["wp"]
    p2["gate_t"] = p["gate_t"] @ Rz.T
    p2["gate_R"] = np.einsum("ij,gjk->gik", Rz, p["gate_R"])
    r2 = solve(p2, (W, b), sc.MODEL, sdf_kind=sdf_kind)
    assert np.allclose(r1["J"], r2["J"], rtol=0, atol=1e-9 * (1 + np.abs(r1["J"]).max()))
    assert np.allclose(r1["U_star"], r2["U_star"], rtol=0, atol=1e-11)


# ---------------------------------------------------------- rotor-thrust rates
from oracle.dynamics import rotor_inputs, rotor_rollout, rotor_torque  # noqa: E402

RM = sc.ROTOR_MODEL


def test_rotor_hover_thrusts_hold_position_and_attitude():
    """Four equal thrusts m g / 4, zero rates, zero body rate: no torque, no
    acceleration (the rotor form of the hover pin)."""
    T, dt = 50, 0.02
    thr = np.full(4, RM["mass"] * RM["gravity"] / 4.0)
    p, q, v = rotor_rollout(_x0(), thr, np.zeros((2, T, 4)), dt, RM)
    assert np.max(np.abs(p)) <= 1e-14
    assert np.max(np.abs(v)) <= 1e-14
    assert np.allclose(q, [1, 0, 0, 0], atol=0)


def test_rotor_torque_layout():
    """X layout: a differential between rotor pairs gives a pure roll, pitch
    or yaw torque of the closed-form size."""
    a, kap = RM["arm_length"] / np.sqrt(2.0), RM["yaw_coeff"]
    c, d = 1.0, 0.1
    assert np.allclose(rotor_torque(np.array([c + d, c - d, c - d, c + d]), RM["arm_length"], kap), [4 * a * d, 0, 0])
    assert np.allclose(rotor_torque(np.array([c - d, c + d, c - d, c + d]), RM["arm_length"], kap), [0, 4 * a * d, 0])
    assert np.allclose(rotor_torque(np.array([c + d, c + d, c - d, c - d]), RM["arm_length"], kap), [0, 0, 4 * kap * d])
    assert np.allclose(rotor_torque(np.full(4, 2.0), RM["arm_length"], kap), 0.0, atol=0)


def test_rotor_yaw_differential_spins_up_linearly():
    """Constant yaw torque about a principal axis: no gyroscopic term, the
    explicit-Euler rate is n dt tau_z / J_z exactly; collective thrust is
    the sum of the four thrusts."""
    T, dt, c, d = 20, 0.01, 0.9, 0.05
    thr = np.array([c + d, c + d, c - d, c - d])
    inp = rotor_inputs(np.zeros(3), thr, np.zeros((1, T, 4)), dt, RM)
    n = np.arange(1, T + 1)
    assert np.allclose(inp[0, :, 3], n * dt * 4 * RM["yaw_coeff"] * d / RM["inertia"][2], rtol=1e-13, atol=0)
    assert np.max(np.abs(inp[0, :, 1:3])) == 0.0
    assert np.allclose(inp[0, :, 0], 4 * c, rtol=1e-15)


def test_rotor_gyroscopic_term_sign():
    """Torque-free body spinning about x and z: one Euler step changes the y
    rate by dt (J_z - J_x) / J_y w_z w_x (the sign of omega x J omega)."""
    dt, wx, wz = 0.005, 1.5, -2.0
    thr = np.full(4, 1.0)
    inp = rotor_inputs(np.array([wx, 0.0, wz]), thr, np.zeros((1, 1, 4)), dt, RM)
    Jx, Jy, Jz = RM["inertia"]
    assert np.isclose(inp[0, 0, 2], dt * (Jz - Jx) / Jy * wz * wx, rtol=1e-13, atol=0)
    assert np.isclose(inp[0, 0, 1], wx, rtol=0, atol=1e-15)      # (J_y - J_z) w_y w_z = 0
    assert np.isclose(inp[0, 0, 3], wz, rtol=0, atol=1e-15)


def test_rotor_thrust_and_rate_limits():
    """Rates integrate the thrusts and saturate at Table I's bounds; zero
    thrusts fall freely (the rotor form of the free-fall pin)."""
    T, dt = 30, 0.05
    u = np.full((1, T, 4), 10.0)
    inp = rotor_inputs(np.zeros(3), np.full(4, 8.0), u, dt, RM)
    assert np.allclose(inp[0, :, 0], np.minimum(4 * (8.0 + 10.0 * dt * np.arange(1, T + 1)), 40.0))
    p, q, v = rotor_rollout(_x0(v=(1.0, 0, 0)), np.zeros(4), np.full((1, T, 4), -10.0), dt, RM)
    t = np.arange(T + 1) * dt
    assert np.max(np.abs(p[0, :, 2] + 0.5 * G * t ** 2)) <= 1e-12
    assert np.max(np.abs(p[0, :, 0] - t)) <= 1e-12
    big = rotor_inputs(np.array([0.0, 0.0, 9.99]), np.array([0.0, 0.0, 10.0, 10.0]), np.zeros((1, 5, 4)), 0.1, RM)
    assert np.all(np.abs(big[0, :, 1:4]) <= RM["rate_max"])


def test_rotor_solve_zero_noise_returns_nominal():
    """MPPI invariant under the rotor input: zero noise gives back the
    nominal rate sequence."""
    prob = sc.rotor_problem(16, 10, 1, seed=3, start="moving", Sigma=np.zeros((4, 4)))
    W, b = sc.xavier_weights((67, 32, 32, 1), seed=1)
    U = np.random.default_rng(0).uniform(-2, 2, size=(10, 4))
    out = solve(prob, (W, b), RM, U_nom=U)
    assert np.allclose(out["U_star"], U, rtol=0, atol=1e-12)
