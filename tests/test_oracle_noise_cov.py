"""Pins of the oracle's control noise with a full covariance (CPU only).

Section IV-A perturbs the nominal sequence with delta u ~ N(0, Sigma); the
oracle samples L n with L L^T = Sigma.  Pins: the factor reproduces Sigma
and equals the library Cholesky routine for a positive definite Sigma; a
semi-definite Sigma factors too (zero pivot -> zero column); non-PSD
matrices are refused; 10^6 drawn perturbations have Sigma as their
covariance within 5 standard errors.
"""
import numpy as np
import pytest

import scenarios as sc
from oracle import control_noise
from oracle.mppi import noise_factor, sample_controls


def _spd(seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((4, 4)) * np.array([2.0, 0.5, 0.5, 0.3])[:, None]
    return A @ A.T + 1e-3 * np.eye(4)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_factor_of_positive_definite_sigma(seed):
    S = _spd(seed)
    L = noise_factor(S)
    assert np.array_equal(L, np.tril(L))
    assert np.max(np.abs(L @ L.T - S)) <= 1e-15 * 4 * np.max(np.abs(S))
    assert np.allclose(L, np.linalg.cholesky(S), rtol=0, atol=1e-14 * np.max(np.abs(L)))


def test_factor_of_semidefinite_sigma():
    # rank 3: rows 1 and 2 of B coincide, dyadic entries keep every pivot exact
    B = np.array([[2.0, 0.0, 0.0], [1.0, 0.5, 0.0], [1.0, 0.5, 0.0], [0.25, 0.0, 0.5]])
    S = B @ B.T
    with pytest.raises(np.linalg.LinAlgError):
        np.linalg.cholesky(S)
    L = noise_factor(S)
    assert np.array_equal(L, np.tril(L))
    assert np.max(np.abs(L @ L.T - S)) <= 1e-15 * np.max(np.abs(S))
    assert L[2, 2] == 0.0 and np.all(L[3:, 2] == 0.0)
    # a zero variance on the diagonal (diagonal Sigma) is a zero row
    Ld = noise_factor(np.diag([4.0, 0.0, 0.25, 0.09]))
    assert np.array_equal(Ld, np.diag([2.0, 0.0, 0.5, 0.3]))


@pytest.mark.parametrize("S", [
    np.array([[1.0, 2.0, 0, 0], [2.0, 1.0, 0, 0], [0, 0, 1.0, 0], [0, 0, 0, 1.0]]),   # indefinite
    np.array([[1.0, 0.1, 0, 0], [0.0, 1.0, 0, 0], [0, 0, 1.0, 0], [0, 0, 0, 1.0]]),   # not symmetric
    np.diag([1.0, -0.1, 1.0, 1.0]),                                                   # negative variance
    np.array([[0.0, 0.5, 0, 0], [0.5, 1.0, 0, 0], [0, 0, 1.0, 0], [0, 0, 0, 1.0]]),   # zero pivot, non-zero column
])
def test_non_psd_sigma_is_refused(S):
    with pytest.raises(ValueError):
        noise_factor(S)


def test_empirical_covariance_of_a_million_draws():
    S = _spd(7)
    L = noise_factor(S)
    K, T = 10_000, 100
    eps = control_noise(11, 3, 2, K, T).reshape(-1, 4) @ L.T
    N = eps.shape[0]
    mean = eps.mean(axis=0)
    assert np.all(np.abs(mean) <= 5.0 * np.sqrt(np.diag(S) / N))
    C = eps.T @ eps / N
    se = np.sqrt((np.outer(np.diag(S), np.diag(S)) + S * S) / N)
    assert np.all(np.abs(C - S) <= 5.0 * se), np.max(np.abs(C - S) / se)


def test_samples_are_nominal_plus_factor_times_normals():
    S = _spd(3)
    prob = sc.make_problem(64, 9, 1, seed=2, Sigma=S, instance_id=5, tick=4)
    model = dict(sc.MODEL, u_lo=np.full(4, -1e9), u_hi=np.full(4, 1e9))
    U = np.tile([3.0, 0.1, -0.2, 0.05], (9, 1))
    u = sample_controls(prob, model, U)
    n = control_noise(prob["seed"], 5, 4, 64, 9)
    assert np.allclose(u - U[None], n @ noise_factor(S).T, rtol=0, atol=1e-14)
