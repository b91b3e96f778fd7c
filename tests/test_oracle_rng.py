"""Pins of the oracle's counter-based noise (CPU only).

* Philox4x64-10 against NumPy's own Philox bit generator (a library
  implementation of the same SC'11 generator).
* The uniform map and Box-Muller normals against distributional facts:
  moments and a Kolmogorov-Smirnov test of N(0, 1), independence of the
  four channels, and the exact range of the uniforms.
"""
import numpy as np
import pytest
from scipy import stats

from oracle import philox4x64_10, uniforms_from_words, box_muller, control_noise


def _numpy_block(ctr, key):
    """NumPy's Philox output block for counter ``ctr`` (it increments word 0
    before producing a block, so start it one below)."""
    ctr = np.array(ctr, dtype=np.uint64)
    start = ctr.copy()
    assert start[0] > 0
    start[0] -= np.uint64(1)
    bg = np.random.Philox(counter=start, key=np.array(key, dtype=np.uint64))
    return bg.random_raw(4)


@pytest.mark.parametrize("ctr,key", [
    ([1, 0, 0, 0], [0, 0]),
    ([7, 3, 11, 13], [0xDEADBEEF12345678, 99]),
    ([2**63 + 5, 2**64 - 1, 2**40 + 1, 77], [2**64 - 1, 2**64 - 2]),
    ([4095, 49, 123456789, 9], [0, 0]),
])
def test_philox_matches_numpy_generator(ctr, key):
    mine = philox4x64_10(np.array(ctr, dtype=np.uint64), np.array(key, dtype=np.uint64))
    assert np.array_equal(mine, _numpy_block(ctr, key))


def test_philox_vectorised_matches_numpy_stream():
    key = np.array([12345, 678], dtype=np.uint64)
    bg = np.random.Philox(counter=np.zeros(4, dtype=np.uint64), key=key)
    stream = bg.random_raw(4 * 1000).reshape(1000, 4)
    ctr = np.zeros((1000, 4), dtype=np.uint64)
    ctr[:, 0] = np.arange(1, 1001, dtype=np.uint64)
    assert np.array_equal(philox4x64_10(ctr, key), stream)


def test_uniform_map_range_and_exactness():
    words = np.array([0, 2**41 - 1, 2**41, 2**64 - 1], dtype=np.uint64)
    u = uniforms_from_words(words)
    assert u[0] == 2.0 ** -24 and u[1] == 2.0 ** -24
    assert u[2] == 3 * 2.0 ** -24
    assert u[3] == 1.0 - 2.0 ** -24
    # every value is exactly representable in float32
    assert np.array_equal(u.astype(np.float32).astype(np.float64), u)


def test_box_muller_known_points():
    # radius sqrt(-2 ln u0) = 1 at u0 = exp(-1/2); angle 2 pi u1
    u = np.array([[np.exp(-0.5), 0.125, np.exp(-2.0), 0.5]])
    n = box_muller(u)[0]
    assert np.allclose(n, [np.sqrt(0.5), np.sqrt(0.5), -2.0, 0.0], atol=1e-15)


def test_normals_distribution():
    n = control_noise(seed=0, instance_id=3, tick=1, K=4096, T=64)   # 1,048,576 normals
    flat = n.reshape(-1, 4)
    N = flat.shape[0]
    for c in range(4):
        x = flat[:, c]
        assert abs(x.mean()) < 5.0 / np.sqrt(N)
        assert abs(x.var() - 1.0) < 5.0 * np.sqrt(2.0 / N)
        assert stats.kstest(x, "norm").pvalue > 1e-4
    corr = np.corrcoef(flat.T)
    assert np.max(np.abs(corr - np.eye(4))) < 5.0 / np.sqrt(N)


def test_noise_counter_fields_change_streams():
    a = control_noise(0, 0, 0, 8, 4)
    assert not np.allclose(a, control_noise(1, 0, 0, 8, 4))
    assert not np.allclose(a, control_noise(0, 1, 0, 8, 4))
    assert not np.allclose(a, control_noise(0, 0, 1, 8, 4))
    # counter = (k, t, ...): a bigger problem contains the smaller one
    big = control_noise(0, 0, 0, 16, 6)
    assert np.array_equal(big[:8, :4], a)
