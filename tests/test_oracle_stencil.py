"""The oracle's windowed K-nearest search equals brute force over all pixels."""
import numpy as np
import pytest

from oracle import healpix, kriging


def _brute(N, th, ph, K):
    v = healpix.all_vec(N)
    t = healpix.ang2vec(th, ph)
    u = 0.5 * np.sum((v - t) ** 2, -1)
    order = np.lexsort((np.arange(len(u)), u))
    return order[:K]


@pytest.mark.parametrize("N,K", [(2, 5), (8, 16), (16, 32), (32, 48), (16, 64)])
def test_window_equals_brute_force(N, K):
    rng = np.random.default_rng(N * 100 + K)
    th = np.concatenate([np.arccos(rng.uniform(-1, 1, 60)),
                         [0.0, np.pi, 1e-4, np.pi - 1e-4, np.arccos(2 / 3), np.arccos(-2 / 3), np.pi / 2]])
    ph = np.concatenate([rng.uniform(-7, 14, 60), [0.3, 2.0, 0.0, 6.283185307179586, 1e-12, -1e-12, 2 * np.pi - 1e-13]])
    st = kriging.stencils(N, th, ph, K)
    for i in range(len(th)):
        ref = _brute(N, th[i], ph[i], K)
        assert np.array_equal(st[i], ref), (N, K, th[i], ph[i])


def test_tie_break_smaller_index():
    """At a pole all pixels of the first ring are equidistant: the smaller index wins."""
    st = kriging.stencils(8, np.array([0.0]), np.array([0.0]), 2)
    assert list(st[0]) == [0, 1]
