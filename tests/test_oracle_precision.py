"""Precision pin of the FP64 oracle at the high-resolution end (N_side 4096,
K = 32, lmax 4096) against an independent 80-bit long-double evaluation of the
same definition: correlation sums by the plain Legendre recurrence, S + eps I
factorised and solved in long double.  The kriging variance there is ~6e-9 of
sigma0^2, a cancellation, so this guards the oracle's solve strategy."""
import numpy as np
import pytest

from oracle import correlation, healpix, kriging
from workload import spectra


def _zeta_ld(u, cl):
    ul = u.astype(np.longdouble)
    ell = np.arange(len(cl))
    w = ((2 * ell + 1) / (4 * np.pi) * cl).astype(np.longdouble)
    w[0] = 0
    p_prev, p = np.ones_like(ul), 1 - ul
    tot = w[0] * p_prev + w[1] * p
    for l in range(1, len(cl) - 1):
        p_prev, p = p, ((2 * l + 1) * (1 - ul) * p - l * p_prev) / (l + 1)
        tot = tot + w[l + 1] * p
    return tot / w.sum()


def _chol_solve_ld(S, b):
    n = S.shape[0]
    L = np.zeros_like(S)
    for j in range(n):
        d = S[j, j] - np.sum(L[j, :j] ** 2)
        L[j, j] = np.sqrt(d)
        L[j + 1:, j] = (S[j + 1:, j] - L[j + 1:, :j] @ L[j, :j]) / L[j, j]
    y = np.zeros_like(b)
    for i in range(n):
        y[i] = (b[i] - L[i, :i] @ y[:i]) / L[i, i]
    x = np.zeros_like(b)
    for i in range(n - 1, -1, -1):
        x[i] = (y[i] - L[i + 1:, i] @ x[i + 1:]) / L[i, i]
    return x


def test_variance_vs_long_double_nside4096():
    nside, K, lmax = 4096, 32, 4096
    tt = spectra.cl_acoustic(lmax)[0]
    rng = np.random.default_rng(7)
    th = np.arccos(rng.uniform(-0.9, 0.9, 3))
    ph = rng.uniform(0, 2 * np.pi, 3)
    st = kriging.stencils(nside, th, ph, K)
    vals = rng.normal(size=(3, K))      # map values do not enter the variance
    _, var, _ = kriging.interpolate(nside, tt, K, 0, lambda pix: vals, th, ph, stencil_idx=st)
    s2 = correlation.zeta(np.zeros(1), tt)[0][0]
    for i in range(3):
        pts = np.concatenate([healpix.ang2vec(th[i], ph[i])[None], healpix.pix2vec(nside, st[i])])
        u = 0.5 * np.sum((pts[:, None] - pts[None]) ** 2, -1)
        V = _zeta_ld(u, tt)
        S = V[1:, 1:] + np.longdouble(kriging.EPS_F64) * np.eye(K, dtype=np.longdouble)
        b = V[1:, 0]
        w = _chol_solve_ld(S, b)
        var_ld = float(1 - b @ w) * s2
        assert 1e-10 * s2 < var_ld < 1e-7 * s2          # the regime this pin is about
        assert var[i] == pytest.approx(var_ld, rel=1e-3)
