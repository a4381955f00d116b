"""Lensing pipeline steps for the oracle (test infrastructure only).

The paper's lensing pipeline (Sec. 3.1): synthesise the unlensed maps and the
deflection field d = grad(phi) from their harmonic coefficients, move every
pixel centre n to n' = cos|d| n + sin|d| d/|d| (the vector form, which needs no
special case at the poles), and interpolate the unlensed maps at n'.

* synth_points: spin-s synthesis F(n) = sum_{l,m} a_lm sY_lm(n) at arbitrary
  directions by brute force, with sY_lm from wigner.sY (the explicit Wigner-d
  formula of App. A; tiny lmax only).  The coefficients are given for m >= 0 as
  a = e + i b, where e and b are each those of a real-type field,
  e_{l,-m} = (-1)^m conj(e_lm) (likewise b).  Then
    spin 0, e = a^T:                 F = T;
    spin 1, e = -sqrt(l(l+1)) phi_lm: F = d_theta + i d_phi (the gradient of phi);
    spin 2, e = -E, b = -B:           F = Q + i U (P = sum 2a_lm 2Y_lm,
                                       2a_lm = -(E_lm + i B_lm)).
* synth_points_spin0_scipy: spin-0 synthesis with scipy's spherical harmonics
  (a library routine; usable at larger l than the explicit formula).
* synth_points_eth: the same synthesis with sY_lm built from scipy's Y_lm and
  its analytic theta/phi derivatives by the spin-raising operator,
  1Y = eth Y / sqrt(l(l+1)) and 2Y = eth^2 Y / sqrt((l-1) l (l+1) (l+2)) with
  eth Y = -(Y_t + i Y_p / sin t) and
  eth^2 Y = Y_tt - cot t Y_t - Y_pp / sin^2 t + 2i (Y_tp - cot t Y_p) / sin t
  (scipy's harmonics are finite to l ~ 600).
* synth_points_recurrence: the same synthesis at any l, with d^l_{m,s'} from
  the standard three-term recurrence in l at fixed (m, s'), started from the
  closed form at l = max(m, |s'|) and carried in scaled arithmetic
  (mantissa x 2^E) so that seeds that underflow near the poles stay exact;
  the negative orders come from d^l_{-m,-s} = (-1)^{m+s} d^l_{m,s}.
* lensed_directions: the vector-form displacement.

Pins (tests/test_oracle_lensing.py): spin 1 against the finite-difference
gradient of the resummed potential; spin 0 against scipy's harmonics; spin 2
against wigner.resum_spin2; synth_points_eth against synth_points (l <= 10);
synth_points_recurrence against synth_points (l <= 10, points at the poles
included) and synth_points_eth (l ~ 300), its d^l_{00} against scipy's
Legendre P_l to l = 4096 and its rows against the unitarity of the rotation
matrix, sum_m (d^l_{m,s})^2 = 1, to l = 2048; the displacement preserves |n|,
moves n by the angle |d| along the bearing of d, and is the identity for
d = 0.
"""
import numpy as np

from . import wigner


def _coeff(a, l, m):
    """a_{l,m} for any m from the stored m >= 0 half (real-type rule)."""
    if m >= 0:
        return a[l, m]
    return (-1) ** m * np.conj(a[l, -m])


def synth_points(spin, elm, blm, theta, phi):
    """F(theta, phi) = sum_{l, m} (e + i b)_lm sY_lm (complex; tiny lmax)."""
    theta = np.asarray(theta, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    lmax = elm.shape[0] - 1
    if blm is None:
        blm = np.zeros_like(elm)
    out = np.zeros(np.broadcast(theta, phi).shape, dtype=np.complex128)
    for l in range(abs(spin), lmax + 1):
        for m in range(-l, l + 1):
            a = _coeff(elm, l, m) + 1j * _coeff(blm, l, m)
            if a != 0:
                out += a * wigner.sY(spin, l, m, theta, phi)
    return out


def synth_points_spin0_scipy(alm, theta, phi):
    """T(theta, phi) = sum_{l,m} a_lm Y_lm with scipy's Y_lm (real field)."""
    from scipy.special import sph_harm_y
    theta = np.asarray(theta, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    lmax = alm.shape[0] - 1
    out = np.zeros(np.broadcast(theta, phi).shape, dtype=np.float64)
    for l in range(lmax + 1):
        for m in range(0, l + 1):
            if alm[l, m] == 0:
                continue
            y = sph_harm_y(l, m, theta, phi)
            term = alm[l, m] * y
            out += term.real if m == 0 else 2.0 * term.real
    return out


def lensed_directions(theta, phi, d_theta, d_phi):
    """(theta', phi') of n' = cos|d| n + sin|d| (d_theta e_theta + d_phi e_phi)/|d|."""
    theta = np.asarray(theta, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    st, ct = np.sin(theta), np.cos(theta)
    sp, cp = np.sin(phi), np.cos(phi)
    n = np.stack([st * cp, st * sp, ct], axis=-1)
    et = np.stack([ct * cp, ct * sp, -st], axis=-1)
    ep = np.stack([-sp, cp, np.zeros_like(sp)], axis=-1)
    dmod = np.hypot(d_theta, d_phi)
    safe = np.where(dmod > 0, dmod, 1.0)
    dhat = (np.asarray(d_theta)[..., None] * et + np.asarray(d_phi)[..., None] * ep) / safe[..., None]
    npr = np.cos(dmod)[..., None] * n + np.sin(dmod)[..., None] * dhat
    th2 = np.arctan2(np.hypot(npr[..., 0], npr[..., 1]), npr[..., 2])
    ph2 = np.mod(np.arctan2(npr[..., 1], npr[..., 0]), 2 * np.pi)
    return th2, ph2


def sY_eth(s, l, m, theta, phi):
    """sY_lm (s = 0, 1, 2) from scipy's Y_lm and its derivatives (eth route)."""
    from scipy.special import sph_harm_y
    theta = np.asarray(theta, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    if l < s:
        return np.zeros(np.broadcast(theta, phi).shape, dtype=np.complex128)
    Y, J, H = sph_harm_y(l, m, theta, phi, diff_n=2)
    if s == 0:
        return Y
    st, ct = np.sin(theta), np.cos(theta)
    Yt, Yp = J[..., 0], J[..., 1]
    if s == 1:
        return -(Yt + 1j * Yp / st) / np.sqrt(l * (l + 1.0))
    Ytt, Ytp, Ypp = H[..., 0, 0], H[..., 0, 1], H[..., 1, 1]
    e2 = Ytt - ct / st * Yt - Ypp / st ** 2 + 2j * (Ytp - ct / st * Yp) / st
    return e2 / np.sqrt((l - 1.0) * l * (l + 1.0) * (l + 2.0))


def synth_points_eth(spin, elm, blm, theta, phi):
    """F = sum_{l,m} (e + i b)_lm sY_lm through sY_eth (l <= ~600)."""
    theta = np.asarray(theta, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    lmax = elm.shape[0] - 1
    if blm is None:
        blm = np.zeros_like(elm)
    out = np.zeros(np.broadcast(theta, phi).shape, dtype=np.complex128)
    for l in range(abs(spin), lmax + 1):
        ms = np.arange(-l, l + 1)
        a = np.array([_coeff(elm, l, m) + 1j * _coeff(blm, l, m) for m in range(-l, l + 1)])
        Y = sY_eth(spin, l, ms[:, None], theta[None, ...], phi[None, ...])
        out += np.tensordot(a, Y, axes=(0, 0))
    return out


_SCALE = 480   # rescaling step (bits) of the scaled recurrence


def _pw(k, lnx):
    """k ln x with 0 ln 0 = 0 (x^0 = 1 at the poles)."""
    with np.errstate(invalid="ignore"):
        return np.where(k == 0, 0.0, k * lnx)


def _seed_log2(m, sp, lc, ls):
    """log2 |d^{l0}_{m,sp}| and its sign at l0 = max(m, |sp|) (closed forms),
    for an int array m, scalar sp and angles given by lc = ln cos(t/2),
    ls = ln sin(t/2) (shape (npts, 1))."""
    from scipy.special import gammaln
    s = abs(sp)
    m = np.asarray(m)
    ln = np.empty(np.broadcast(m, lc).shape)
    sign = np.ones(m.shape)
    hi = m >= s
    # l0 = m: d^m_{m,sp} = (-1)^{m-sp} sqrt((2m)!/((m+sp)!(m-sp)!)) c^{m+sp} s^{m-sp}
    mh = np.where(hi, m, s)
    ln_hi = (0.5 * (gammaln(2.0 * mh + 1) - gammaln(mh + sp + 1.0) - gammaln(mh - sp + 1.0))
             + _pw(mh + sp, lc) + _pw(mh - sp, ls))
    sign_hi = np.where((mh - sp) % 2 == 1, -1.0, 1.0)
    # l0 = s > m: d^s_{m,s} = sqrt((2s)!/((s+m)!(s-m)!)) c^{s+m} s^{s-m};
    #             d^s_{m,-s} = (-1)^{m+s} sqrt((2s)!/((s-m)!(s+m)!)) c^{s-m} s^{s+m}
    ml = np.where(hi, 0, m)
    if sp >= 0:
        ln_lo = (0.5 * (gammaln(2.0 * s + 1) - gammaln(s + ml + 1.0) - gammaln(s - ml + 1.0))
                 + _pw(s + ml, lc) + _pw(s - ml, ls))
        sign_lo = np.ones(m.shape)
    else:
        ln_lo = (0.5 * (gammaln(2.0 * s + 1) - gammaln(s - ml + 1.0) - gammaln(s + ml + 1.0))
                 + _pw(s - ml, lc) + _pw(s + ml, ls))
        sign_lo = np.where((ml + s) % 2 == 1, -1.0, 1.0)
    ln = np.where(hi, ln_hi, ln_lo)
    sign = np.where(hi, sign_hi, sign_lo)
    return ln / np.log(2.0), sign


def wigner_d_by_l(sp, lmax, theta):
    """Yields (l, d) for l = 0..lmax, d[p, m] = d^l_{m,sp}(theta_p) for
    0 <= m <= lmax (zero where m > l or l < |sp|)."""
    theta = np.atleast_1d(np.asarray(theta, dtype=np.float64))[:, None]
    x = np.cos(theta)
    # cos(t/2) = sin((pi - t)/2) keeps its relative accuracy near the south pole
    with np.errstate(divide="ignore"):
        lc = np.log(np.where(theta > 0.5 * np.pi, np.sin(0.5 * (np.pi - theta)), np.cos(0.5 * theta)))
        ls = np.log(np.sin(0.5 * theta))
    m = np.arange(lmax + 1)
    s = abs(sp)
    l0 = np.maximum(m, s)
    shape = (theta.shape[0], lmax + 1)
    cur = np.zeros(shape)
    prev = np.zeros(shape)
    E = np.zeros(shape, dtype=np.int64)
    lg2, sign = _seed_log2(m, sp, lc, ls)
    with np.errstate(invalid="ignore"):
        E0 = _SCALE * np.floor(lg2 / _SCALE)
        E0 = np.where(np.isfinite(E0), E0, -(1 << 40)).astype(np.int64)
        mant0 = sign * np.exp2(np.where(np.isfinite(lg2), lg2 - E0, -np.inf))
    mf = m.astype(np.float64)
    for l in range(0, lmax + 1):
        start = l0 == l
        if np.any(start):
            cur[:, start] = mant0[:, start]
            prev[:, start] = 0.0
            E[:, start] = E0[:, start]
        act = l0 <= l
        with np.errstate(under="ignore"):
            d = np.where(act[None, :], cur * np.exp2(np.maximum(E, -1100).astype(np.float64)), 0.0)
        yield l, d
        if l == lmax:
            break
        # d^{l+1} = [(2l+1)(l(l+1)x - m sp) d^l - (l+1) sqrt((l^2-m^2)(l^2-sp^2)) d^{l-1}]
        #           / [l sqrt(((l+1)^2-m^2)((l+1)^2-sp^2))]
        if l == 0:
            nxt = x * cur
        else:
            with np.errstate(invalid="ignore", divide="ignore"):
                den = l * np.sqrt(((l + 1.0) ** 2 - mf ** 2) * ((l + 1.0) ** 2 - sp * sp))
                a = (2 * l + 1.0) * (l * (l + 1.0) * x - mf * sp) / den
                b = (l + 1.0) * np.sqrt(np.maximum((l * l - mf ** 2) * (l * l - sp * sp), 0.0)) / den
                nxt = np.where(act[None, :], a * cur - b * prev, 0.0)
        prev, cur = np.where(act[None, :], cur, prev), nxt
        big = (np.abs(cur) > 2.0 ** _SCALE) & (E < 0)
        if np.any(big):
            cur = np.where(big, cur * 2.0 ** -_SCALE, cur)
            prev = np.where(big, prev * 2.0 ** -_SCALE, prev)
            E = np.where(big, E + _SCALE, E)


def synth_points_recurrence(spin, elm, blm, theta, phi):
    """F = sum_{l,m} (e + i b)_lm sY_lm with sY_lm = (-1)^s N_l e^{i m phi}
    d^l_{m,-s}(theta) and the d from wigner_d_by_l (any l)."""
    theta = np.atleast_1d(np.asarray(theta, dtype=np.float64))
    phi = np.atleast_1d(np.asarray(phi, dtype=np.float64))
    lmax = elm.shape[0] - 1
    if blm is None:
        blm = np.zeros_like(elm)
    m = np.arange(lmax + 1)
    eimp = np.exp(1j * phi[:, None] * m[None, :])       # e^{i m phi}
    sgn_m = np.where(m % 2 == 1, -1.0, 1.0)
    out = np.zeros(theta.shape, dtype=np.complex128)
    gen_neg = wigner_d_by_l(-spin, lmax, theta)          # d^l_{m,-s}
    gen_pos = wigner_d_by_l(spin, lmax, theta) if spin else None
    for l, dneg in gen_neg:
        dpos = next(gen_pos)[1] if spin else dneg
        if l < spin:
            continue
        nl = np.sqrt((2 * l + 1) / (4 * np.pi))
        e, b = elm[l], blm[l]
        # m >= 0: a_lm = e + i b
        ap = e + 1j * b
        tot = np.sum(ap[None, :] * eimp * dneg, axis=1)
        # m = -mu < 0: a = (-1)^mu conj(e) + i (-1)^mu conj(b) and
        # d^l_{-mu,-s} = (-1)^{mu+s} d^l_{mu,s}
        an = sgn_m * (np.conj(e) + 1j * np.conj(b))
        dn = sgn_m * (-1.0) ** spin * dpos
        tot += np.sum((an * (m > 0))[None, :] * np.conj(eimp) * dn, axis=1)
        out += (-1.0) ** spin * nl * tot
    return out
