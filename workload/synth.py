"""Gaussian a_lm draws and spin-s HEALPix synthesis at pixel centres.

F_s(n) = sum_{l,m} e_lm sY_lm(n) with e_{l,-m} = (-1)^m conj(e_lm) ("E-type"
coefficients of a real scalar potential), sY_lm = (-1)^s sqrt((2l+1)/4pi)
e^{i m phi} d^l_{m,-s}(theta).  With this convention
  T            = F_0 with e = a^T,
  Q + i U      = F_2 with e = -a^E (B = 0),
  d_th + i d_ph = F_1 with e = -sqrt(l(l+1)) phi_lm   (gradient of phi).
The Wigner d_{m, +-s}(theta) are advanced by their three-term l-recurrence, all
(m, ring) pairs at once, in scaled arithmetic (mantissa x 2^E) so that seeds
like sin^m(theta/2) that underflow double precision near the poles stay exact.
On CPU the recurrences run as torch tensor loops; on a GPU device the Legendre
stage runs in a small HIP kernel (workload/csrc/synth.hip).  The ring sums over m
use numpy FFTs in both cases.  Input generation only, not part of the interpolation path.
"""
import math
import numpy as np
import torch

from .rings import ring_geometry

_SCALE_BITS = 200


def draw_alm(rng, cl, lmax):
    """Complex a_lm[l, m] (m <= l) with <|a_lm|^2> = C_l: real for m = 0."""
    a = np.zeros((lmax + 1, lmax + 1), dtype=np.complex128)
    g1 = rng.standard_normal((lmax + 1, lmax + 1))
    g2 = rng.standard_normal((lmax + 1, lmax + 1))
    return _shape_alm(np.sqrt(np.maximum(cl[: lmax + 1], 0.0)), g1, g2, a)


def _shape_alm(amp, g1, g2, out):
    lmax = out.shape[0] - 1
    l_idx, m_idx = np.tril_indices(lmax + 1)
    re = g1[l_idx, m_idx]
    im = np.where(m_idx == 0, 0.0, g2[l_idx, m_idx])
    scale = np.where(m_idx == 0, 1.0, math.sqrt(0.5))
    out[l_idx, m_idx] = amp[l_idx] * scale * (re + 1j * im)
    return out


def draw_alm_te(rng, tt, ee, te, lmax):
    """Correlated (a^T, a^E): a^T = sqrt(TT) g1, a^E = TE/sqrt(TT) g1 + sqrt(EE - TE^2/TT) g2."""
    shape = (lmax + 1, lmax + 1)
    g = [rng.standard_normal(shape) for _ in range(4)]      # re/im of g1, re/im of g2
    tt = tt[: lmax + 1]
    ee = ee[: lmax + 1]
    te = te[: lmax + 1]
    safe = np.where(tt > 0, tt, 1.0)
    c1 = np.where(tt > 0, te / np.sqrt(safe), 0.0)
    c2 = np.sqrt(np.maximum(ee - np.where(tt > 0, te * te / safe, 0.0), 0.0))
    aT = _shape_alm(np.sqrt(tt), g[0], g[1], np.zeros(shape, np.complex128))
    u1 = _shape_alm(np.ones(lmax + 1), g[0], g[1], np.zeros(shape, np.complex128))
    u2 = _shape_alm(np.ones(lmax + 1), g[2], g[3], np.zeros(shape, np.complex128))
    aE = c1[:, None] * u1 + c2[:, None] * u2
    return aT, aE


def _seed_log(m, mp, lc, ls):
    """log|d^{l0}_{m, mp}| and its sign at l0 = max(m, |mp|), for m >= 0 (vectors over m)."""
    s = abs(mp)
    m = m.to(torch.float64)
    big = m >= s
    # m >= |mp|: d^m_{m,mp} = (-1)^{m-mp} sqrt(C(2m, m+mp)) c^{m+mp} s^{m-mp}
    lb = 0.5 * (torch.lgamma(2 * m + 1) - torch.lgamma(m + mp + 1) - torch.lgamma((m - mp).clamp(min=0) + 1))
    logv_big = lb[:, None] + (m + mp)[:, None] * lc[None, :] + (m - mp)[:, None] * ls[None, :]
    sign_big = torch.where(((m - mp).round().long() % 2) == 0, 1.0, -1.0).to(torch.float64)
    if mp >= 0:
        # m < s, l0 = s: d^s_{m,s} = sqrt(C(2s, s+m)) c^{s+m} s^{s-m}
        lsm = 0.5 * (math.lgamma(2 * s + 1) - torch.lgamma(s + m + 1) - torch.lgamma((s - m).clamp(min=0) + 1))
        logv_small = lsm[:, None] + (s + m)[:, None] * lc[None, :] + (s - m)[:, None] * ls[None, :]
        sign_small = torch.ones_like(m)
    else:
        # m < s, l0 = s: d^s_{m,-s} = (-1)^{m+s} sqrt(C(2s, s-m)) c^{s-m} s^{s+m}
        lsm = 0.5 * (math.lgamma(2 * s + 1) - torch.lgamma((s - m).clamp(min=0) + 1) - torch.lgamma(s + m + 1))
        logv_small = lsm[:, None] + (s - m)[:, None] * lc[None, :] + (s + m)[:, None] * ls[None, :]
        sign_small = torch.where(((m + s).round().long() % 2) == 0, 1.0, -1.0).to(torch.float64)
    logv = torch.where(big[:, None], logv_big, logv_small)
    sign = torch.where(big, sign_big, sign_small)
    return logv, sign


def _wigner_sums(coef, s, theta, lmax, device):
    """A[m, r] = sum_l coef[l, m] (d_{m,-s} + d_{m,s})(theta_r),
    B[m, r] = sum_l coef[l, m] (d_{m,-s} - d_{m,s})(theta_r)."""
    th = torch.as_tensor(theta, dtype=torch.float64, device=device)
    R = th.numel()
    M = lmax + 1
    x = torch.cos(th)
    lc = torch.log(torch.cos(0.5 * th))
    ls = torch.log(torch.sin(0.5 * th))
    coef = torch.as_tensor(coef, device=device)
    mvec = torch.arange(M, device=device)
    mps = [0] if s == 0 else [-s, s]
    st = {}
    for mp in mps:
        logv, sign = _seed_log(mvec, mp, lc, ls)
        log2v = logv / math.log(2.0)
        E0 = torch.floor(log2v)
        mant0 = sign[:, None] * torch.exp2(log2v - E0)
        st[mp] = dict(prev=torch.zeros(M, R, dtype=torch.float64, device=device),
                      cur=torch.zeros(M, R, dtype=torch.float64, device=device),
                      E=torch.zeros(M, R, dtype=torch.float64, device=device),
                      mant0=mant0, E0=E0)
    A = torch.zeros(M, R, dtype=torch.complex128, device=device)
    B = torch.zeros(M, R, dtype=torch.complex128, device=device) if s > 0 else None
    l0 = torch.clamp(mvec, min=s)
    down = 2.0 ** (-_SCALE_BITS)
    for ell in range(0, lmax + 1):
        hi = ell + 1                                    # rows m <= ell
        mrow = mvec[:hi].to(torch.float64)[:, None]
        L = ell - 1                                     # step d^{L} -> d^{L+1} = d^{ell}
        vals = {}
        for mp in mps:
            S = st[mp]
            prev, cur, E = S["prev"][:hi], S["cur"][:hi], S["E"][:hi]
            if ell >= 1:
                a1 = (2 * L + 1) * (L * (L + 1) * x[None, :] - mrow * mp)
                c1 = (L + 1) * torch.sqrt(torch.clamp((L * L - mrow ** 2) * (L * L - mp * mp), min=0.0))
                den = L * torch.sqrt(torch.clamp(((L + 1) ** 2 - mrow ** 2) * ((L + 1) ** 2 - mp * mp), min=0.0))
                den = torch.where(den > 0, den, torch.ones_like(den))
                new = (a1 * cur - c1 * prev) / den
                if L == 0 and mp == 0:                  # d^1_{00} = cos(theta)
                    new[0] = x * cur[0]
                adv = (l0[:hi] <= L)[:, None]
                prev.copy_(torch.where(adv, cur, prev))
                cur.copy_(torch.where(adv, new, cur))
            seed_rows = (l0[:hi] == ell)
            if bool(seed_rows.any()):
                idx = torch.nonzero(seed_rows).flatten()
                cur[idx] = S["mant0"][idx]
                prev[idx] = 0.0
                E[idx] = S["E0"][idx]
            big = (cur.abs() > 2.0 ** _SCALE_BITS)
            if bool(big.any()):
                cur.copy_(torch.where(big, cur * down, cur))
                prev.copy_(torch.where(big, prev * down, prev))
                E.copy_(torch.where(big, E + _SCALE_BITS, E))
            act = (l0[:hi] <= ell)[:, None]
            vals[mp] = torch.where(act, torch.ldexp(cur, E), torch.zeros_like(cur))
        if ell < s:
            continue
        c = coef[ell, :hi][:, None]
        if s == 0:
            A[:hi] += c * (2.0 * vals[0])
        else:
            A[:hi] += c * (vals[-s] + vals[s])
            B[:hi] += c * (vals[-s] - vals[s])
    return A, B


def _rings_to_map(A, B, s, rg, lmax):
    """Sum over m on every ring with FFTs (numpy pocketfft: any ring length, no
    per-length kernel compilation); returns (re, im) numpy maps in RING order."""
    A = A.cpu().numpy() if isinstance(A, torch.Tensor) else A
    if B is not None:
        B = B.cpu().numpy() if isinstance(B, torch.Tensor) else B
    npix = int(rg["first"][-1] + rg["count"][-1])
    re = np.zeros(npix)
    im = np.zeros(npix)
    M = lmax + 1
    mvec = np.arange(M)
    cm = np.where(mvec == 0, 0.5, 1.0)
    counts = rg["count"]

    def fold(G, n):
        """G[..., m] -> sum over m = k (mod n), k = 0..n-1."""
        pad = (-G.shape[-1]) % n
        if pad:
            G = np.concatenate([G, np.zeros(G.shape[:-1] + (pad,), G.dtype)], axis=-1)
        return G.reshape(G.shape[:-1] + (-1, n)).sum(axis=-2)

    for n in np.unique(counts):
        n = int(n)
        rows = np.nonzero(counts == n)[0]
        for c0 in range(0, len(rows), 512):
            rr = rows[c0:c0 + 512]
            ph = np.exp(1j * mvec[None, :] * rg["phi0"][rr][:, None]) * cm[None, :]
            ya = np.fft.ifft(fold(A[:, rr].T * ph, n), axis=-1) * n
            yb = np.fft.ifft(fold(B[:, rr].T * ph, n), axis=-1) * n if B is not None else None
            if s % 2 == 0:
                r_part = ya.real
                i_part = yb.imag if yb is not None else 0.0 * ya.real
            else:
                r_part = yb.real
                i_part = ya.imag
            pix = (rg["first"][rr][:, None] + np.arange(n)[None, :]).ravel()
            re[pix] = r_part.ravel()
            im[pix] = i_part.ravel()
    return re, im


def synth(elm, s, nside, device="cpu"):
    """Spin-s synthesis of E-type coefficients elm[l, m] on a RING map.

    Returns a float64 tensor (npix,) for s = 0, or (re, im) tensors for s > 0.
    """
    lmax = elm.shape[0] - 1
    rg = ring_geometry(nside)
    ell = np.arange(lmax + 1, dtype=np.float64)
    norm = np.sqrt((2 * ell + 1) / (4 * np.pi)) * (-1.0) ** s
    coef = elm * norm[:, None]
    coef[:s] = 0.0
    if str(device).startswith("cuda"):
        from .gpu_synth import wigner_sums
        A, B = wigner_sums(coef, s, rg["theta"], lmax, device)
    else:
        A, B = _wigner_sums(coef, s, rg["theta"], lmax, device)
    re, im = _rings_to_map(A, B, s, rg, lmax)
    re = torch.as_tensor(re, device=device)
    im = torch.as_tensor(im, device=device)
    return re if s == 0 else (re, im)
