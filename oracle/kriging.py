"""Kriging (Gaussian conditional mean) interpolation: the oracle's main entry.

Test infrastructure only (see oracle/__init__.py).  Follows the paper's steps in
its order (Sec. 2.5, "The interpolation algorithm"), with the stencil rule read as
"the K nearest pixel centres" (chord distance, ties to the smaller RING index):

 1. resolution N_side and band limit lmax (given);
 2. the correlation function (oracle.correlation, exact per pair, no table);
 3. the neighbour covariance S (Eq. fundamental_variance / variance_matrix for
    spin 0, Eq. v_spins for spin s), regularised S + n I (Sec. 2.4, nugget),
    factorised S + n I = L L^T (Sec. 2.4) and solved by forward and back
    substitution (the paper inverts L; same result in exact arithmetic, see
    _solve_via_cholesky);
 4. the neighbours of each direction (K nearest, ties to the smaller index);
 5. the weighted sum, Eq. best_temperature_field (spin 0) / Eq. major_eq (spin 2);
 6. the kriging variance, Eq. gaussvar / Eq. gaussvar_pol (exponent read as 2).

Spin 2 has two modes: "full" (default) is the exact Gaussian conditional mean of
(Q, U) using both <P P*> (xi_+) and <P P> (xi_-) as a real 2K x 2K system;
"paper" keeps only the Hermitian term, i.e. the complex K x K estimator exactly as
the paper writes it.  The spin-2 covariance uses the bearing psi_ab of the great
circle a -> b, measured at a from e_theta towards e_phi:
    <P_a P_b*> = xi_+(beta_ab) exp(2i (psi_ab - psi_ba)),
    <P_a P_b>  = xi_-(beta_ab) exp(2i (psi_ab + psi_ba)),
pinned against the brute-force addition theorem (App. A) in
tests/test_oracle_spin2.py.

Nugget (Sec. 2.4): n = -lambda_min + eps with eps = 2^-26 = 1.49e-8 for double.
Policy "always" (default) adds eps on every point and escalates to
-lambda_min(S) + eps only if the Cholesky factorisation still fails; policy
"on_failure" (the paper's literal wording) adds nothing unless S itself fails.
"""
import numpy as np

from . import healpix
from .correlation import zeta, xi_pm

EPS_F64 = 2.0 ** -26          # square root of the double-precision epsilon


# --------------------------------------------------------------------------- stencil
def stencil(nside, theta, phi, K, rt=None, allvec=None):
    """Indices of the K nearest RING pixel centres to (theta, phi).

    Distance u = |n_t - n_p|^2 / 2 in FP64 from the difference vector; ties go to
    the smaller pixel index.  The search window is a proven superset of the disc of
    angular radius r, and the result is accepted only when the K-th distance is
    strictly inside that disc (else r doubles).
    """
    npix = healpix.npix(nside)
    if K > npix:
        raise ValueError("K exceeds the number of pixels")
    t = healpix.ang2vec(theta, phi)
    if rt is None:
        rt = healpix.ring_table(nside)
    r = 2.5 * np.sqrt(K / 3.0) / nside
    while True:
        if r >= np.pi or npix <= 4 * K:
            cand = np.arange(npix, dtype=np.int64)
        else:
            cand = healpix.window_pixels(nside, theta, np.mod(phi, 2 * np.pi), r, rt)
        if cand.size >= K:
            v = allvec[cand] if allvec is not None else healpix.pix2vec(nside, cand)
            u = 0.5 * np.sum((v - t) ** 2, axis=-1)
            order = np.lexsort((cand, u))[:K]
            if cand.size == npix or u[order[-1]] < 1.0 - np.cos(r):
                return cand[order], u[order]
        r *= 2.0


def pixel_stencils(nside, theta, phi, K):
    """Stencil tied to the pixel containing each direction (Sec. 2.3: the
    neighbours of a direction are those of its pixel), read as the K pixel
    centres nearest to the centre of that pixel (ties to the smaller index)."""
    pix = healpix.ang2pix(nside, theta, phi)
    thc, phc = healpix.pix2ang(nside, pix)
    return stencils(nside, thc, phc, K)


def stencils(nside, theta, phi, K):
    theta = np.atleast_1d(theta)
    phi = np.atleast_1d(phi)
    rt = healpix.ring_table(nside)
    allvec = healpix.all_vec(nside) if healpix.npix(nside) <= 3_200_000 else None
    out = np.empty((theta.size, K), dtype=np.int64)
    for p in range(theta.size):
        out[p], _ = stencil(nside, theta[p], phi[p], K, rt, allvec)
    return out


# --------------------------------------------------------------------------- geometry
def _frames(theta, phi):
    """Unit vector, e_theta, e_phi for directions (theta, phi) (vector form, so the
    frame at a pole is defined through the given phi, as Sec. 3.1 recommends)."""
    st, ct = np.sin(theta), np.cos(theta)
    sp, cp = np.sin(phi), np.cos(phi)
    n = np.stack([st * cp, st * sp, ct], axis=-1)
    et = np.stack([ct * cp, ct * sp, -st], axis=-1)
    ep = np.stack([-sp, cp, np.zeros_like(sp)], axis=-1)
    return n, et, ep


def _pixel_frames(nside, pix):
    theta, phi = healpix.pix2ang(nside, pix)
    return _frames(theta, phi)


# --------------------------------------------------------------------------- linear algebra
def _cholesky_with_nugget(S, policy, eps=EPS_F64):
    """Factor S + n I per point with the paper's nugget rule.  Returns (L, n)."""
    B, n_ = S.shape[0], S.shape[-1]
    eye = np.eye(n_)
    n0 = eps if policy == "always" else 0.0
    nug = np.full(B, n0)
    L = np.empty_like(S)
    try:
        L[:] = np.linalg.cholesky(S + n0 * eye)
        return L, nug
    except np.linalg.LinAlgError:
        pass
    for p in range(B):
        try:
            L[p] = np.linalg.cholesky(S[p] + n0 * eye)
        except np.linalg.LinAlgError:
            lam_min = np.linalg.eigvalsh(S[p])[0]
            nug[p] = max(-lam_min, 0.0) + eps
            while True:
                try:
                    L[p] = np.linalg.cholesky(S[p] + nug[p] * eye)
                    break
                except np.linalg.LinAlgError:
                    nug[p] += eps        # rounding can leave the shifted matrix singular
    return L, nug


def _forward(L, B):
    """Solve L Y = B for lower-triangular L by forward substitution (batched)."""
    Y = np.zeros(np.broadcast_shapes(B.shape, B.shape), dtype=np.result_type(L, B))
    n = L.shape[-1]
    for i in range(n):
        acc = B[:, i, :] - np.einsum("bk,bkm->bm", L[:, i, :i], Y[:, :i, :])
        Y[:, i, :] = acc / L[:, i, i][:, None]
    return Y


def _backward_h(L, Y):
    """Solve L^H X = Y (L lower-triangular) by back substitution (batched)."""
    X = np.zeros_like(Y)
    n = L.shape[-1]
    LH = np.conj(np.swapaxes(L, -1, -2))
    for i in range(n - 1, -1, -1):
        acc = Y[:, i, :] - np.einsum("bk,bkm->bm", LH[:, i, i + 1:], X[:, i + 1:, :])
        X[:, i, :] = acc / LH[:, i, i][:, None]
    return X


def _solve_via_cholesky(S, rhs, policy):
    """(S + n I)^-1 rhs with S + n I = L L^H, by forward and back substitution.

    rhs: (B, n, m).  The paper inverts L explicitly (Sec. 2.4); in exact
    arithmetic that is the same, but at the high-resolution end (N_side 4096)
    the variance 1 - b^T S^-1 b is ~1e-8 and an explicit inverse loses it to
    rounding (error ~ eps cond(S)), while substitution is backward stable.
    """
    L, nug = _cholesky_with_nugget(S, policy)
    return _backward_h(L, _forward(L, rhs)), nug


# --------------------------------------------------------------------------- spin 0
def krige_spin0(t_theta, t_phi, nvec, vals, cl, nugget="always", var_kind="paper"):
    """Spin-0 kriging for a batch of points with given stencils.

    nvec: (B, K, 3) neighbour unit vectors, vals: (B, K) map values.
    Returns value (B,), var (B,), nugget (B,).
    """
    t = healpix.ang2vec(t_theta, t_phi)                       # (B, 3)
    pts = np.concatenate([t[:, None, :], nvec], axis=1)       # (B, K+1, 3): index 0 = target
    diff = pts[:, :, None, :] - pts[:, None, :, :]
    u = 0.5 * np.sum(diff * diff, axis=-1)                    # (B, K+1, K+1)
    z, _ = zeta(u, cl)
    sigma2 = zeta(np.zeros(1), cl)[0][0]
    V = z / sigma2                                             # Eq. fundamental_variance
    S = V[:, 1:, 1:]
    b = V[:, 1:, 0]
    w, nug = _solve_via_cholesky(S, b[:, :, None], nugget)
    w = w[:, :, 0]                                             # w = (S + n I)^-1 b
    value = np.einsum("bi,bi->b", w, vals)                    # Eq. best_temperature_field
    var = sigma2 * (1.0 - np.einsum("bi,bi->b", b, w))        # Eq. gaussvar
    if var_kind == "mse":
        var = var - sigma2 * nug * np.einsum("bi,bi->b", w, w)
    return value, var, nug


# --------------------------------------------------------------------------- spin 2
def spin2_gamma_pi(n, et, ep, cl_ee, cl_bb):
    """<P_a P_b*> and <P_a P_b> for all pairs of a batch of point sets.

    n, et, ep: (B, M, 3).  Returns Gamma, Pi (B, M, M) complex and xi_+(0).
    """
    diff = n[:, :, None, :] - n[:, None, :, :]
    u = 0.5 * np.sum(diff * diff, axis=-1)
    xp, xm, xp0 = xi_pm(u, cl_ee, cl_bb)
    # bearing at a of the great circle towards b: atan2(n_b . e_phi(a), n_b . e_theta(a))
    ya = np.einsum("bjk,bik->bij", n, ep)
    xa = np.einsum("bjk,bik->bij", n, et)
    psi = np.arctan2(ya, xa)                                   # psi[a, b]
    psiT = np.swapaxes(psi, -1, -2)                            # psi[b, a]
    same = u == 0.0
    gph = np.where(same, 1.0, np.exp(2j * (psi - psiT)))
    pph = np.where(same, 1.0, np.exp(2j * (psi + psiT)))
    return xp * gph, xm * pph, xp0


def krige_spin2(t_theta, t_phi, nvec, et_n, ep_n, qvals, uvals, cl_ee, cl_bb,
                mode="full", nugget="always", var_kind="paper"):
    """Spin-2 kriging for a batch.  Returns (Q, U) (B, 2), (varQ, varU) (B, 2), nugget."""
    t, tet, tep = _frames(np.asarray(t_theta, float), np.asarray(t_phi, float))
    n = np.concatenate([t[:, None, :], nvec], axis=1)
    et = np.concatenate([tet[:, None, :], et_n], axis=1)
    ep = np.concatenate([tep[:, None, :], ep_n], axis=1)
    G, P, xp0 = spin2_gamma_pi(n, et, ep, cl_ee, cl_bb)
    B, M = G.shape[0], G.shape[1]
    K = M - 1
    if mode == "paper":
        Gn = G / xp0                                           # Eq. v_spins
        S = Gn[:, 1:, 1:]
        g = Gn[:, 0, 1:]                                       # <P_0 P_b*> / xi_+(0)
        # row vector g^T S^-1 = (S^-1 g^*)^* ^T for Hermitian S
        wc, nug = _solve_via_cholesky(S, np.conj(g)[:, :, None], nugget)
        wgt = np.conj(wc[:, :, 0])
        p = qvals + 1j * uvals
        Phat = np.einsum("bi,bi->b", wgt, p)                   # Eq. major_eq
        quad = np.einsum("bi,bi->b", wgt, np.conj(g)).real
        varP = xp0 * (1.0 - quad)                              # Eq. gaussvar_pol
        if var_kind == "mse":
            varP = varP - xp0 * nug * np.einsum("bi,bi->b", wgt, np.conj(wgt)).real
        val = np.stack([Phat.real, Phat.imag], axis=-1)
        var = np.stack([0.5 * varP, 0.5 * varP], axis=-1)
        return val, var, nug
    # full mode: real covariance of x = (Q_1..Q_K, U_1..U_K), normalised by xi_+(0)/2
    Gn, Pn = G / xp0, P / xp0
    CQQ = (Gn + Pn).real
    CUU = (Gn - Pn).real
    CQU = (Pn - Gn).imag                                       # Cov(Q_a, U_b)
    CUQ = (Pn + Gn).imag                                       # Cov(U_a, Q_b)
    C = np.empty((B, 2 * K, 2 * K))
    C[:, :K, :K] = CQQ[:, 1:, 1:]
    C[:, :K, K:] = CQU[:, 1:, 1:]
    C[:, K:, :K] = CUQ[:, 1:, 1:]
    C[:, K:, K:] = CUU[:, 1:, 1:]
    cQ = np.concatenate([CQQ[:, 1:, 0], CUQ[:, 1:, 0]], axis=1)   # Cov(x, Q_0)
    cU = np.concatenate([CQU[:, 1:, 0], CUU[:, 1:, 0]], axis=1)   # Cov(x, U_0)
    W, nug = _solve_via_cholesky(C, np.stack([cQ, cU], axis=-1), nugget)
    wQ, wU = W[:, :, 0], W[:, :, 1]
    x = np.concatenate([qvals, uvals], axis=1)
    val = np.stack([np.einsum("bi,bi->b", wQ, x), np.einsum("bi,bi->b", wU, x)], axis=-1)
    s2 = 0.5 * xp0
    vQ = s2 * (1.0 - np.einsum("bi,bi->b", cQ, wQ))
    vU = s2 * (1.0 - np.einsum("bi,bi->b", cU, wU))
    if var_kind == "mse":
        vQ = vQ - s2 * nug * np.einsum("bi,bi->b", wQ, wQ)
        vU = vU - s2 * nug * np.einsum("bi,bi->b", wU, wU)
    return val, np.stack([vQ, vU], axis=-1), nug


# --------------------------------------------------------------------------- driver
def interpolate(nside, cl, K, spin, maps, theta, phi, mode="full", nugget="always",
                var_kind="paper", stencil_idx=None, batch=256, stencil_rule="nearest"):
    """Oracle interpolation of a RING map at directions (theta, phi).

    spin 0: cl = C^TT[0..lmax], maps = T[npix];  returns value (n,), var (n,).
    spin 2: cl = (C^EE, C^BB), maps = (Q[npix], U[npix]);  returns (n, 2), (n, 2).
    A map may also be given as a function pix -> values (for maps too large to
    hold on the host; only the stencil pixels are read).
    Directions with theta outside [0, pi] or non-finite give NaN.
    stencil_rule "nearest": the K pixel centres nearest to each direction;
    "pixel": the K nearest to the centre of the pixel containing it.
    Also returns the stencils (n, K) used.
    """
    theta = np.atleast_1d(np.asarray(theta, dtype=np.float64))
    phi = np.atleast_1d(np.asarray(phi, dtype=np.float64))
    n = theta.size
    good = np.isfinite(theta) & np.isfinite(phi) & (theta >= 0.0) & (theta <= np.pi)
    if stencil_idx is None:
        stencil_idx = np.full((n, K), -1, dtype=np.int64)
        gi = np.nonzero(good)[0]
        if gi.size:
            rule = pixel_stencils if stencil_rule == "pixel" else stencils
            stencil_idx[gi] = rule(nside, theta[gi], phi[gi], K)
    shape = (n,) if spin == 0 else (n, 2)
    val = np.full(shape, np.nan)
    var = np.full(shape, np.nan)
    gi = np.nonzero(good)[0]
    for s in range(0, gi.size, batch):
        idx = gi[s:s + batch]
        st = stencil_idx[idx]
        nv, et, ep = _pixel_frames(nside, st)
        take = lambda m: m(st) if callable(m) else np.asarray(m)[st]
        if spin == 0:
            v, w, _ = krige_spin0(theta[idx], phi[idx], nv, take(maps), cl,
                                  nugget=nugget, var_kind=var_kind)
        else:
            Q, U = maps
            v, w, _ = krige_spin2(theta[idx], phi[idx], nv, et, ep, take(Q), take(U),
                                  cl[0], cl[1], mode=mode, nugget=nugget, var_kind=var_kind)
        val[idx] = v
        var[idx] = w
    return val, var, stencil_idx
