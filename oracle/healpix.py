"""HEALPix RING geometry for the oracle (test infrastructure only).

The paper interpolates maps on the HEALPix pixelisation (Sec. 1 and Sec. 2.3 of
the paper; pixelisation defined in Gorski et al. 2005, ApJ 622, 759).  The
formulas below restate that definition:

* N_pix = 12 N_side^2 pixels on 4 N_side - 1 iso-latitude rings, ring index
  i = 1 .. 4 N_side - 1 from north to south.
* North polar cap, i < N_side: 4 i pixels, z = 1 - i^2 / (3 N_side^2),
  phi_j = (pi / (2 i)) (j + 1/2), j = 0 .. 4 i - 1.
* Equatorial belt, N_side <= i <= 3 N_side: 4 N_side pixels,
  z = 4/3 - 2 i / (3 N_side), phi_j = (pi / (2 N_side)) (j + s/2) with
  s = 1 when (i - N_side) is even and s = 0 otherwise, so the first belt ring
  (z = 2/3) starts half a pixel east of phi = 0 and the next one at phi = 0.
* South polar cap: mirror image of the north cap (z -> -z), same phi rule.
* RING order numbers pixels ring by ring from the north pole, each ring in
  increasing phi starting from the smallest phi_j >= 0.

* The pixel containing a direction (ang2pix, RING): with t = 2 phi / pi in
  [0, 4), the boundaries of the equatorial-zone pixels are the two families of
  lines N_side (1/2 + t) -/+ (3/4) N_side z = integer; those of a polar cap
  are t' r = integer and (1 - t') r = integer with t' = frac(t) and
  r = N_side sqrt(3 (1 - |z|)), r rounded up giving the ring counted from the
  pole.

Pins: tests check N_pix, ring counts, the N_side = 1 base-pixel centres
(tests/golden/healpix_nside1.txt), equal pixel areas by Monte Carlo, and
north/south mirror symmetry; ang2pix maps every pixel centre to its pixel,
gives equal counts to uniform points, returns a pixel whose centre is one of
the nearest few, and agrees with a second transcription in the tests.
"""
import numpy as np


def npix(nside):
    return 12 * nside * nside


def nrings(nside):
    return 4 * nside - 1


def ring_table(nside):
    """Per-ring arrays (index 0 holds ring i = 1).

    Returns dict with
      first  first pixel index of the ring (int64)
      count  number of pixels in the ring
      z      cos(theta) of the ring
      omz    1 - z computed without cancellation (north) / 1 + z (south) helper
      sth    sin(theta) of the ring
      phi0   phi of the first pixel
      dphi   phi spacing of the ring
    """
    N = nside
    i = np.arange(1, 4 * N, dtype=np.int64)
    count = np.empty_like(i)
    first = np.empty_like(i)
    z = np.empty(i.shape, dtype=np.float64)
    sth = np.empty(i.shape, dtype=np.float64)
    phi0 = np.empty(i.shape, dtype=np.float64)
    north = i < N
    south = i > 3 * N
    belt = ~(north | south)
    # north cap
    iN = i[north]
    count[north] = 4 * iN
    first[north] = 2 * iN * (iN - 1)
    one_minus_z = iN.astype(np.float64) ** 2 / (3.0 * N * N)
    z[north] = 1.0 - one_minus_z
    sth[north] = np.sqrt(one_minus_z * (2.0 - one_minus_z))
    phi0[north] = np.pi / (2.0 * iN) * 0.5
    # belt
    iB = i[belt]
    count[belt] = 4 * N
    first[belt] = 2 * N * (N - 1) + 4 * N * (iB - N)
    zb = 4.0 / 3.0 - 2.0 * iB / (3.0 * N)
    z[belt] = zb
    sth[belt] = np.sqrt((1.0 - zb) * (1.0 + zb))
    shift = np.where((iB - N) % 2 == 0, 0.5, 0.0)
    phi0[belt] = np.pi / (2.0 * N) * shift
    # south cap (mirror of the north cap)
    iS = 4 * N - i[south]
    count[south] = 4 * iS
    first[south] = 12 * N * N - 2 * iS * (iS + 1)
    one_plus_z = iS.astype(np.float64) ** 2 / (3.0 * N * N)
    z[south] = -(1.0 - one_plus_z)
    sth[south] = np.sqrt(one_plus_z * (2.0 - one_plus_z))
    phi0[south] = np.pi / (2.0 * iS) * 0.5
    dphi = 2.0 * np.pi / count
    return dict(first=first, count=count, z=z, sth=sth, phi0=phi0, dphi=dphi)


def pix_ring(nside, pix):
    """0-based ring index and in-ring index of RING pixels (vectorised)."""
    rt = ring_table(nside)
    pix = np.asarray(pix, dtype=np.int64)
    r = np.searchsorted(rt["first"], pix, side="right") - 1
    return r, pix - rt["first"][r]


def pix2ang(nside, pix):
    """(theta, phi) of RING pixel centres."""
    rt = ring_table(nside)
    r, j = pix_ring(nside, pix)
    theta = np.arctan2(rt["sth"][r], rt["z"][r])
    phi = rt["phi0"][r] + j * rt["dphi"][r]
    return theta, phi


def pix2vec(nside, pix):
    """Unit vectors of RING pixel centres, shape (..., 3)."""
    rt = ring_table(nside)
    r, j = pix_ring(nside, pix)
    phi = rt["phi0"][r] + j * rt["dphi"][r]
    s = rt["sth"][r]
    return np.stack([s * np.cos(phi), s * np.sin(phi), rt["z"][r]], axis=-1)


def all_vec(nside):
    return pix2vec(nside, np.arange(npix(nside), dtype=np.int64))


def ang2vec(theta, phi):
    theta = np.asarray(theta, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    st = np.sin(theta)
    return np.stack([st * np.cos(phi), st * np.sin(phi), np.cos(theta)], axis=-1)


def window_pixels(nside, theta, phi, radius, rt=None):
    """All RING pixels whose centre may lie within angular distance `radius`.

    A superset: rings whose colatitude is within `radius` of theta, and in each
    ring the pixels within the spherical-triangle bound on |dphi| plus one pixel
    of slack.  Used by the stencil search; correctness of the superset is what
    matters, not tightness.
    """
    if rt is None:
        rt = ring_table(nside)
    th_r = np.arctan2(rt["sth"], rt["z"])
    sel = np.nonzero(np.abs(th_r - theta) <= radius + 1e-12)[0]
    out = []
    st, ct = np.sin(theta), np.cos(theta)
    for r in sel:
        n = int(rt["count"][r])
        if theta - radius <= 0.0 or theta + radius >= np.pi or st == 0.0:
            out.append(rt["first"][r] + np.arange(n))
            continue
        c = (np.cos(radius) - ct * rt["z"][r]) / (st * rt["sth"][r])
        if c <= -1.0:
            out.append(rt["first"][r] + np.arange(n))
            continue
        half = np.arccos(min(c, 1.0)) + rt["dphi"][r]
        if 2 * half >= 2 * np.pi:
            out.append(rt["first"][r] + np.arange(n))
            continue
        jlo = int(np.floor((phi - half - rt["phi0"][r]) / rt["dphi"][r]))
        jhi = int(np.ceil((phi + half - rt["phi0"][r]) / rt["dphi"][r]))
        js = np.unique(np.mod(np.arange(jlo, jhi + 1), n))
        out.append(rt["first"][r] + js)
    if not out:
        return np.zeros(0, dtype=np.int64)
    return np.concatenate(out).astype(np.int64)


def ang2pix(nside, theta, phi):
    """RING index of the pixel containing each direction (theta, phi)."""
    N = int(nside)
    theta = np.atleast_1d(np.asarray(theta, dtype=np.float64))
    phi = np.atleast_1d(np.asarray(phi, dtype=np.float64))
    z = np.cos(theta)
    st = np.sin(theta)
    za = np.abs(z)
    t = np.mod(phi, 2.0 * np.pi) * (2.0 / np.pi)
    t = np.where(t >= 4.0, 0.0, t)
    out = np.empty(theta.shape, dtype=np.int64)
    eq = za <= 2.0 / 3.0
    # equatorial zone: indices of the ascending (a) and descending (d) boundary
    # lines below the point; the ring follows from their difference, the
    # position in the ring from their sum
    u = N * (0.5 + t[eq])
    v = 0.75 * N * z[eq]
    a = np.floor(u - v).astype(np.int64)
    d = np.floor(u + v).astype(np.int64)
    ring_from_top = N + 1 + a - d                  # 1 .. 2N + 1 from z = 2/3
    odd = ring_from_top % 2                        # odd rings carry the half-pixel shift
    j = (a + d - N + (1 - odd) + 1) // 2
    j = np.mod(j, 4 * N)
    out[eq] = 2 * N * (N - 1) + (ring_from_top - 1) * 4 * N + j
    # polar caps
    pc = ~eq
    one_minus = st[pc] ** 2 / (1.0 + za[pc])       # 1 - |z| without cancellation
    r = N * np.sqrt(3.0 * one_minus)
    tp = t[pc] - np.floor(t[pc])
    a = np.floor(tp * r).astype(np.int64)
    d = np.floor((1.0 - tp) * r).astype(np.int64)
    k = np.clip(a + d + 1, 1, N)                   # ring counted from the pole
    j = np.mod(np.floor(t[pc] * k).astype(np.int64), 4 * k)
    north = z[pc] > 0
    out[pc] = np.where(north, 2 * k * (k - 1) + j, 12 * N * N - 2 * k * (k + 1) + j)
    return out
