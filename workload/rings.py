"""HEALPix RING ring table for the input generator (own copy of the published
Gorski et al. 2005 geometry; the generator imports nothing from the oracle)."""
import numpy as np


def ring_geometry(nside):
    N = int(nside)
    i = np.arange(1, 4 * N, dtype=np.int64)
    cap = np.minimum(i, 4 * N - i)                  # distance from the nearer pole, in rings
    polar = cap < N
    count = np.where(polar, 4 * cap, 4 * N)
    first = np.concatenate([[0], np.cumsum(count)[:-1]]).astype(np.int64)
    z = np.where(polar, 1.0 - cap.astype(np.float64) ** 2 / (3.0 * N * N),
                 4.0 / 3.0 - 2.0 * np.minimum(i, 4 * N - i) / (3.0 * N))
    z = np.where(i > 2 * N, -z, z)
    # 1 - |z| without cancellation near the poles
    omz = np.where(polar, cap.astype(np.float64) ** 2 / (3.0 * N * N), 1.0 - np.abs(z))
    sth = np.sqrt(omz * (2.0 - omz))
    half = np.where(polar, 0.5, np.where((i - N) % 2 == 0, 0.5, 0.0))
    dphi = 2.0 * np.pi / count
    phi0 = half * dphi
    theta = np.arctan2(sth, z)
    return dict(first=first, count=count, z=z, sth=sth, phi0=phi0, dphi=dphi, theta=theta)
