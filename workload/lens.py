"""Lensing deflection and displaced directions (paper Sec. 3.1).

The lensed direction is n' = cos|d| n + sin|d| (cos a e_theta + sin a e_phi) with
d = grad(phi) = d_theta e_theta + d_phi e_phi, written in vector form so nothing
is singular at the poles.
"""
import numpy as np
import torch

from .rings import ring_geometry


def pixel_geometry(nside, pix, device="cpu"):
    """z, sin(theta), phi of RING pixel centres (torch, float64)."""
    rg = ring_geometry(nside)
    first = torch.as_tensor(rg["first"], device=device)
    r = torch.searchsorted(first, pix, right=True) - 1
    j = (pix - first[r]).to(torch.float64)
    z = torch.as_tensor(rg["z"], device=device)[r]
    sth = torch.as_tensor(rg["sth"], device=device)[r]
    phi = torch.as_tensor(rg["phi0"], device=device)[r] + j * torch.as_tensor(rg["dphi"], device=device)[r]
    return z, sth, phi


def displace(z, sth, phi, dth, dph):
    """(theta', phi') of n' for pixels (z, sin theta, phi) and deflection components."""
    cp, sp = torch.cos(phi), torch.sin(phi)
    n = torch.stack([sth * cp, sth * sp, z], dim=-1)
    et = torch.stack([z * cp, z * sp, -sth], dim=-1)
    ep = torch.stack([-sp, cp, torch.zeros_like(sp)], dim=-1)
    dmod = torch.sqrt(dth * dth + dph * dph)
    safe = torch.where(dmod > 0, dmod, torch.ones_like(dmod))
    along = (dth[:, None] * et + dph[:, None] * ep) / safe[:, None]
    npr = torch.cos(dmod)[:, None] * n + torch.sin(dmod)[:, None] * along
    rho = torch.sqrt(npr[:, 0] ** 2 + npr[:, 1] ** 2)
    theta = torch.atan2(rho, npr[:, 2])
    ph = torch.remainder(torch.atan2(npr[:, 1], npr[:, 0]), 2 * np.pi)
    return theta, ph


def displaced_pixel_centres(nside, dth, dph, device="cpu", chunk=1 << 24):
    npix = 12 * nside * nside
    th = torch.empty(npix, dtype=torch.float64, device=device)
    ph = torch.empty(npix, dtype=torch.float64, device=device)
    for s in range(0, npix, chunk):
        e = min(npix, s + chunk)
        pix = torch.arange(s, e, device=device)
        z, sth, phi = pixel_geometry(nside, pix, device)
        th[s:e], ph[s:e] = displace(z, sth, phi, dth[s:e], dph[s:e])
    return th, ph
