"""Helpers shared by the GPU parity tests (not collected by pytest)."""
import numpy as np
import torch

import paper_1003_4984_amd as fl
from oracle import healpix, kriging


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def gpu_stencil(plan, th, ph):
    idx = fl.stencil(plan, dev(th), dev(ph))
    torch.cuda.synchronize()
    return idx.cpu().numpy()


def reconcile_stencils(nside, th, ph, st_gpu, st_ora, rel=1e-9):
    """Where the two stencils differ, both must be valid K-nearest sets: same
    multiset of distances up to rounding.  Returns the number of differing rows."""
    diff = np.nonzero(np.any(np.sort(st_gpu, 1) != np.sort(st_ora, 1), axis=1))[0]
    for i in diff:
        t = healpix.ang2vec(th[i], ph[i])
        ug = np.sort(0.5 * np.sum((healpix.pix2vec(nside, st_gpu[i]) - t) ** 2, -1))
        uo = np.sort(0.5 * np.sum((healpix.pix2vec(nside, st_ora[i]) - t) ** 2, -1))
        assert np.all(st_gpu[i] >= 0), f"GPU stencil missing at row {i}"
        assert np.allclose(ug, uo, rtol=rel, atol=1e-300), (i, ug[-3:], uo[-3:])
    return len(diff)


def run_gpu(plan, maps, th, ph, want_var=True):
    m = dev(np.concatenate([np.asarray(x) for x in maps]) if isinstance(maps, (tuple, list)) else maps)
    out, var = fl.interpolate(plan, m, dev(th), dev(ph), want_var=want_var)
    torch.cuda.synchronize()
    n = len(th)
    o = out.cpu().numpy()
    v = var.cpu().numpy() if var is not None else None
    if plan.spin == 2:
        o = o.reshape(2, n).T
        v = v.reshape(2, n).T if v is not None else None
    return o, v


def compare(val_g, var_g, val_o, var_o, val_tol, var_rel, var_abs):
    """Element-wise: |value| error relative to the rms of the oracle values, and
    variance within var_rel * var + var_abs."""
    scale = np.sqrt(np.mean(val_o ** 2))
    e_val = np.max(np.abs(val_g - val_o)) / scale
    assert e_val <= val_tol, f"value error {e_val:.3e} > {val_tol:.1e}"
    if var_g is not None:
        bad = np.abs(var_g - var_o) > var_rel * np.abs(var_o) + var_abs
        assert not bad.any(), f"{bad.sum()} variances out of tolerance; worst " \
            f"{np.max(np.abs(var_g - var_o) / (np.abs(var_o) + 1e-300)):.3e}"
    return e_val
