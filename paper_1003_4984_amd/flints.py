"""ctypes binding of libflints.so (argument marshalling only).

Every step of the interpolation runs in the HIP kernels behind the C ABI; torch
tensors are used for device memory and streams.  There is no CPU fallback: if the
library is missing, every call raises.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libflints.so")

FP64, FP32_IR = 0, 1
S2_FULL, S2_PAPER = 0, 1
NUG_ALWAYS, NUG_ON_FAILURE = 0, 1
VAR_PAPER, VAR_MSE = 0, 1
STENCIL_NEAREST, STENCIL_PIXEL = 0, 1
MAP_F64, MAP_F32 = 0, 1

_lib = None


class FlintsError(RuntimeError):
    pass


class _Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("spin2_mode", ctypes.c_int),
                ("nugget", ctypes.c_int), ("var_kind", ctypes.c_int),
                ("table_tol", ctypes.c_double), ("pivot_ratio_min", ctypes.c_double),
                ("refine_tol", ctypes.c_double), ("fp32_max_reject", ctypes.c_double),
                ("stencil", ctypes.c_int), ("map_type", ctypes.c_int)]


class _Info(ctypes.Structure):
    _fields_ = [("nside", ctypes.c_int64), ("lmax", ctypes.c_int), ("K", ctypes.c_int),
                ("spin", ctypes.c_int), ("ntab", ctypes.c_int), ("table_step", ctypes.c_double),
                ("table_smax", ctypes.c_double), ("table_err", ctypes.c_double),
                ("sigma2", ctypes.c_double), ("search_r0", ctypes.c_double),
                ("search_rcap", ctypes.c_double), ("nugget_eps", ctypes.c_double),
                ("precision", ctypes.c_int), ("fp32_probe_reject", ctypes.c_double),
                ("stencil", ctypes.c_int), ("pixel_classes", ctypes.c_int64),
                ("class_nuggets", ctypes.c_int64), ("table_bytes", ctypes.c_int64),
                ("map_type", ctypes.c_int)]


class _Stats(ctypes.Structure):
    _fields_ = [("bad_inputs", ctypes.c_int64), ("nugget_escalations", ctypes.c_int64),
                ("clamped_vars", ctypes.c_int64), ("fp64_fallbacks", ctypes.c_int64),
                ("search_failures", ctypes.c_int64), ("table_range", ctypes.c_int64)]


class _Job(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("map", ctypes.c_void_p), ("theta", ctypes.c_void_p),
                ("phi", ctypes.c_void_p), ("n", ctypes.c_int64), ("out", ctypes.c_void_p),
                ("var", ctypes.c_void_p)]


class _BatchInfo(ctypes.Structure):
    _fields_ = [("njobs", ctypes.c_int), ("points", ctypes.c_int64), ("fused_jobs", ctypes.c_int),
                ("classes", ctypes.c_int), ("tiles", ctypes.c_int * 24), ("tile_points", ctypes.c_int * 24),
                ("waves_per_block", ctypes.c_int * 24), ("captured", ctypes.c_int)]


BATCH_AUTOTUNE = 1

EXPORTS = ["flints_default_opts", "flints_plan", "flints_plan_ex", "flints_interpolate",
           "flints_interpolate_tqu", "flints_interpolate_tqu_noalloc", "flints_tqu_shared",
           "flints_supersample", "flints_pixel_centres", "flints_synthesize", "flints_lensed_directions",
           "flints_stencil", "flints_table_eval", "flints_plan_info", "flints_plan_stats",
           "flints_plan_reset_stats", "flints_plan_destroy", "flints_last_error",
           "flints_batch_create", "flints_batch_run", "flints_batch_capture", "flints_batch_info",
           "flints_batch_destroy"]


def load_library(path=LIB_PATH):
    """Load libflints.so and declare its signatures (no device work)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FlintsError(f"{path} is not built; run `python -m paper_1003_4984_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i64, c_int, dp = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
    lib.flints_default_opts.argtypes = [ctypes.POINTER(_Opts)]
    lib.flints_default_opts.restype = None
    lib.flints_plan.argtypes = [i64, c_int, ctypes.POINTER(ctypes.c_double), c_int, c_int]
    lib.flints_plan.restype = vp
    lib.flints_plan_ex.argtypes = [i64, c_int, ctypes.POINTER(ctypes.c_double), c_int, c_int,
                                   ctypes.POINTER(_Opts)]
    lib.flints_plan_ex.restype = vp
    lib.flints_interpolate.argtypes = [vp, dp, dp, dp, i64, dp, dp, vp]
    lib.flints_interpolate.restype = c_int
    lib.flints_interpolate_tqu.argtypes = [vp, vp, dp, dp, dp, dp, i64, dp, dp, dp, dp, vp]
    lib.flints_interpolate_tqu.restype = c_int
    lib.flints_interpolate_tqu_noalloc.argtypes = [vp, vp, dp, dp, dp, dp, i64, dp, dp, dp, dp, vp]
    lib.flints_interpolate_tqu_noalloc.restype = c_int
    lib.flints_pixel_centres.argtypes = [i64, dp, dp, vp]
    lib.flints_pixel_centres.restype = c_int
    lib.flints_supersample.argtypes = [vp, dp, i64, dp, dp, vp]
    lib.flints_supersample.restype = c_int
    lib.flints_synthesize.argtypes = [i64, c_int, c_int, dp, dp, dp, vp]
    lib.flints_synthesize.restype = c_int
    lib.flints_lensed_directions.argtypes = [i64, dp, dp, dp, vp]
    lib.flints_lensed_directions.restype = c_int
    lib.flints_tqu_shared.argtypes = [vp, vp, c_int, c_int]
    lib.flints_tqu_shared.restype = c_int
    lib.flints_stencil.argtypes = [vp, dp, dp, i64, dp, vp]
    lib.flints_stencil.restype = c_int
    lib.flints_table_eval.argtypes = [vp, dp, i64, dp, vp]
    lib.flints_table_eval.restype = c_int
    lib.flints_plan_info.argtypes = [vp, ctypes.POINTER(_Info)]
    lib.flints_plan_info.restype = c_int
    lib.flints_plan_stats.argtypes = [vp, ctypes.POINTER(_Stats), vp]
    lib.flints_plan_stats.restype = c_int
    lib.flints_plan_reset_stats.argtypes = [vp, vp]
    lib.flints_plan_reset_stats.restype = c_int
    lib.flints_plan_destroy.argtypes = [vp]
    lib.flints_plan_destroy.restype = None
    lib.flints_last_error.argtypes = []
    lib.flints_last_error.restype = ctypes.c_char_p
    lib.flints_batch_create.argtypes = [ctypes.POINTER(_Job), c_int, c_int]
    lib.flints_batch_create.restype = vp
    lib.flints_batch_run.argtypes = [vp, vp]
    lib.flints_batch_run.restype = c_int
    lib.flints_batch_capture.argtypes = [vp, vp]
    lib.flints_batch_capture.restype = c_int
    lib.flints_batch_info.argtypes = [vp, ctypes.POINTER(_BatchInfo)]
    lib.flints_batch_info.restype = c_int
    lib.flints_batch_destroy.argtypes = [vp]
    lib.flints_batch_destroy.restype = None
    _lib = lib
    return lib


def _err(lib):
    return lib.flints_last_error().decode(errors="replace")


def _check(lib, rc, what):
    if rc != 0:
        raise FlintsError(f"{what} failed ({rc}): {_err(lib)}")


def _ptr(t, name, dtype=None):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise FlintsError(f"{name} must be a CUDA (HIP) torch tensor")
    if dtype is not None and t.dtype != dtype:
        raise FlintsError(f"{name} must have dtype {dtype}")
    if not t.is_contiguous():
        raise FlintsError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Plan:
    """A FLINTS plan: tabulated correlation function for (nside, lmax, C_l, K, spin)."""

    def __init__(self, nside, lmax, cl, K, spin, precision=FP64, spin2_mode=S2_FULL,
                 nugget=NUG_ALWAYS, var_kind=VAR_PAPER, table_tol=0.0,
                 pivot_ratio_min=0.0, refine_tol=0.0, fp32_max_reject=0.0, stencil=STENCIL_NEAREST,
                 map_type=MAP_F64):
        lib = load_library()
        cl = np.ascontiguousarray(np.asarray(cl, dtype=np.float64).ravel())
        need = (lmax + 1) * (1 if spin == 0 else 2)
        if cl.size != need:
            raise FlintsError(f"cl must hold {need} values for spin {spin}, lmax {lmax}")
        o = _Opts()
        lib.flints_default_opts(ctypes.byref(o))
        o.precision, o.spin2_mode, o.nugget, o.var_kind = precision, spin2_mode, nugget, var_kind
        o.table_tol, o.pivot_ratio_min, o.refine_tol = table_tol, pivot_ratio_min, refine_tol
        o.fp32_max_reject = fp32_max_reject
        o.stencil = stencil
        o.map_type = map_type
        h = lib.flints_plan_ex(int(nside), int(lmax), cl.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               int(K), int(spin), ctypes.byref(o))
        if not h:
            raise FlintsError(f"flints_plan failed: {_err(lib)}")
        self._lib, self._h = lib, ctypes.c_void_p(h)
        self.nside, self.lmax, self.K, self.spin = int(nside), int(lmax), int(K), int(spin)
        self.npix = 12 * self.nside * self.nside
        self.nfield = 1 if spin == 0 else 2
        self.map_type = int(map_type)

    @property
    def map_dtype(self):
        import torch
        return torch.float32 if self.map_type == MAP_F32 else torch.float64

    @property
    def handle(self):
        return self._h

    def info(self):
        i = _Info()
        _check(self._lib, self._lib.flints_plan_info(self._h, ctypes.byref(i)), "flints_plan_info")
        return {k: getattr(i, k) for k, _ in _Info._fields_}

    def stats(self, stream=None):
        """Counters, read on `stream` (default: torch's current stream)."""
        s = _Stats()
        _check(self._lib, self._lib.flints_plan_stats(self._h, ctypes.byref(s), _stream(stream)),
               "flints_plan_stats")
        return {k: getattr(s, k) for k, _ in _Stats._fields_}

    def reset_stats(self, stream=None):
        _check(self._lib, self._lib.flints_plan_reset_stats(self._h, _stream(stream)),
               "flints_plan_reset_stats")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.flints_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def interpolate(plan, map_, theta, phi, out=None, var=None, want_var=True, stream=None):
    """Interpolate `map_` (device float64, RING; spin 2: Q plane then U plane)."""
    import torch
    n = theta.numel()
    if phi.numel() != n:
        raise FlintsError("theta and phi must have the same length")
    if map_.numel() != plan.npix * plan.nfield:
        raise FlintsError(f"map must hold {plan.npix * plan.nfield} values")
    if out is None:
        out = torch.empty(plan.nfield * n, dtype=torch.float64, device=theta.device)
    if var is None and want_var:
        var = torch.empty(plan.nfield * n, dtype=torch.float64, device=theta.device)
    if out.numel() != plan.nfield * n or (var is not None and var.numel() != plan.nfield * n):
        raise FlintsError("out/var have the wrong size")
    lib = plan._lib
    rc = lib.flints_interpolate(plan.handle, _ptr(map_, "map", plan.map_dtype),
                                _ptr(theta, "theta", torch.float64), _ptr(phi, "phi", torch.float64),
                                int(n), _ptr(out, "out", torch.float64),
                                _ptr(var, "var", torch.float64), _stream(stream))
    _check(lib, rc, "flints_interpolate")
    return out, var


def interpolate_tqu(plan_t, plan_qu, map_t, map_qu, theta, phi, out_t=None, var_t=None, out_qu=None,
                    var_qu=None, want_var=True, stream=None, noalloc=False):
    """T and Q/U at the same targets with one stencil search per target
    (flints_interpolate_tqu, or with noalloc=True flints_interpolate_tqu_noalloc,
    whose stencil buffer is the library's static device workspace).  Returns
    (out_t, var_t, out_qu, var_qu)."""
    import torch
    n = theta.numel()
    if phi.numel() != n:
        raise FlintsError("theta and phi must have the same length")
    if plan_t.nfield != 1 or plan_qu.nfield != 2:
        raise FlintsError("plan_t must be spin 0 and plan_qu spin 2")
    if map_t.numel() != plan_t.npix or map_qu.numel() != 2 * plan_qu.npix:
        raise FlintsError("map_t must hold npix values and map_qu 2 npix")
    dev = theta.device
    if out_t is None:
        out_t = torch.empty(n, dtype=torch.float64, device=dev)
    if out_qu is None:
        out_qu = torch.empty(2 * n, dtype=torch.float64, device=dev)
    if want_var and var_t is None:
        var_t = torch.empty(n, dtype=torch.float64, device=dev)
    if want_var and var_qu is None:
        var_qu = torch.empty(2 * n, dtype=torch.float64, device=dev)
    if (out_t.numel() != n or out_qu.numel() != 2 * n or (var_t is not None and var_t.numel() != n)
            or (var_qu is not None and var_qu.numel() != 2 * n)):
        raise FlintsError("outputs have the wrong size")
    lib = plan_t._lib
    fn = lib.flints_interpolate_tqu_noalloc if noalloc else lib.flints_interpolate_tqu
    rc = fn(plan_t.handle, plan_qu.handle, _ptr(map_t, "map_t", plan_t.map_dtype),
            _ptr(map_qu, "map_qu", plan_qu.map_dtype), _ptr(theta, "theta", torch.float64),
            _ptr(phi, "phi", torch.float64), int(n), _ptr(out_t, "out_t", torch.float64),
            _ptr(var_t, "var_t", torch.float64), _ptr(out_qu, "out_qu", torch.float64),
            _ptr(var_qu, "var_qu", torch.float64), _stream(stream))
    _check(lib, rc, "flints_interpolate_tqu_noalloc" if noalloc else "flints_interpolate_tqu")
    return out_t, var_t, out_qu, var_qu


def supersample(plan, map_, nside_out, out=None, var=None, want_var=True, stream=None):
    """Interpolate `map_` (the plan's N_side) at every pixel centre of a RING
    map of `nside_out` (flints_supersample).  Returns (out, var), RING maps of
    nside_out (spin 2: the Q map then the U map)."""
    import torch
    if map_.numel() != plan.npix * plan.nfield:
        raise FlintsError(f"map must hold {plan.npix * plan.nfield} values")
    n = 12 * int(nside_out) * int(nside_out)
    if out is None:
        out = torch.empty(plan.nfield * n, dtype=torch.float64, device=map_.device)
    if var is None and want_var:
        var = torch.empty(plan.nfield * n, dtype=torch.float64, device=map_.device)
    if out.numel() != plan.nfield * n or (var is not None and var.numel() != plan.nfield * n):
        raise FlintsError("out/var have the wrong size")
    lib = plan._lib
    rc = lib.flints_supersample(plan.handle, _ptr(map_, "map", plan.map_dtype), int(nside_out),
                                _ptr(out, "out", torch.float64), _ptr(var, "var", torch.float64),
                                _stream(stream))
    _check(lib, rc, "flints_supersample")
    return out, var


def pixel_centres(nside, device="cuda", stream=None):
    """(theta, phi) of every RING pixel centre of `nside`, computed on the
    device by the kernel flints_supersample uses for its targets."""
    import torch
    lib = load_library()
    n = 12 * int(nside) * int(nside)
    th = torch.empty(n, dtype=torch.float64, device=device)
    ph = torch.empty(n, dtype=torch.float64, device=device)
    rc = lib.flints_pixel_centres(int(nside), _ptr(th, "theta", torch.float64), _ptr(ph, "phi", torch.float64),
                                  _stream(stream))
    _check(lib, rc, "flints_pixel_centres")
    return th, ph


def alm_mmajor(a):
    """Host complex a[l, m] (m <= l, numpy) -> float64 array of the m-major
    interleaved layout flints_synthesize takes ((l, m) at m(2 lmax+3-m)/2 + l-m)."""
    import numpy as np
    a = np.asarray(a)
    lmax = a.shape[0] - 1
    out = np.empty(((lmax + 1) * (lmax + 2) // 2, 2), dtype=np.float64)
    pos = 0
    for m in range(lmax + 1):
        col = a[m:, m]
        out[pos:pos + col.size, 0] = col.real
        out[pos:pos + col.size, 1] = col.imag
        pos += col.size
    return out.reshape(-1)


def synthesize(nside, lmax, spin, alm, blm=None, out=None, stream=None):
    """Spin-s synthesis on the device (flints_synthesize): spin 0 alm = T_lm ->
    T; spin 1 alm = phi_lm -> (d_theta, d_phi); spin 2 (alm, blm) = (E_lm, B_lm)
    -> (Q, U).  alm/blm: device float64 tensors in the m-major interleaved
    layout (alm_mmajor).  Returns the map tensor (planes of 12 nside^2)."""
    import torch
    lib = load_library()
    nalm = 2 * (int(lmax) + 1) * (int(lmax) + 2) // 2
    if alm.numel() != nalm or (blm is not None and blm.numel() != nalm):
        raise FlintsError(f"alm/blm must hold {nalm} float64 values (lmax {lmax})")
    npix = 12 * int(nside) * int(nside)
    planes = 1 if spin == 0 else 2
    if out is None:
        out = torch.empty(planes * npix, dtype=torch.float64, device=alm.device)
    if out.numel() != planes * npix:
        raise FlintsError("out has the wrong size")
    rc = lib.flints_synthesize(int(nside), int(lmax), int(spin), _ptr(alm, "alm", torch.float64),
                               _ptr(blm, "blm", torch.float64), _ptr(out, "map", torch.float64),
                               _stream(stream))
    _check(lib, rc, "flints_synthesize")
    return out


def lensed_directions(nside, defl, theta=None, phi=None, stream=None):
    """Displaced pixel centres (flints_lensed_directions) for a deflection map
    defl = (d_theta, d_phi) planes.  Returns (theta', phi')."""
    import torch
    lib = load_library()
    npix = 12 * int(nside) * int(nside)
    if defl.numel() != 2 * npix:
        raise FlintsError(f"defl must hold 2 x {npix} values")
    if theta is None:
        theta = torch.empty(npix, dtype=torch.float64, device=defl.device)
    if phi is None:
        phi = torch.empty(npix, dtype=torch.float64, device=defl.device)
    rc = lib.flints_lensed_directions(int(nside), _ptr(defl, "defl", torch.float64),
                                      _ptr(theta, "theta", torch.float64), _ptr(phi, "phi", torch.float64),
                                      _stream(stream))
    _check(lib, rc, "flints_lensed_directions")
    return theta, phi


def lens_tqu(plan_t, plan_qu, lmax, tlm, elm, blm, plm, want_var=True, stream=None):
    """The lensing pipeline of paper Sec. 3.1 on the device: unlensed T and
    (Q, U) maps and the deflection grad(phi) by synthesis, the displaced pixel
    centres, and T+Q/U interpolation there.  Plans of one N_side (spin 0 and
    spin 2); harmonic coefficients as device tensors in the m-major layout.
    Returns (out_t, var_t, out_qu, var_qu, theta', phi')."""
    nside = plan_t.nside
    if plan_qu.nside != nside:
        raise FlintsError("plans must share N_side")
    t_map = synthesize(nside, lmax, 0, tlm, stream=stream)
    qu_map = synthesize(nside, lmax, 2, elm, blm, stream=stream)
    defl = synthesize(nside, lmax, 1, plm, stream=stream)
    th, ph = lensed_directions(nside, defl, stream=stream)
    del defl
    res = interpolate_tqu(plan_t, plan_qu, t_map, qu_map, th, ph, want_var=want_var, stream=stream)
    return (*res, th, ph)


def tqu_shared(plan_t, plan_qu, with_var=True):
    """True if interpolate_tqu shares one search between the two plans."""
    rc = plan_t._lib.flints_tqu_shared(plan_t.handle, plan_qu.handle, int(with_var), int(with_var))
    _check(plan_t._lib, min(rc, 0), "flints_tqu_shared")
    return rc == 1


def stencil(plan, theta, phi, stream=None):
    import torch
    n = theta.numel()
    idx = torch.empty((n, plan.K), dtype=torch.int64, device=theta.device)
    rc = plan._lib.flints_stencil(plan.handle, _ptr(theta, "theta", torch.float64),
                                  _ptr(phi, "phi", torch.float64), int(n),
                                  _ptr(idx, "idx", torch.int64), _stream(stream))
    _check(plan._lib, rc, "flints_stencil")
    return idx


def table_eval(plan, s, stream=None):
    import torch
    n = s.numel()
    nf = plan.nfield
    out = torch.empty((n, nf), dtype=torch.float64, device=s.device)
    rc = plan._lib.flints_table_eval(plan.handle, _ptr(s, "s", torch.float64), int(n),
                                     _ptr(out, "out", torch.float64), _stream(stream))
    _check(plan._lib, rc, "flints_table_eval")
    return out


class Batch:
    """Many interpolation jobs in persistent fused launches (flints_batch_*).

    jobs: sequence of (plan, map, theta, phi, out, var) with device tensors (var
    may be None).  The tensors are borrowed: keep them alive while the batch is.
    """

    def __init__(self, jobs, autotune=False):
        import torch
        lib = load_library()
        arr = (_Job * len(jobs))()
        self._keep = []
        for i, (plan, map_, theta, phi, out, var) in enumerate(jobs):
            n = theta.numel()
            if phi.numel() != n or out.numel() != plan.nfield * n:
                raise FlintsError(f"job {i}: theta/phi/out sizes disagree")
            if map_.numel() != plan.npix * plan.nfield:
                raise FlintsError(f"job {i}: map must hold {plan.npix * plan.nfield} values")
            if var is not None and var.numel() != plan.nfield * n:
                raise FlintsError(f"job {i}: var has the wrong size")
            def addr(t, name):
                p = _ptr(t, name, torch.float64)
                return None if p is None else p.value
            arr[i].plan = plan.handle.value
            arr[i].map = _ptr(map_, "map", plan.map_dtype).value
            arr[i].theta = addr(theta, "theta")
            arr[i].phi = addr(phi, "phi")
            arr[i].n = n
            arr[i].out = addr(out, "out")
            arr[i].var = addr(var, "var")
            self._keep.append((plan, map_, theta, phi, out, var))
        h = lib.flints_batch_create(arr, len(jobs), BATCH_AUTOTUNE if autotune else 0)
        if not h:
            raise FlintsError(f"flints_batch_create failed: {_err(lib)}")
        self._lib, self._h = lib, ctypes.c_void_p(h)

    def run(self, stream=None):
        _check(self._lib, self._lib.flints_batch_run(self._h, _stream(stream)), "flints_batch_run")

    def capture(self, stream):
        _check(self._lib, self._lib.flints_batch_capture(self._h, _stream(stream)), "flints_batch_capture")

    def info(self):
        i = _BatchInfo()
        _check(self._lib, self._lib.flints_batch_info(self._h, ctypes.byref(i)), "flints_batch_info")
        d = {k: getattr(i, k) for k, _ in _BatchInfo._fields_}
        for k in ("tiles", "tile_points", "waves_per_block"):
            d[k] = list(d[k])
        return d

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.flints_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
