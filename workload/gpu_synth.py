"""GPU Legendre stage of the input synthesiser (harness only; loads
workload/libflints_synth.so built from workload/csrc/synth.hip)."""
import ctypes
import os
import subprocess

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libflints_synth.so")
_lib = None
_fn = None


def build():
    src = os.path.join(HERE, "csrc", "synth.hip")
    cmd = ["/opt/rocm/bin/hipcc", "-O3", "-fPIC", "-shared", "--offload-arch=gfx950",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wno-unused-command-line-argument", src, "-o", LIB + ".tmp"]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError(r.stdout.decode())
    os.replace(LIB + ".tmp", LIB)
    return LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        raise RuntimeError(f"{LIB} not built (workload.gpu_synth.build())")
    lib = ctypes.CDLL(LIB)
    lib.synth_wigner_sums.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                      ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.synth_wigner_sums.restype = ctypes.c_int
    _lib = lib
    return lib


def wigner_sums(coef, s, theta, lmax, device):
    """A, B complex tensors [lmax+1, R] on `device` (a CUDA device)."""
    lib = _load()
    R = len(theta)
    c = torch.as_tensor(np.ascontiguousarray(np.stack([coef.real, coef.imag], -1)),
                        dtype=torch.float64, device=device)
    th = torch.as_tensor(np.ascontiguousarray(theta), dtype=torch.float64, device=device)
    A = torch.empty((lmax + 1, R, 2), dtype=torch.float64, device=device)
    B = torch.empty((lmax + 1, R, 2), dtype=torch.float64, device=device) if s > 0 else None
    stream = torch.cuda.current_stream(device).cuda_stream
    rc = lib.synth_wigner_sums(c.data_ptr(), lmax, s, th.data_ptr(), R, A.data_ptr(),
                               B.data_ptr() if B is not None else None, stream)
    if rc != 0:
        raise RuntimeError(f"synthesis kernel launch failed: {rc}")
    A = torch.view_as_complex(A)
    B = torch.view_as_complex(B) if B is not None else None
    return A, B
