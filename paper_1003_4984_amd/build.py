"""Build libflints.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_1003_4984_amd.build   (or call build())
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libflints.so")
# interp_*.hip each instantiate one spin / precision class of the kernels so
# that the translation units compile in parallel.
SOURCES = ["capi.hip", "tables.hip", "interp.hip", "interp_s0.hip", "interp_s2.hip", "interp_f32_s0.hip",
           "interp_f32_s2.hip", "interp_mse64_s0.hip", "interp_mse64_s2.hip", "interp_mse32_s0.hip",
           "interp_mse32_s2.hip", "interp_tqu.hip", "supersample.hip", "fixed.hip", "batch.hip", "sht.hip"]
ARCH = os.environ.get("FLINTS_OFFLOAD_ARCH", "gfx950")

# Packed FP32 instructions are disabled: some of their forms have produced wrong
# results on this hardware, so the compiler must not emit them.
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument"]


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose=False, jobs=None):
    cc = hipcc()
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, "_obj_" + src.replace(".hip", ".o"))
        cmd = [cc, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        if p.returncode != 0:
            failed.append((src, text))
        elif verbose and text.strip():
            print(text)
    if failed:
        msg = "\n".join(f"--- {s}\n{t}" for s, t in failed)
        raise RuntimeError("hipcc failed:\n" + msg)
    tmp = LIB + ".tmp"
    cmd = [cc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout.decode(errors="replace"))
    os.replace(tmp, LIB)
    for o in objs:
        try:
            os.remove(o)
        except OSError:
            pass
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
