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


# Host-side AddressSanitizer + UndefinedBehaviorSanitizer build of the same
# sources (device code is compiled as usual; every -fsanitize is host-only).
# Loaded by tests/test_host_sanitizers.py with the clang ASan runtime preloaded.
HOSTSAN_LIB = os.path.join(HERE, "libflints_hostsan.so")
HOSTSAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
                 "-Xarch_host", "-shared-libsan"]


def build(verbose=False, jobs=None, out_path=LIB, extra=(), tag=""):
    cc = hipcc()
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, "_obj_" + tag + src.replace(".hip", ".o"))
        cmd = [cc, *HIP_FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
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
    tmp = out_path + ".tmp"
    cmd = [cc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *extra, *objs, "-o", tmp]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout.decode(errors="replace"))
    os.replace(tmp, out_path)
    for o in objs:
        try:
            os.remove(o)
        except OSError:
            pass
    return out_path


def build_hostsan(verbose=False):
    """libflints_hostsan.so: the library with host-side ASan + UBSan."""
    return build(verbose, out_path=HOSTSAN_LIB, extra=HOSTSAN_FLAGS, tag="san_")


def asan_runtime():
    """The clang ASan runtime matching hipcc (to preload for the sanitized library)."""
    import glob
    root = os.path.dirname(os.path.dirname(os.path.realpath(hipcc())))
    cands = sorted(glob.glob(os.path.join(root, "llvm", "lib", "clang", "*", "lib", "linux",
                                          "libclang_rt.asan-x86_64.so")) +
                   glob.glob(os.path.join(root, "lib", "llvm", "lib", "clang", "*", "lib", "linux",
                                          "libclang_rt.asan-x86_64.so")))
    return cands[-1] if cands else None


if __name__ == "__main__":
    if "--hostsan" in sys.argv:
        print(build_hostsan(verbose="-v" in sys.argv))
    else:
        print(build(verbose="-v" in sys.argv))
