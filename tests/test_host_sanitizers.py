"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer.

libflints_hostsan.so is the library built with host-only -fsanitize=address and
-fsanitize=undefined (`python -m paper_1003_4984_amd.build --hostsan`; device
code unchanged).  A child Python process with the clang ASan runtime preloaded
drives every entry point's argument validation and error reporting; on a machine
without a GPU the calls that pass validation fail at their first device call,
which exercises those error paths too.  Any sanitizer report aborts the child
and fails the test.  Skipped when the sanitized library has not been built."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_1003_4984_amd import build as B  # noqa: E402

DRIVER = textwrap.dedent(r'''
    import ctypes, sys
    sys.path.insert(0, ROOT)
    import paper_1003_4984_amd.flints as F
    lib = F.load_library(LIB)
    c = ctypes
    vp, dp = c.c_void_p, c.c_void_p
    def err():
        return lib.flints_last_error().decode()
    o = F._Opts()
    lib.flints_default_opts(c.byref(o))
    assert o.precision == F.FP64 and o.stencil == F.STENCIL_NEAREST and o.map_type == F.MAP_F64
    cl = (c.c_double * 129)(*([0.0, 0.0] + [1.0 / (l * (l + 1)) for l in range(2, 129)]))
    bad_cl = (c.c_double * 129)(*([float("nan")] * 129))
    cases = [
        (lambda: lib.flints_plan(0, 128, cl, 16, 0), "nside"),
        (lambda: lib.flints_plan(64, 0, cl, 16, 0), "lmax"),
        (lambda: lib.flints_plan(64, 128, None, 16, 0), "cl"),
        (lambda: lib.flints_plan(64, 128, cl, 0, 0), "K"),
        (lambda: lib.flints_plan(64, 128, cl, 65, 0), "K"),
        (lambda: lib.flints_plan(64, 128, cl, 16, 1), "spin"),
        (lambda: lib.flints_plan(64, 128, bad_cl, 16, 0), ""),
    ]
    for fn, word in cases:
        h = fn()
        assert not h, "plan accepted"
        assert word.lower() in err().lower() and err(), (word, err())
    o2 = F._Opts(); lib.flints_default_opts(c.byref(o2)); o2.precision = 7
    assert not lib.flints_plan_ex(64, 128, cl, 16, 0, c.byref(o2)) and "precision" in err()
    o2 = F._Opts(); lib.flints_default_opts(c.byref(o2)); o2.stencil = 5
    assert not lib.flints_plan_ex(64, 128, cl, 16, 0, c.byref(o2)) and err()
    o2 = F._Opts(); lib.flints_default_opts(c.byref(o2)); o2.map_type = 9
    assert not lib.flints_plan_ex(64, 128, cl, 16, 0, c.byref(o2)) and err()
    cl2 = (c.c_double * 258)(*([0.0, 0.0] + [1.0 / (l * (l + 1)) for l in range(2, 129)]) * 2)
    o2 = F._Opts(); lib.flints_default_opts(c.byref(o2)); o2.var_kind = F.VAR_MSE
    assert not lib.flints_plan_ex(64, 128, cl2, 40, 2, c.byref(o2)) and "VAR_MSE" in err()
    # a valid plan: on a host without a GPU it fails at its first device call
    h = lib.flints_plan(64, 128, cl, 16, 0)
    if h:
        lib.flints_plan_destroy(h)
    else:
        assert err()
    lib.flints_plan_destroy(None)
    assert lib.flints_interpolate(None, None, None, None, 10, None, None, None) == F_EINVAL
    assert lib.flints_interpolate_tqu(None, None, None, None, None, None, 10, None, None, None, None, None) == F_EINVAL
    assert lib.flints_interpolate_tqu_noalloc(None, None, None, None, None, None, 10, None, None, None, None, None) == F_EINVAL
    assert lib.flints_tqu_shared(None, None, 1, 1) < 0
    assert lib.flints_stencil(None, None, None, 1, None, None) == F_EINVAL
    assert lib.flints_table_eval(None, None, 1, None, None) == F_EINVAL
    assert lib.flints_supersample(None, None, 8, None, None, None) == F_EINVAL
    assert lib.flints_pixel_centres(0, None, None, None) == F_EINVAL
    assert lib.flints_synthesize(0, 8, 0, 1, None, 1, None) == F_EINVAL and "nside" in err()
    assert lib.flints_synthesize(8, -1, 0, 1, None, 1, None) == F_EINVAL and "lmax" in err()
    assert lib.flints_synthesize(8, 8, 3, 1, None, 1, None) == F_EINVAL and "spin" in err()
    assert lib.flints_synthesize(8, 8, 0, 1, 1, 1, None) == F_EINVAL and "blm" in err()
    assert lib.flints_synthesize(8, 8, 0, None, None, 1, None) == F_EINVAL
    assert lib.flints_lensed_directions(8, None, 1, 1, None) == F_EINVAL
    assert lib.flints_lensed_directions(0, 1, 1, 1, None) == F_EINVAL
    assert not lib.flints_batch_create(None, 0, 0) and err()
    jobs = (F._Job * 2)()
    assert not lib.flints_batch_create(jobs, 2, 0) and "job 0" in err()
    assert lib.flints_batch_run(None, None) == F_EINVAL
    assert lib.flints_batch_capture(None, None) == F_EINVAL
    lib.flints_batch_destroy(None)
    assert lib.flints_plan_info(None, None) == F_EINVAL
    assert lib.flints_plan_stats(None, None, None) == F_EINVAL
    assert lib.flints_plan_reset_stats(None, None) == F_EINVAL
    print("hostsan ok")
''')


@pytest.mark.skipif(not os.path.exists(B.HOSTSAN_LIB) or B.asan_runtime() is None,
                    reason="host-sanitizer build absent (python -m paper_1003_4984_amd.build --hostsan)")
def test_entry_points_under_host_sanitizers():
    env = dict(os.environ)
    env["LD_PRELOAD"] = B.asan_runtime()
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["HIP_VISIBLE_DEVICES"] = ""       # host paths only, also on a GPU machine
    script = (f"ROOT = {ROOT!r}\nLIB = {B.HOSTSAN_LIB!r}\nF_EINVAL = -1\n" + DRIVER)
    r = subprocess.run([sys.executable, "-c", script], env=env, stdout=subprocess.PIPE,
                       stderr=subprocess.STDOUT, timeout=300)
    out = r.stdout.decode(errors="replace")
    assert r.returncode == 0 and "hostsan ok" in out, out[-4000:]
