"""Address and undefined-behaviour sanitizers over the code that runs on the
CPU: the plain-C oracle built by gcc with -fsanitize=address,undefined runs
small whole pipelines (square and chessboard windows, the Eq. (4) loop, the
refinement energy); the library's host code (argument checks, handle,
tuning-table and batch-layout code) built with the same sanitizers on its
host side only runs the argument validation of every entry point without a
GPU.  Each run is a child process with the sanitizer runtime preloaded; a
report makes it exit non-zero."""
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2007_12623_amd", "csrc")

ORACLE_RUN = r"""
import sys
sys.path.insert(0, {root!r})
import numpy as np
from oracle import oracle
from paper_2007_12623_amd import synth
oracle.LIB = {lib!r}
oracle._lib = None
oracle.build = lambda force=False: {lib!r}
p = synth.make_pair(40, 72, 15, 31)
L, R = p["left"], p["right"]
for chess in (False, True):
    oracle.match(L, R, 0, 15, 7, chess=chess)
    oracle.match(L, R, 0, 15, 5, rows=(3, 30), brute=True, chess=chess)
oracle.pipeline(L, R, 0, 15, 7, oracle.params_c1())
oracle.pipeline(L, R, 0, 15, 7, oracle.params_c2(radial_r0=3, radial_dr=2, smooth_radius=4))
oracle.pipeline(L, R, 0, 15, 7, oracle.params_c2(smooth_radius=4, research=1))
oracle.pipeline(L, R, 0, 15, 7, oracle.params_c2(smooth_radius=4, chess=1))
d = np.full(L.shape, 5.25)
oracle.refine_energy(L, R, d, np.ones(L.shape, np.uint8), 7, 0.1)
print("oracle ok")
"""

LIB_RUN = r"""
import ctypes as C, sys
sys.path.insert(0, {root!r})
from paper_2007_12623_amd.binding import st_params, st_pair
L = C.CDLL({lib!r})
L.st_last_error.restype = C.c_char_p
L.st_variant_name.restype = C.c_char_p
L.st_version.restype = C.c_char_p
p = st_params()
L.st_default_params(C.byref(p))
assert L.st_version().startswith(b"stereo_mi355x")
for v in range(-1, L.st_num_variants() + 1):
    L.st_variant_name(v)
def match(fn, **kw):
    a = dict(left=1, right=1, H=100, W=100, pitch=100, dmin=0, dmax=31, win=7, d=1, m=1)
    a.update(kw)
    q = kw.get("params", p)
    return fn(None, C.c_void_p(a["left"]) if a["left"] else None, C.c_void_p(a["right"]),
              a["H"], a["W"], a["pitch"], a["dmin"], a["dmax"], a["win"], C.byref(q),
              C.c_void_p(a["d"]), C.c_void_p(a["m"]) if a["m"] else None, None)
for fn in (L.stereo_match, L.stereo_match_noalloc):
    for kw in (dict(win=4), dict(win=17), dict(dmin=5, dmax=4), dict(dmin=0, dmax=256),
               dict(dmin=-2 ** 31, dmax=2 ** 31 - 1), dict(H=5), dict(pitch=99), dict(left=0),
               dict(m=0), dict(dmax=3), dict()):
        assert match(fn, **kw) != 0
        L.st_last_error()
    bad = st_params()
    L.st_default_params(C.byref(bad))
    bad.struct_size = 12
    assert match(fn, params=bad) != 0
arr = (st_pair * 3)()
arr[0] = st_pair(1, 1, 50, 60, 60, 0, 31, 7, 1, 1)
arr[1] = st_pair(1, 1, 50, 60, 60, 0, 31, 8, 1, 1)
arr[2] = st_pair(1, 1, 50, 60, 60, 0, 3, 7, 1, 1)
for n in (0, 2, 3):
    assert L.stereo_match_batched(None, arr, n, C.byref(p), None) != 0
    L.st_last_error()
best = (C.c_int * 3)()
assert L.st_autotune_batched(None, arr, 1, C.byref(p), 3, best, None) != 0
assert L.st_batch_variant(None, 7) == -1
assert L.st_set_variant(None, 0) != 0
assert L.st_autotune(None, 100, 100, 0, 31, 6, 0, None, None) != 0
ptr = C.c_void_p()
assert L.stereo_debug_get(None, b"o_wta", C.byref(ptr)) != 0
assert L.stereo_refine_forward(None, 1, 1, 1, 1, 20, 20, 20, 8, C.c_float(0.1), None, 1, None) != 0
assert L.stereo_refine_step(None, None, 1, 1, 10, 10, C.c_float(0.1), C.c_float(0.2), None) != 0
assert L.st_fill(None, 1, 1, 10, 10, 50, 5, 20, C.c_float(0.25), 2, 3, None) != 0
h = C.c_void_p()
assert L.st_create(C.byref(h), 0) != 0
L.st_last_error()
L.st_destroy(None)
print("library ok")
"""


def _run(script, preload, extra_env=None):
    env = dict(os.environ, LD_PRELOAD=preload, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")
    env.update(extra_env or {})
    r = subprocess.run([sys.executable, "-c", script], env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    return r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is not installed")
def test_oracle_under_sanitizers(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fopenmp",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-fno-omit-frame-pointer", "-shared", "-fPIC",
                           os.path.join(ROOT, "oracle", "stereo_oracle.c"), "-o", lib, "-lm"])
    pre = ":".join(subprocess.check_output(["gcc", f"-print-file-name={n}"], text=True).strip()
                   for n in ("libasan.so", "libubsan.so"))
    assert "oracle ok" in _run(ORACLE_RUN.format(root=ROOT, lib=lib), pre)


def _clang_asan_runtime():
    base = "/opt/rocm/llvm/lib/clang"
    if not os.path.isdir(base):
        return None
    for v in sorted(os.listdir(base), reverse=True):
        so = os.path.join(base, v, "lib", "linux", "libclang_rt.asan-x86_64.so")
        if os.path.exists(so):
            return so
    return None


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc") or _clang_asan_runtime() is None,
                    reason="hipcc or its sanitizer runtime is not installed")
def test_library_host_code_under_sanitizers(tmp_path):
    from paper_2007_12623_amd import build as hb
    objs = []
    procs = []
    for src in hb.SOURCES:
        obj = str(tmp_path / src.replace(".hip", ".o"))
        cmd = [hb.hipcc(), "-O1", "-g", "-std=c++17", f"--offload-arch={hb.ARCH}", "-fPIC",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-I", CSRC, "-I", os.path.join(ROOT, "include"),
               "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
               "-Xarch_host", "-fno-omit-frame-pointer",
               "-c", os.path.join(CSRC, src), "-o", obj]
        procs.append(subprocess.Popen(cmd, stdout=subprocess.DEVNULL, stderr=subprocess.PIPE))
        objs.append(obj)
    for p in procs:
        _, err = p.communicate()
        assert p.returncode == 0, err.decode()[-3000:]
    lib = str(tmp_path / "libstereo_san.so")
    subprocess.check_call([hb.hipcc(), f"--offload-arch={hb.ARCH}", "-shared", "-fPIC",
                           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                           "-shared-libsan", *objs, "-o", lib, *hb.LIBS])
    assert "library ok" in _run(LIB_RUN.format(root=ROOT, lib=lib), _clang_asan_runtime())
