"""The C ABI without a GPU: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching any device."""
import ctypes as C
import os
import re

import pytest

from paper_2007_12623_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "stereo.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", text)
    keep = [n for n in names if n.startswith(("st_", "stereo_")) and n not in ("st_status",)]
    return sorted(set(keep))


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(B.LIB_PATH)
    declared = header_functions()
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(lib, name), name
    assert set(B.EXPORTS) == set(declared)


def test_default_params_are_the_papers_constants():
    p = B.st_default_params()
    assert p.struct_size == C.sizeof(B.st_params)
    assert (p.radial_iters, p.radial_r0, p.radial_dr) == (3, 10, 10)
    assert p.radial_thresh == 2.5
    assert (p.fill_radial_r, p.fill_disk_r) == (50, 20)
    assert p.smooth_radius == 15 and abs(p.smooth_alpha - 0.1) < 1e-7
    assert p.precision == B.ST_FP32
    assert B.lib().st_version().startswith(b"stereo_mi355x")
    assert B.st_num_variants() >= 4 and B.st_variant_name(0).startswith("TY=")
    assert B.st_variant_name(-1) == ""


def _match(**kw):
    args = dict(h=None, left=1, right=1, H=100, W=100, pitch=100, dmin=0, dmax=31, win=7,
                disp=1, mask=1)
    args.update(kw)
    p = kw.get("params", B.st_default_params())
    return B.lib().stereo_match(args["h"], args["left"], args["right"], args["H"], args["W"],
                                args["pitch"], args["dmin"], args["dmax"], args["win"],
                                C.byref(p) if p is not None else None, args["disp"],
                                args["mask"], None)


@pytest.mark.parametrize("kw,msg", [
    (dict(win=4), "odd"), (dict(win=17), "odd"), (dict(win=1), "odd"),
    (dict(dmin=5, dmax=4), "dmax < dmin"), (dict(dmin=0, dmax=256), "at most 256"),
    (dict(dmin=-2 ** 31, dmax=2 ** 31 - 1), "4096"), (dict(dmin=-5000, dmax=-4990), "4096"),
    (dict(H=5), "smaller"), (dict(W=6), "smaller"),
    (dict(pitch=99), "pitch"), (dict(left=None), "NULL"), (dict(mask=None), "NULL"),
    (dict(), "NULL handle"),
])
def test_stereo_match_argument_errors(kw, msg):
    assert _match(**kw) == B.ST_EINVAL
    assert msg in B.st_last_error()


@pytest.mark.parametrize("dmax", [0, 3, 6])
def test_short_ranges_are_unsupported(dmax):
    """Fewer than 8 candidates is a valid request that the library does not
    implement: ST_EUNSUPPORTED, before any device call, also in a batch."""
    assert _match(dmin=0, dmax=dmax) == B.ST_EUNSUPPORTED
    assert "fewer than 8" in B.st_last_error()
    arr = (B.st_pair * 2)()
    arr[0] = B.st_pair(1, 1, 50, 60, 60, 0, 31, 7, 1, 1)
    arr[1] = B.st_pair(1, 1, 50, 60, 60, 0, dmax, 7, 1, 1)
    p = B.st_default_params()
    assert B.lib().stereo_match_batched(None, arr, 2, C.byref(p), None) == B.ST_EUNSUPPORTED
    assert "pair 1" in B.st_last_error()


def test_params_struct_guard():
    p = B.st_default_params()
    p.struct_size = 12
    assert _match(params=p) == B.ST_EINVAL and "struct_size" in B.st_last_error()
    p = B.st_default_params(precision=7)
    assert _match(params=p) == B.ST_EINVAL and "precision" in B.st_last_error()
    p = B.st_default_params(fill_min_lines=0)
    assert _match(params=p) == B.ST_EINVAL


def test_stage_argument_errors():
    L = B.lib()
    assert L.st_radial_outlier(None, 1, 1, 10, 10, 0, 2.5, 2, None) == B.ST_EINVAL
    assert L.st_radial_outlier(None, 1, 1, 10, 10, 5, 2.5, 1, None) == B.ST_EINVAL  # aliasing
    assert L.st_fill(None, 1, 1, 10, 10, 50, 5, 20, 0.25, 2, 3, None) == B.ST_EINVAL
    assert L.st_hc_smooth(None, 1, 1, 10, 10, -1, 1, 0.1, 2, None) == B.ST_EINVAL
    assert L.stereo_refine_forward(None, 1, 1, 1, 1, 20, 20, 20, 8, 0.1, None, 1, None) == B.ST_EINVAL
    assert L.stereo_refine_forward(None, 1, 1, 1, 1, 20, 20, 20, 7, 0.1, None, None, None) == B.ST_EINVAL
    assert L.st_set_variant(None, 0) == B.ST_EINVAL
    assert L.st_autotune(None, 100, 100, 0, 31, 6, 0, None, None) == B.ST_EINVAL


def test_batched_argument_errors():
    arr = (B.st_pair * 2)()
    arr[0] = B.st_pair(1, 1, 50, 60, 60, 0, 31, 7, 1, 1)
    arr[1] = B.st_pair(1, 1, 50, 60, 60, 0, 31, 8, 1, 1)
    p = B.st_default_params()
    assert B.lib().stereo_match_batched(None, arr, 2, C.byref(p), None) == B.ST_EINVAL
    assert "pair 1" in B.st_last_error()
    assert B.lib().stereo_match_batched(None, arr, 0, C.byref(p), None) == B.ST_EINVAL


def test_create_without_device():
    from conftest import gpu_available
    if gpu_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    assert B.lib().st_create(C.byref(h), 0) == B.ST_ENODEV
    assert "device" in B.st_last_error()
