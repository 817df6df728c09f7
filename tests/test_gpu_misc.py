"""FP16/BF16 storage, the autotuner and GPU-side error paths."""
import ctypes as C
import json
import os

import numpy as np
import pytest

from gpu_util import cu, np_
from paper_2007_12623_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_2007_12623_amd import binding
    return binding


@pytest.mark.parametrize("prec,quantum", [(1, 2.0 ** -10), (2, 2.0 ** -7)], ids=["fp16", "bf16"])
def test_half_precision_storage(B, orc, prec, quantum):
    """FP16/BF16 images (lossless for 0..255), fp32 accumulation, FP64
    normalisation, z held at the storage precision: disparities equal the
    oracle wherever its top-2 gap exceeds two storage quanta."""
    p = synth.make_pair(200, 480, 63, 91)
    L, R = p["left"], p["right"]
    oL, mL, oR, mR = (np_(t) for t in B.st_match_wta(cu(L), cu(R), 0, 63, 11, precision=prec))
    ref = orc.match(L, R, 0, 63, 11)
    assert np.array_equal(mL, ref["mL"])
    sel = (ref["mL"] == 1) & (np.nan_to_num(ref["gap"], nan=np.inf) > quantum)
    assert np.array_equal(oL[sel], ref["oL"][sel])
    dis = (oL != ref["oL"]) & (ref["mL"] == 1)
    assert dis.mean() < 0.02


def test_integer_shift_exact_in_half_precision(B):
    r = np.random.default_rng(8)
    Hh, Ww, k = 40, 200, 5
    wide = r.integers(0, 256, size=(Hh, Ww + k), dtype=np.uint8)
    L, R = wide[:, :Ww].copy(), wide[:, k:].copy()
    for prec in (1, 2):
        oL, mL, oR, mR = (np_(t) for t in B.st_match_wta(cu(L), cu(R), 0, 15, 7, precision=prec))
        assert (oL[3:Hh - 3, 3 + k:Ww - 3] == k).all()


def test_autotune_and_cache(B, tmp_path):
    path = tmp_path / "tune.json"
    os.environ["STEREO_TUNE_CACHE"] = str(path)
    try:
        h = B.Handle(0)
        best = B.st_autotune(300, 500, 0, 63, 11, handle=h)
        assert 0 <= best < B.st_num_variants()
        h.close()
        table = json.loads(path.read_text())
        assert list(table.values()) == [best]
        h2 = B.Handle(0)   # the cache is read back
        p = synth.make_pair(300, 500, 63, 4)
        B.st_match_wta(cu(p["left"]), cu(p["right"]), 0, 63, 11, handle=h2)
        h2.close()
    finally:
        del os.environ["STEREO_TUNE_CACHE"]


def test_injected_allocation_failure(B):
    os.environ["STEREO_FAULT"] = "alloc"
    try:
        h = B.Handle(0)
        p = synth.make_pair(60, 80, 15, 1)
        with pytest.raises(B.StereoError) as ei:
            B.stereo_match(cu(p["left"]), cu(p["right"]), 0, 15, 7, handle=h)
        assert ei.value.status == B.ST_ENOMEM
        assert "injected" in B.st_last_error()
        h.close()
    finally:
        del os.environ["STEREO_FAULT"]


def test_debug_get_errors(B):
    h = B.Handle(0)
    try:
        ptr = C.c_void_p()
        assert B.lib().stereo_debug_get(h.h, b"o_wta", C.byref(ptr)) == B.ST_EINVAL
    finally:
        h.close()


def test_create_bad_device(B):
    h = C.c_void_p()
    assert B.lib().st_create(C.byref(h), 99) == B.ST_ENODEV


def test_reproject_matches_oracle(B, orc):
    r = np.random.default_rng(12)
    H, Ww = 70, 130
    d = r.uniform(-5.0, 90.0, size=(H, Ww)).astype(np.float32)
    d[r.random((H, Ww)) < 0.1] = np.nan
    d[0, :4] = 0.0
    Q = r.normal(size=(4, 4))
    Q[3, 2] = 0.2
    g = np_(B.st_reproject(cu(d), Q))
    ref = orc.reproject(d.astype(np.float64), Q)
    assert np.array_equal(np.isnan(g), np.isnan(ref))
    fin = ~np.isnan(ref)
    np.testing.assert_allclose(g[fin], ref[fin].astype(np.float32), rtol=1e-6, atol=1e-6)
