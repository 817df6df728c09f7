"""stereo_match_noalloc (every intermediate in the library's fixed per-GPU
scratch array, no device allocation) against stereo_match on the same pairs:
masks and disparities identical, bit for bit, on calls in a row whose inputs
shrink and grow again; its size and debug limits rejected on the host."""
import numpy as np
import pytest

from gpu_util import cu, np_
from paper_2007_12623_amd import synth

pytestmark = pytest.mark.gpu


def _same(B, h, L, R, dmin, dmax, win, params):
    import torch
    H, W = L.shape
    ref_d, ref_m = B.stereo_match(L, R, dmin, dmax, win, params, handle=h)
    # outputs start as garbage so that nothing left from before can pass
    d = torch.full((H, W), 123.25, dtype=torch.float32, device=L.device)
    m = torch.full((H, W), 7, dtype=torch.uint8, device=L.device)
    B.stereo_match_noalloc(L, R, dmin, dmax, win, params, d, m, handle=h)
    torch.cuda.synchronize()
    assert np.array_equal(np_(m), np_(ref_m)), "masks differ"
    assert np.array_equal(np_(d), np_(ref_d), equal_nan=True), "disparities differ"
    return int((np_(m) > 0).sum())


def test_noalloc_equals_stereo_match():
    from paper_2007_12623_amd import binding as B
    h = B.Handle(0)
    try:
        f = synth.c2_sequence(1)[0]
        L2, R2 = cu(f["left"]), cu(f["right"])
        p1 = synth.make_pair(240, 320, 31, 1001)
        L1, R1 = cu(p1["left"]), cu(p1["right"])
        pp = synth.paper_pair()
        Lp, Rp = cu(pp["left"]), cu(pp["right"])
        steps = [
            ("960x540 0..127 11x11 full", L2, R2, 0, 127, 11, B.preset("full")),
            ("320x240 0..31 7x7 small", L1, R1, 0, 31, 7, B.preset("small")),
            ("960x540 -20..80 chessboard fp16", Lp, Rp, -20, 80, 11,
             B.preset("full", chessboard=1, precision=B.ST_FP16)),
            ("320x240 0..31 7x7 full re-search", L1, R1, 0, 31, 7, B.preset("full", research=1)),
        ]
        for name, L, R, dmin, dmax, win, params in steps:
            print(name, flush=True)
            nv = _same(B, h, L, R, dmin, dmax, win, params)
            assert nv > 0.5 * L.numel()
    finally:
        h.close()


def test_noalloc_limits():
    import torch
    from paper_2007_12623_amd import binding as B
    h = B.Handle(0)
    try:
        big = torch.zeros((720, 1280), dtype=torch.uint8, device="cuda")
        d = torch.empty((720, 1280), dtype=torch.float32, device="cuda")
        m = torch.empty((720, 1280), dtype=torch.uint8, device="cuda")
        with pytest.raises(B.StereoError) as ei:
            B.stereo_match_noalloc(big, big, 0, 127, 11, B.preset("full"), d, m, handle=h)
        assert ei.value.status == B.ST_EUNSUPPORTED and "bytes of scratch" in str(ei.value)
        small = torch.zeros((240, 320), dtype=torch.uint8, device="cuda")
        with pytest.raises(B.StereoError) as ei:
            B.stereo_match_noalloc(small, small, 0, 31, 7, B.preset("small", debug_outputs=1),
                                   d[:240, :320].contiguous(), m[:240, :320].contiguous(), handle=h)
        assert ei.value.status == B.ST_EINVAL
    finally:
        h.close()
