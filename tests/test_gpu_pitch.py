"""Row pitch and start alignment of the input images.

The path reads the images through a row pitch and a base pointer of the
caller's choosing; the staging of the sub-pixel step, the padded matcher
planes and the window statistics realign every row on their own.  What
they compute depends on the pixel values only, so a pair handed over as a
column slice of wider buffers (pitch above the width, odd pitches whose
rows start at every byte offset within a dword, start pointers off a dword
boundary) must give bit-identical outputs to the same pair packed densely.
"""
import numpy as np
import pytest

from gpu_util import cu, np_
from paper_2007_12623_amd import synth

pytestmark = pytest.mark.gpu

# (extra columns past the image, start offset in bytes)
LAYOUTS = [(1, 0), (3, 1), (13, 2), (64, 3), (7, 5)]


@pytest.fixture(scope="module")
def B():
    from paper_2007_12623_amd import binding
    return binding


def _view(a, extra, off):
    import torch
    H, W = a.shape
    big = torch.zeros((H, W + extra + off), dtype=torch.uint8, device="cuda")
    big[:, off:off + W] = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    v = big[:, off:off + W]
    assert v.stride(0) == W + extra + off
    return v


def _same(a, b):
    return np.array_equal(np_(a), np_(b), equal_nan=True)


@pytest.mark.parametrize("extra,off", LAYOUTS)
def test_pipeline_independent_of_layout(B, extra, off):
    p = synth.make_pair(70, 213, 31, 21)
    L, R = p["left"], p["right"]
    params = B.preset("full", smooth_radius=4, smooth_iters=2)
    d0, m0 = B.stereo_match(cu(L), cu(R), 0, 31, 7, params)
    d1, m1 = B.stereo_match(_view(L, extra, off), _view(R, extra, off), 0, 31, 7, params)
    assert _same(m0, m1) and _same(d0, d1)


@pytest.mark.parametrize("extra,off", LAYOUTS[:3])
def test_batched_independent_of_layout(B, extra, off):
    pairs0, pairs1 = [], []
    for i, (H, W, D, win) in enumerate([(60, 180, 24, 7), (45, 251, 31, 11), (52, 199, 15, 5)]):
        p = synth.make_pair(H, W, D, 90 + i)
        L, R = p["left"], p["right"]
        pairs0.append(dict(left=cu(L), right=cu(R), dmin=0, dmax=D, win=win))
        pairs1.append(dict(left=_view(L, extra, off), right=_view(R, extra, off), dmin=0, dmax=D,
                           win=win))
    params = B.preset("small")
    out0 = B.stereo_match_batched(pairs0, params)
    out1 = B.stereo_match_batched(pairs1, params)
    for (d0, m0), (d1, m1) in zip(out0, out1):
        assert _same(m0, m1) and _same(d0, d1)


@pytest.mark.parametrize("extra,off", LAYOUTS)
@pytest.mark.parametrize("win", [5, 11, 15])
def test_subpixel_independent_of_layout(B, orc, extra, off, win):
    p = synth.make_pair(48, 300, 40, 33)
    L, R = p["left"], p["right"]
    ref = orc.match(L, R, 0, 40, win)
    o, m = cu(ref["oL"].astype(np.int16)), cu(ref["mL"])
    a = B.st_subpixel(cu(L), cu(R), 0, 40, win, o, m)
    b = B.st_subpixel(_view(L, extra, off), _view(R, extra, off), 0, 40, win, o, m)
    for x, y in zip(a, b):
        assert _same(x, y)
