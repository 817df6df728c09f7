"""Seeded generator: determinism and the statistics the recipe fixes."""
import hashlib

import numpy as np

from paper_2007_12623_amd import synth


def _h(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def test_same_seed_same_bytes():
    a = synth.make_pair(60, 90, 31, 123)
    b = synth.make_pair(60, 90, 31, 123)
    assert _h(a["left"]) == _h(b["left"]) and _h(a["right"]) == _h(b["right"])
    c = synth.make_pair(60, 90, 31, 124)
    assert _h(a["left"]) != _h(c["left"])


def test_ranges_and_field():
    p = synth.make_pair(120, 200, 63, 7)
    L, R = p["left"], p["right"]
    assert L.dtype == np.uint8 and R.dtype == np.uint8 and L.shape == (120, 200)
    sc = synth.Scene(120, 200, 63, 7)
    assert sc.canvas.min() == 0 and sc.canvas.max() == 255  # min-max scaled canvas
    assert L.std() > 20
    g = p["gt_right"]
    ok = ~np.isnan(g)
    assert ok.mean() > 0.5
    assert g[ok].min() >= 1.0 - 1e-12 and g[ok].max() <= 61.0 + 1e-12


def test_flat_patches_low_texture():
    sc = synth.Scene(200, 300, 31, 99)
    fr = sc.frame()
    L = fr["left"].astype(np.int64)
    for py, px in sc.patches:
        patch = L[py:py + 40, px:px + 40]
        assert patch.max() - patch.min() <= 4
        assert 0.8 < patch.std() < 2.0  # uniform {-2..2} has std sqrt(2)


def test_left_ground_truth_consistent():
    p = synth.make_pair(80, 160, 31, 5)
    gl = p["gt_left"]
    ok = ~np.isnan(gl)
    assert ok.mean() > 0.7
    # x - gt_left(x) is a right column whose field maps back onto x
    y, x = np.nonzero(ok)
    xr = x - gl[y, x]
    assert (xr >= 0).all() and (xr <= 159).all()


def test_sequence_shifts_bounded():
    seq = synth.make_sequence(64, 96, 15, 11, 5)
    assert len(seq) == 5 and seq[0]["shift"] == (0, 0)
    for a, b in zip(seq, seq[1:]):
        assert abs(a["shift"][0] - b["shift"][0]) <= 4 and abs(a["shift"][1] - b["shift"][1]) <= 4
    # a pure shift of the texture: frame 1 left equals frame 0 left displaced
    (ty0, tx0), (ty1, tx1) = seq[0]["shift"], seq[1]["shift"]
    dy, dx = ty1 - ty0, tx1 - tx0
    A, B = seq[0]["left"], seq[1]["left"]
    ys = slice(max(0, -dy), min(64, 64 - dy))
    xs = slice(max(0, -dx), min(96, 96 - dx))
    yd = slice(ys.start + dy, ys.stop + dy)
    xd = slice(xs.start + dx, xs.stop + dx)
    assert np.array_equal(B[ys, xs], A[yd, xd])


def test_batch_layout():
    lay = synth.c4_layout()
    assert len(lay) == 64
    for p in lay:
        assert (p["H"], p["W"]) in synth.C4_SHAPES
        assert 32 <= p["dmax"] + 1 <= 192 and p["dmin"] == 0 and p["win"] in (7, 11)
