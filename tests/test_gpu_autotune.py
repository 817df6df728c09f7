"""Matcher variants with 4 disparities per lane, and the autotuner of the
batched launch: every variant gives the same winners, the tuned choice is
kept per window size of the batch layout and used by the batched path,
whose output stays bit-identical to the per-pair path."""
import numpy as np
import pytest

from gpu_util import cu, np_, tie_mask
from paper_2007_12623_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_2007_12623_amd import binding
    return binding


def _batch():
    # two window sizes, uneven shapes and ranges (one signed, one of 12)
    spec = [(120, 200, 0, 31, 7), (90, 330, 0, 47, 11), (64, 96, -4, 7, 7),
            (150, 610, 5, 90, 11), (100, 260, 0, 63, 7)]
    out = []
    for i, (H, W, dmin, dmax, win) in enumerate(spec):
        p = synth.make_pair(H, W, max(dmax, 8), 900 + i)
        out.append({"left": cu(p["left"]), "right": cu(p["right"]), "dmin": dmin, "dmax": dmax,
                    "win": win})
    return out


def _chunk4_variants(B):
    return [v for v in range(B.st_num_variants()) if "DC=4" in B.st_variant_name(v)]


def test_variant_names(B):
    names = [B.st_variant_name(v) for v in range(B.st_num_variants())]
    assert all(n.startswith("TY=") and ",DC=" in n for n in names)
    assert any("DC=4" in n for n in names) and any("DC=8" in n for n in names)
    assert B.st_variant_name(B.st_num_variants()) == ""


@pytest.mark.parametrize("win", [3, 7, 11, 15])
def test_chunks_of_four_against_oracle(B, orc, win):
    """Winners of every 4-disparity variant: validity exact, disparities
    exact where the oracle's top-2 gap exceeds 1e-5 (a last chunk shifted
    to end at dmax included: 30 disparities)."""
    p = synth.make_pair(70, 300, 29, 4400 + win)
    L, R = p["left"], p["right"]
    ref = orc.match(L, R, 0, 29, win)
    h = B.Handle(0)
    try:
        for v in _chunk4_variants(B):
            B.st_set_variant(v, handle=h)
            oL, mL, oR, mR = [np_(t) for t in B.st_match_wta(cu(L), cu(R), 0, 29, win, handle=h)]
            assert np.array_equal(mL, ref["mL"]) and np.array_equal(mR, ref["mR"])
            sel = (ref["mL"] == 1) & ~tie_mask(ref["gap"])
            selr = (ref["mR"] == 1) & ~tie_mask(ref["gapR"])
            assert np.array_equal(oL[sel], ref["oL"][sel]), B.st_variant_name(v)
            assert np.array_equal(oR[selr], ref["oR"][selr]), B.st_variant_name(v)
    finally:
        h.close()


def test_forced_chunks_of_four_batched(B):
    """The batched path under each 4-disparity variant equals the default
    batched output and the per-pair path bit for bit."""
    import torch
    batch = _batch()
    params = B.preset("full", radial_r0=5, radial_dr=5, smooth_radius=4)
    h = B.Handle(0)
    try:
        ref = [(np_(d), np_(m)) for d, m in B.stereo_match_batched(batch, params, handle=h)]
        for v in _chunk4_variants(B):
            B.st_set_variant(v, handle=h)
            outs = B.stereo_match_batched(batch, params, handle=h)
            torch.cuda.synchronize()
            for q, (d, m), (dr, mr) in zip(batch, outs, ref):
                assert np.array_equal(np_(m), mr)
                assert np.array_equal(np_(d), dr, equal_nan=True)
                ds, ms = B.stereo_match(q["left"], q["right"], q["dmin"], q["dmax"], q["win"],
                                        params, handle=h)
                assert np.array_equal(np_(ms), mr)
                assert np.array_equal(np_(ds), dr, equal_nan=True)
    finally:
        h.close()


def test_autotune_batched_choice_is_used(B):
    """st_autotune_batched picks one variant per window size, the batched
    graph is rebuilt with it (st_batch_variant), and the output is the same
    bit for bit as before tuning and as the per-pair path."""
    import torch
    batch = _batch()
    params = B.preset("full", radial_r0=5, radial_dr=5, smooth_radius=4)
    h = B.Handle(0)
    try:
        before = [(np_(d), np_(m)) for d, m in B.stereo_match_batched(batch, params, handle=h)]
        assert B.st_batch_variant(7, handle=h) == 0 and B.st_batch_variant(11, handle=h) == 0
        assert B.st_batch_variant(9, handle=h) == -1
        best = B.st_autotune_batched(batch, params, reps=2, handle=h)
        assert len(best) == len(batch)
        for w in (7, 11):
            vs = {b for q, b in zip(batch, best) if q["win"] == w}
            assert len(vs) == 1
            v = vs.pop()
            assert 0 <= v < B.st_num_variants()
            assert B.st_batch_variant(w, handle=h) == v
        outs = B.stereo_match_batched(batch, params, handle=h)
        torch.cuda.synchronize()
        for w in (7, 11):   # the replay keeps the tuned graph
            v = [b for q, b in zip(batch, best) if q["win"] == w][0]
            assert B.st_batch_variant(w, handle=h) == v
        for q, (d, m), (db, mb) in zip(batch, outs, before):
            assert np.array_equal(np_(m), mb)
            assert np.array_equal(np_(d), db, equal_nan=True)
    finally:
        h.close()
