"""Batched persistent launch: equal to the per-pair path bit for bit, stable
across graph replays, and independent of the matcher's tile variant; every
pair of the 64-pair uneven batch checked against the oracle stage by stage."""
import numpy as np
import pytest

import e2e
from gpu_util import cu, np_
from paper_2007_12623_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_2007_12623_amd import binding
    return binding


def _mini_batch():
    # uneven shapes, ranges (one with D < 16) and windows
    spec = [(120, 200, 0, 31, 7), (90, 330, 0, 47, 11), (64, 96, -4, 11, 5),
            (150, 610, 5, 90, 9), (75, 128, 0, 7, 3), (100, 260, 0, 63, 13)]
    out = []
    for i, (H, W, dmin, dmax, win) in enumerate(spec):
        p = synth.make_pair(H, W, max(dmax, 8), 500 + i)
        out.append({"left": cu(p["left"]), "right": cu(p["right"]), "dmin": dmin, "dmax": dmax,
                    "win": win})
    return out


def test_batched_equals_single(B):
    import torch
    batch = _mini_batch()
    params = B.preset("full", radial_r0=5, radial_dr=5, smooth_radius=4)
    h = B.Handle(0)
    try:
        outs = B.stereo_match_batched(batch, params, handle=h)
        torch.cuda.synchronize()
        for q, (d, m) in zip(batch, outs):
            ds, ms = B.stereo_match(q["left"], q["right"], q["dmin"], q["dmax"], q["win"], params,
                                    handle=h)
            assert np.array_equal(np_(m), np_(ms))
            assert np.array_equal(np_(d), np_(ds), equal_nan=True)
    finally:
        h.close()


def test_graph_replay_reads_live_inputs(B):
    import torch
    batch = _mini_batch()[:3]
    params = B.preset("small")
    h = B.Handle(0)
    try:
        first = [(np_(d), np_(m)) for d, m in B.stereo_match_batched(batch, params, handle=h)]
        for _ in range(3):
            again = B.stereo_match_batched(batch, params, handle=h)   # graph replay
            torch.cuda.synchronize()
            for (d0, m0), (d1, m1) in zip(first, again):
                assert np.array_equal(m0, np_(m1))
                assert np.array_equal(d0, np_(d1), equal_nan=True)
        # same pointers, new image contents: the replay must see them
        batch[0]["right"].copy_(torch.roll(batch[0]["right"], 1, dims=1))
        d1, m1 = B.stereo_match_batched(batch, params, handle=h)[0]
        ds, ms = B.stereo_match(batch[0]["left"], batch[0]["right"], batch[0]["dmin"],
                                batch[0]["dmax"], batch[0]["win"], params, handle=h)
        assert np.array_equal(np_(m1), np_(ms))
        assert np.array_equal(np_(d1), np_(ds), equal_nan=True)
    finally:
        h.close()


def test_matcher_variants_bit_identical(B):
    p = synth.make_pair(130, 700, 95, 77)
    L, R = cu(p["left"]), cu(p["right"])
    h = B.Handle(0)
    try:
        ref = None
        for v in range(B.st_num_variants()):
            B.st_set_variant(v, handle=h)
            got = [np_(t) for t in B.st_match_wta(L, R, 0, 95, 11, handle=h)]
            if ref is None:
                ref = got
            for a, b in zip(ref, got):
                assert np.array_equal(a, b), B.st_variant_name(v)
    finally:
        h.close()


@pytest.fixture(scope="module")
def c4(B):
    """The 64-pair batch of four shapes, 32..192 candidates, 7x7 and 11x11,
    run once through the batched launch."""
    import torch
    batch = synth.c4_batch()
    pairs = [{"left": cu(q["left"]), "right": cu(q["right"]), "dmin": q["dmin"], "dmax": q["dmax"],
              "win": q["win"]} for q in batch]
    h = B.Handle(0)
    try:
        outs = B.stereo_match_batched(pairs, B.preset("full"), handle=h)
        torch.cuda.synchronize()
        res = [(np_(d), np_(m)) for d, m in outs]
        single = []
        for q in pairs:
            ds, ms = B.stereo_match(q["left"], q["right"], q["dmin"], q["dmax"], q["win"],
                                    B.preset("full"), handle=h)
            single.append((np_(ds), np_(ms)))
    finally:
        h.close()
    return batch, res, single


def test_uneven_batch_of_64_equals_single(c4):
    """Every pair of the batch equals the per-pair path bit for bit."""
    batch, res, single = c4
    for i, ((d, m), (ds, ms)) in enumerate(zip(res, single)):
        assert np.array_equal(m, ms), i
        assert np.array_equal(d, ds, equal_nan=True), i


@pytest.mark.parametrize("part", range(4))
def test_uneven_batch_of_64_against_oracle(B, orc, c4, part):
    """Every pair of the batch against the oracle (16 pairs per part): the
    pair's debug run through the per-pair path gives the batched output bit
    for bit, and every stage of it equals the oracle's stage run on the same
    input (matching exact away from near-ties, later stages exact or within
    the smoothing bar)."""
    batch, res, _ = c4
    po = orc.params_c2()
    h = B.Handle(0)
    try:
        for i in range(16 * part, 16 * part + 16):
            q = batch[i]
            L, R, dmin, dmax, win = q["left"], q["right"], q["dmin"], q["dmax"], q["win"]
            g = e2e.run_debug(B, L, R, dmin, dmax, win, B.preset("full"), handle=h)
            assert np.array_equal(g["mask"], res[i][1]), i
            assert np.array_equal(g["disp"], res[i][0], equal_nan=True), i
            ref = orc.match(L, R, dmin, dmax, win)
            rep = e2e.stagewise(orc, L, R, dmin, dmax, win, g, po, ref)
            print(f"pair {i} {q['W']}x{q['H']} D={dmax - dmin + 1} win={win}: stage-wise exact; "
                  f"{rep['int_disagree_px']} near-tie winners differ", flush=True)
    finally:
        h.close()


def test_rebuild_on_a_side_stream_without_host_sync(B):
    """Two batch layouts in a row on one non-default stream, no host
    synchronisation between them: the second call replaces the graph and
    the device tables that the first call's replay reads, so it must order
    itself after that replay.  Both outputs equal the per-pair path."""
    import torch
    a = _mini_batch()
    b = _mini_batch()[1:4]
    params = B.preset("full", radial_r0=5, radial_dr=5, smooth_radius=4)
    h = B.Handle(0)
    s = torch.cuda.Stream()
    try:
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            oa = B.stereo_match_batched(a, params, handle=h)
            oa2 = B.stereo_match_batched(a, params, handle=h)   # graph replay
            ob = B.stereo_match_batched(b, params, handle=h)    # rebuild
        s.synchronize()
        for batch, outs in ((a, oa2), (b, ob)):
            for q, (d, m) in zip(batch, outs):
                ds, ms = B.stereo_match(q["left"], q["right"], q["dmin"], q["dmax"], q["win"],
                                        params, handle=h)
                torch.cuda.synchronize()
                assert np.array_equal(np_(m), np_(ms))
                assert np.array_equal(np_(d), np_(ds), equal_nan=True)
    finally:
        h.close()
