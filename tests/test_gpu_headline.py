"""The measured workload itself: the 30-frame 960x540 sequence (disparities
0..127, 11x11, full post-processing, FP32) as one batched launch replayed
from its graph, every frame against the oracle's pipeline from its images:
masks exact and disparities within the smoothing bar outside the reach of
the matcher's near-ties."""
import numpy as np
import pytest

import e2e
from gpu_util import cu, np_
from paper_2007_12623_amd import synth

pytestmark = pytest.mark.gpu

FRAMES, DMIN, DMAX, WIN = 30, 0, 127, 11


@pytest.fixture(scope="module")
def run():
    import torch
    from paper_2007_12623_amd import binding as B
    seq = synth.c2_sequence(FRAMES)
    pairs = [{"left": cu(f["left"]), "right": cu(f["right"]), "dmin": DMIN, "dmax": DMAX,
              "win": WIN} for f in seq]
    h = B.Handle(0)
    try:
        B.stereo_match_batched(pairs, B.preset("full"), handle=h)
        outs = B.stereo_match_batched(pairs, B.preset("full"), handle=h)   # a replay
        torch.cuda.synchronize()
        res = [(np_(d), np_(m)) for d, m in outs]
    finally:
        h.close()
    return seq, res


@pytest.mark.parametrize("part", range(3))
def test_headline_frames_against_oracle(orc, run, part):
    seq, res = run
    po = orc.params_c2()
    for f in range(10 * part, 10 * part + 10):
        L, R = seq[f]["left"], seq[f]["right"]
        ref = orc.match(L, R, DMIN, DMAX, WIN)
        n_cmp, n_excl = e2e.against_pipeline(orc, L, R, DMIN, DMAX, WIN, res[f][0], res[f][1],
                                             po, ref)
        print(f"frame {f}: compared {n_cmp} px, {n_excl} px within near-tie reach")
