"""Eq. (4) re-search (Section II-C) on the GPU against the oracle: one
re-search step on identical inputs, then the whole pipeline in the
re-search mode."""
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


def _cost(L, R, y, x, c, d, win, eta, chess=False):
    h = win // 2
    a = L[y - h:y + h + 1, x - h:x + h + 1].astype(np.float64)
    b = R[y - h:y + h + 1, x - c - h:x - c + h + 1].astype(np.float64)
    if chess:  # the cells of the window's corner parity
        keep = (np.add.outer(np.arange(win), np.arange(win)) % 2) == 0
        a, b = a[keep], b[keep]
    z = np.corrcoef(a.ravel(), b.ravel())[0, 1]
    return 1.0 / max(z, 1e-3) + eta * (c - d) ** 2


# spread: d drawn over the whole range, so that a block's candidates span
# most of it (the widest R stage)
@pytest.mark.parametrize("win,rng_,eta,chess,spread", [
    (11, 5, 0.01, False, False), (7, 3, 0.05, False, False), (15, 8, 0.0, False, False),
    (11, 5, 0.01, True, False), (3, 1, 0.2, True, False), (13, 64, 0.02, False, True),
    (9, 6, 0.01, True, True)])
def test_research_step_matches_oracle(B, orc, win, rng_, eta, chess, spread):
    import torch
    p = synth.make_pair(90, 260, 47, 31 + win)
    L, R = p["left"], p["right"]
    ref = orc.match(L, R, 0, 47, win, chess=chess)
    o = ref["oL"].astype(np.int16)
    m = ref["mL"].copy()
    r = np.random.default_rng(win)
    if spread:
        d = r.uniform(-3.0, 50.0, size=L.shape)
    else:
        d = np.where(np.isnan(p["gt_left"]), o, p["gt_left"]) + r.uniform(-1.5, 1.5, size=L.shape)
    m[r.random(L.shape) < 0.05] = 0
    g = np_(B.st_research(cu(L), cu(R), 0, 47, win, cu(o), cu(m),
                          torch.tensor(d, dtype=torch.float64, device="cuda"), rng_, eta,
                          chess=chess))
    eta32 = float(np.float32(eta))  # the library takes eta as a float
    want = orc.research(L, R, 0, 47, win, o.astype(np.int32), m, d, rng_, eta32, chess=chess)
    bad = np.argwhere(g != want)
    # only exact floating-point ties may differ
    for (y, x) in bad:
        cg = _cost(L, R, y, x, int(g[y, x]), d[y, x], win, eta32, chess)
        cw = _cost(L, R, y, x, int(want[y, x]), d[y, x], win, eta32, chess)
        assert abs(cg - cw) < 1e-9, (y, x, g[y, x], want[y, x], cg, cw)
    assert len(bad) <= 3
    assert np.array_equal(g[m == 0], o[m == 0])
    assert (g != o).any()  # the step moved some pixels


@pytest.mark.parametrize("win,chess", [(15, False), (9, True)])
def test_research_step_widest_stage(B, orc, win, chess):
    """256 disparities, range 64 and d spread over the whole range: a block's
    candidates span up to 255 disparities, the widest R stage (the largest
    LDS allocation of the kernel)."""
    import torch
    p = synth.make_pair(40, 420, 255, 91)
    L, R = p["left"], p["right"]
    r = np.random.default_rng(256 + win)
    o = r.integers(0, 256, size=L.shape).astype(np.int16)
    m = (r.random(L.shape) >= 0.05).astype(np.uint8)
    d = r.uniform(-10.0, 265.0, size=L.shape)
    g = np_(B.st_research(cu(L), cu(R), 0, 255, win, cu(o), cu(m),
                          torch.tensor(d, dtype=torch.float64, device="cuda"), 64, 0.01,
                          chess=chess))
    eta32 = float(np.float32(0.01))
    want = orc.research(L, R, 0, 255, win, o.astype(np.int32), m, d, 64, eta32, chess=chess)
    bad = np.argwhere(g != want)
    for (y, x) in bad:
        cg = _cost(L, R, y, x, int(g[y, x]), d[y, x], win, eta32, chess)
        cw = _cost(L, R, y, x, int(want[y, x]), d[y, x], win, eta32, chess)
        assert abs(cg - cw) < 1e-9, (y, x, g[y, x], want[y, x], cg, cw)
    assert len(bad) <= 3
    assert np.array_equal(g[m == 0], o[m == 0])
    assert (g != o).mean() > 0.3


@pytest.mark.parametrize("H,W,far", [(11, 30, False), (11, 30, True), (13, 140, False)])
def test_research_step_degenerate(B, orc, H, W, far):
    """A frame one window high (a single row of pixels can have candidates,
    one band, one partial block) and one whose smoothed d lie far outside
    the range (no pixel has a candidate: the output is o)."""
    import torch
    r = np.random.default_rng(H * W)
    L = r.integers(0, 256, size=(H, W)).astype(np.uint8)
    R = np.roll(L, -3, axis=1)
    o = r.integers(0, 8, size=(H, W)).astype(np.int16)
    m = (r.random((H, W)) >= 0.1).astype(np.uint8)
    d = np.full((H, W), 1e4) if far else r.uniform(-1.0, 8.0, size=(H, W))
    g = np_(B.st_research(cu(L), cu(R), 0, 7, 11, cu(o), cu(m),
                          torch.tensor(d, dtype=torch.float64, device="cuda"), 5, 0.01))
    eta32 = float(np.float32(0.01))
    want = orc.research(L, R, 0, 7, 11, o.astype(np.int32), m, d, 5, eta32)
    for (y, x) in np.argwhere(g != want):
        cg = _cost(L, R, y, x, int(g[y, x]), d[y, x], 11, eta32)
        cw = _cost(L, R, y, x, int(want[y, x]), d[y, x], 11, eta32)
        assert abs(cg - cw) < 1e-9, (y, x, g[y, x], want[y, x], cg, cw)
    assert (g != want).sum() <= 1
    if far:
        assert np.array_equal(g, o)


def test_research_step_eight_row_bands(B, orc):
    """A frame large enough that the single-pair launch takes 8-row bands
    (1088 x 1024: 9 x 128 blocks; smaller launches take 4-row bands)."""
    import torch
    p = synth.make_pair(1024, 1088, 63, 1024)
    L, R = p["left"], p["right"]
    gt = p["gt_left"]
    r = np.random.default_rng(1088)
    o = np.where(np.isnan(gt), 0, np.rint(np.nan_to_num(gt))).astype(np.int16)
    m = (~np.isnan(gt) & (r.random(L.shape) >= 0.05)).astype(np.uint8)
    d = o.astype(np.float64) + r.uniform(-3.0, 3.0, size=L.shape)
    g = np_(B.st_research(cu(L), cu(R), 0, 63, 11, cu(o), cu(m),
                          torch.tensor(d, dtype=torch.float64, device="cuda"), 5, 0.01))
    eta32 = float(np.float32(0.01))
    want = orc.research(L, R, 0, 63, 11, o.astype(np.int32), m, d, 5, eta32)
    bad = np.argwhere(g != want)
    for (y, x) in bad:
        cg = _cost(L, R, y, x, int(g[y, x]), d[y, x], 11, eta32)
        cw = _cost(L, R, y, x, int(want[y, x]), d[y, x], 11, eta32)
        assert abs(cg - cw) < 1e-9, (y, x, g[y, x], want[y, x], cg, cw)
    assert len(bad) <= 3
    assert (g != o).mean() > 0.01


def test_research_step_full_frame(B, orc):
    """One re-search step on the 960x540 frame of the 30-frame workload, in
    the launch shape of the pipeline (every block of the frame): o the
    rounded ground truth, d that plus noise, 5 % of the pixels masked."""
    import torch
    fr = synth.c2_sequence(1)[0]
    L, R = fr["left"], fr["right"]
    gt = fr["gt_left"]
    r = np.random.default_rng(540)
    o = np.where(np.isnan(gt), 0, np.rint(np.nan_to_num(gt))).astype(np.int16)
    m = (~np.isnan(gt) & (r.random(L.shape) >= 0.05)).astype(np.uint8)
    d = o.astype(np.float64) + r.uniform(-2.0, 2.0, size=L.shape)
    g = np_(B.st_research(cu(L), cu(R), 0, 127, 11, cu(o), cu(m),
                          torch.tensor(d, dtype=torch.float64, device="cuda"), 5, 0.01))
    eta32 = float(np.float32(0.01))
    want = orc.research(L, R, 0, 127, 11, o.astype(np.int32), m, d, 5, eta32)
    bad = np.argwhere(g != want)
    for (y, x) in bad:
        cg = _cost(L, R, y, x, int(g[y, x]), d[y, x], 11, eta32)
        cw = _cost(L, R, y, x, int(want[y, x]), d[y, x], 11, eta32)
        assert abs(cg - cw) < 1e-9, (y, x, g[y, x], want[y, x], cg, cw)
    assert len(bad) <= 3
    assert np.array_equal(g[m == 0], o[m == 0])
    assert (g != o).mean() > 0.01


def test_research_step_pitched(B, orc):
    """Rows at an odd pitch (every row at another byte alignment), a ragged
    band and block at both ends."""
    import torch
    p = synth.make_pair(61, 203, 31, 5)
    L, R = p["left"], p["right"]
    ref = orc.match(L, R, 0, 31, 9)
    o = ref["oL"].astype(np.int16)
    m = ref["mL"].copy()
    r = np.random.default_rng(3)
    d = np.where(np.isnan(p["gt_left"]), o, p["gt_left"]) + r.uniform(-2.0, 2.0, size=L.shape)
    pitch = 211
    Lp = torch.zeros((61, pitch), dtype=torch.uint8, device="cuda")
    Rp = torch.zeros((61, pitch), dtype=torch.uint8, device="cuda")
    Lp[:, :203] = cu(L)
    Rp[:, :203] = cu(R)
    g = np_(B.st_research(Lp[:, :203], Rp[:, :203], 0, 31, 9, cu(o), cu(m),
                          torch.tensor(d, dtype=torch.float64, device="cuda"), 4, 0.03))
    eta32 = float(np.float32(0.03))
    want = orc.research(L, R, 0, 31, 9, o.astype(np.int32), m, d, 4, eta32)
    bad = np.argwhere(g != want)
    for (y, x) in bad:
        cg = _cost(L, R, y, x, int(g[y, x]), d[y, x], 9, eta32)
        cw = _cost(L, R, y, x, int(want[y, x]), d[y, x], 9, eta32)
        assert abs(cg - cw) < 1e-9, (y, x, g[y, x], want[y, x], cg, cw)
    assert len(bad) <= 3


@pytest.mark.parametrize("K,rad,shape", [(3, 15, (160, 400)), (4, 15, (160, 400)),
                                         (3, 64, (120, 260))])
def test_research_pipeline(B, orc, K, rad, shape):
    """The whole path with Eqs. (1)-(4) (radius 15, and 64, the largest the
    re-search mode takes), checked iteration by
    iteration on the GPU's own state: each smoothing step from the GPU's
    (o, d) must give the GPU's next d (FP64 on both sides), each re-search
    around that d the GPU's next o (a differing pixel only where both
    choices cost the same up to rounding), and the last step the output
    within the smoothing bar.  Before the loop, every stage is checked as
    in the plain pipeline."""
    import torch
    p = synth.make_pair(shape[0], shape[1], 63, 77)
    L, R = p["left"], p["right"]
    Hh, Ww = L.shape
    prm = B.preset("full", research=1, smooth_iters=K, smooth_radius=rad)
    po = orc.params_c2(research=1, smooth_iters=K, smooth_radius=rad)
    h = B.Handle(0)
    try:
        g = e2e.run_debug(B, L, R, 0, 63, 11, prm, handle=h)
        o_rs = [np_(B.stereo_debug_get(f"o_rs{j}", (Hh, Ww), torch.int16, handle=h)).astype(np.int32)
                for j in range(1, K)]
        d_rs = [np_(B.stereo_debug_get(f"d_rs{j}", (Hh, Ww), torch.float64, handle=h))
                for j in range(1, K)]
    finally:
        h.close()
    ref = orc.match(L, R, 0, 63, 11)
    e2e.stagewise(orc, L, R, 0, 63, 11, g, po, ref)
    m = g["m_post"]
    v = m > 0
    assert np.array_equal(g["mask"], m)
    assert np.isnan(g["disp"][~v]).all()
    alpha, eta = float(np.float32(0.1)), float(np.float32(0.01))
    o, d = g["o_post"], np.where(v, g["o_post"], 0).astype(np.float64)
    ties = 0
    for j in range(1, K + 1):
        dref, _ = orc.hc_research(L, R, 0, 63, 11, o, m, rad, 1, alpha, eta, 5, d_init=d)
        if j == K:
            err = np.abs(g["disp"][v] - dref[v])
            assert (err <= e2e.smooth_bar(dref[v])).all(), err.max()
            break
        dg = d_rs[j - 1]
        np.testing.assert_allclose(dg[v], dref[v], rtol=0, atol=1e-9)
        og = o_rs[j - 1]
        want = orc.research(L, R, 0, 63, 11, o, m, dg, 5, eta)
        assert np.array_equal(og[~v], o[~v])
        for (y, x) in np.argwhere(og != want):
            cg = _cost(L, R, y, x, int(og[y, x]), dg[y, x], 11, eta)
            cw = _cost(L, R, y, x, int(want[y, x]), dg[y, x], 11, eta)
            assert abs(cg - cw) < 1e-9, (j, y, x, og[y, x], want[y, x], cg, cw)
            ties += 1
        o, d = og, dg
    print(f"re-search pipeline K={K}: {ties} re-search decisions were cost ties")
