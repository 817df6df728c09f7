"""HIP path against the CPU oracle, stage by stage and end to end.

Bars: integer disparities and masks bit-exact wherever the oracle's top-2
ZNCC gap exceeds 1e-5 (the matcher quantises z + 2 to 2^-18 before its
argmax); ZNCC values and sub-pixel offsets within 1e-5; smoothed
disparities within max(1e-5, 1 ulp).  Sizes span several tiles, ragged
edges, signed disparity ranges and every window size.
"""
import numpy as np
import pytest

import e2e
from gpu_util import cu, np_, tie_mask
from paper_2007_12623_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_2007_12623_amd import binding
    return binding


def _pair(H, W, D, seed):
    p = synth.make_pair(H, W, D, seed)
    return p["left"], p["right"]


CASES = [
    # (H, W, dmin, dmax, win, seed)
    (240, 320, 0, 31, 7, 1001),     # the 320x240 workload
    (37, 150, -5, 27, 5, 11),       # ragged, negative disparities
    (61, 530, 3, 70, 3, 12),        # two spans, 68 candidates
    (45, 200, 0, 15, 9, 13),        # D = 16
    (50, 190, -12, -5, 11, 14),     # D = 8, all negative
    (40, 260, 0, 40, 13, 15),
    (48, 300, 10, 60, 15, 16),
    (30, 600, 0, 255, 7, 17),       # D = 256, the largest range
    (30, 560, -3, 246, 5, 18),      # D = 250: last chunk shifted to d0 - dmin = 242
    (7, 200, 0, 31, 7, 19),         # H = win: a single row of windows
    (40, 60, 0, 127, 5, 20),        # W <= dmax: chunks with no valid candidate
    (15, 100, -60, 140, 15, 22),    # both, with a signed range wider than the image
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}_d{c[2]}..{c[3]}_w{c[4]}" for c in CASES])
def test_window_stats(B, orc, case):
    H, W, dmin, dmax, win, seed = case
    L, _ = _pair(H, W, max(dmax, 8), seed)
    S, SS, inv = B.st_window_stats(cu(L), win)
    rS, rSS, rV, ins = orc.window_stats(L, win)
    assert np.array_equal(np_(S), rS.astype(np.int32))
    assert np.array_equal(np_(SS), rSS.astype(np.int32))
    g = np_(inv)
    ok = (ins == 1) & (rV > 0)
    ref = (1.0 / np.sqrt(rV[ok].astype(np.float64))).astype(np.float32)
    assert np.all(np.isnan(g[~ok]))
    np.testing.assert_array_max_ulp(g[ok], ref, maxulp=1)


def _check_wta(out, ref, oL, mL, oR, mR):
    assert np.array_equal(mL, ref["mL"]), "left validity"
    assert np.array_equal(mR, ref["mR"]), "right validity"
    sel = (ref["mL"] == 1) & ~tie_mask(ref["gap"])
    bad = np.nonzero(oL[sel] != ref["oL"][sel])[0]
    assert bad.size == 0, f"{bad.size} left disparities differ"
    selr = (ref["mR"] == 1) & ~tie_mask(ref["gapR"])
    badr = np.nonzero(oR[selr] != ref["oR"][selr])[0]
    assert badr.size == 0, f"{badr.size} right disparities differ"


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}_d{c[2]}..{c[3]}_w{c[4]}" for c in CASES])
def test_match_wta(B, orc, case):
    H, W, dmin, dmax, win, seed = case
    L, R = _pair(H, W, max(dmax, 8), seed)
    oL, mL, oR, mR = (np_(t) for t in B.st_match_wta(cu(L), cu(R), dmin, dmax, win))
    ref = orc.match(L, R, dmin, dmax, win)
    _check_wta(None, ref, oL, mL, oR, mR)


def test_match_wta_every_variant(B, orc):
    H, W, dmin, dmax, win, seed = 70, 420, 0, 47, 7, 21
    L, R = _pair(H, W, dmax, seed)
    ref = orc.match(L, R, dmin, dmax, win)
    h = B.Handle(0)
    try:
        for v in range(B.st_num_variants()):
            B.st_set_variant(v, handle=h)
            oL, mL, oR, mR = (np_(t) for t in B.st_match_wta(cu(L), cu(R), dmin, dmax, win, handle=h))
            _check_wta(None, ref, oL, mL, oR, mR)
    finally:
        h.close()


def test_match_wta_integer_shift_exact(B):
    r = np.random.default_rng(3)
    H, W, k = 64, 300, 9
    wide = r.integers(0, 256, size=(H, W + k), dtype=np.uint8)
    L, R = wide[:, :W].copy(), wide[:, k:].copy()
    oL, mL, oR, mR = (np_(t) for t in B.st_match_wta(cu(L), cu(R), 0, 23, 7))
    h = 3
    assert (oL[h:H - h, h + k:W - h] == k).all()
    assert (oR[h:H - h, h:W - h - k] == k).all()


def test_match_full_size_frame(B, orc):
    """960x540, 128 candidates, 11x11: the whole frame against the oracle."""
    seq = synth.c2_sequence(1)
    L, R = seq[0]["left"], seq[0]["right"]
    oL, mL, oR, mR = (np_(t) for t in B.st_match_wta(cu(L), cu(R), 0, 127, 11))
    ref = orc.match(L, R, 0, 127, 11)
    _check_wta(None, ref, oL, mL, oR, mR)


def test_match_paper_range_frame(B, orc):
    """The paper's candidate range -20..80 (101 values) at 960x540, 11x11."""
    p = synth.paper_pair()
    L, R = p["left"], p["right"]
    oL, mL, oR, mR = (np_(t) for t in B.st_match_wta(cu(L), cu(R), -20, 80, 11))
    ref = orc.match(L, R, -20, 80, 11)
    _check_wta(None, ref, oL, mL, oR, mR)


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}_d{c[2]}..{c[3]}_w{c[4]}" for c in CASES])
def test_subpixel_every_window(B, orc, case):
    """Exact z at o-1, o, o+1 for every window size, ragged shapes (rows not
    a multiple of the 4-row blocks, columns not of 128) and signed ranges."""
    H, W, dmin, dmax, win, seed = case
    L, R = _pair(H, W, max(dmax, 8), seed)
    ref = orc.match(L, R, dmin, dmax, win)
    zb, zm, zp, dl = (np_(t) for t in B.st_subpixel(cu(L), cu(R), dmin, dmax, win,
                                                       cu(ref["oL"].astype(np.int16)), cu(ref["mL"])))
    v = ref["mL"] == 1
    np.testing.assert_allclose(zb[v], ref["zbest"][v], atol=1e-12)
    for key, g in (("zm", zm), ("zp", zp)):
        assert np.array_equal(np.isnan(g[v]), np.isnan(ref[key][v])), key
        f = v & ~np.isnan(ref[key])
        np.testing.assert_allclose(g[f], ref[key][f], atol=1e-12)
    rd = orc.subpixel(ref["oL"], ref["mL"], ref["zm"], ref["zbest"], ref["zp"], dmin, dmax)
    assert np.abs(dl[v] - rd[v]).max() <= 1e-5
    assert (dl[~v] == 0).all() and np.isnan(zb[~v]).all()


def test_subpixel_exact_z(B, orc):
    L, R = _pair(60, 250, 31, 31)
    ref = orc.match(L, R, 0, 31, 7)
    zb, zm, zp, dl = (np_(t) for t in B.st_subpixel(cu(L), cu(R), 0, 31, 7,
                                                       cu(ref["oL"].astype(np.int16)), cu(ref["mL"])))
    v = ref["mL"] == 1
    np.testing.assert_allclose(zb[v], ref["zbest"][v], atol=1e-12)
    np.testing.assert_allclose(zm[v], ref["zm"][v], atol=1e-12)
    np.testing.assert_allclose(zp[v], ref["zp"][v], atol=1e-12)
    rd = orc.subpixel(ref["oL"], ref["mL"], ref["zm"], ref["zbest"], ref["zp"], 0, 31)
    assert np.abs(dl[v] - rd[v]).max() <= 1e-5
    assert (dl[~v] == 0).all()


def _maps(orc, L, R, dmin, dmax, win):
    ref = orc.match(L, R, dmin, dmax, win)
    return ref


def test_lr_check_stage(B, orc):
    L, R = _pair(120, 300, 31, 41)
    ref = orc.match(L, R, 0, 31, 7)
    args = [cu(ref["oL"].astype(np.int16)), cu(ref["mL"]), cu(ref["oR"].astype(np.int16)), cu(ref["mR"])]
    for tol in (0, 1, 3):
        g = np_(B.st_lr_check(*args, tol=tol))
        assert np.array_equal(g, orc.lr_check(ref["oL"], ref["mL"], ref["oR"], ref["mR"], tol))


def test_outlier_stage_unaligned_masks(B, orc):
    """Mask buffers that start off a dword boundary (views one byte into a
    larger buffer) at a width that is a multiple of 4: the per-pixel kernels
    then take their pixels one by one instead of four per wide load, with
    the same result."""
    import torch
    H, W = 64, 400
    L, R = _pair(H, W, 31, 44)
    ref = orc.match(L, R, 0, 31, 7)
    m = orc.lr_check(ref["oL"], ref["mL"], ref["oR"], ref["mR"], 1)
    o = cu(ref["oL"].astype(np.int16))
    want = orc.radial_outlier(ref["oL"], m, 20, 2.5)
    buf = torch.zeros(H * W + 1, dtype=torch.uint8, device="cuda")
    m_in = buf[1:].view(H, W)
    m_in.copy_(cu(m))
    assert m_in.data_ptr() % 4 == 1
    out = torch.zeros(H * W + 3, dtype=torch.uint8, device="cuda")
    m_out = out[3:].view(H, W)
    from paper_2007_12623_amd import binding
    binding._check(binding.lib().st_radial_outlier(binding._h(None), o.data_ptr(), m_in.data_ptr(), H, W,
                                                   20, 2.5, m_out.data_ptr(), binding._stream(None)))
    torch.cuda.synchronize()
    assert np.array_equal(np_(m_out), want)
    assert np.array_equal(np_(B.st_radial_outlier(o, cu(m), 20, 2.5)), want)


@pytest.mark.parametrize("H,W", [(140, 330), (300, 70), (23, 700), (19, 1100), (12, 2100), (7, 4200)])
def test_outlier_and_fill_stages(B, orc, H, W):
    """Rows, columns and both diagonals cut into scan segments: shapes with
    lines shorter and longer than one segment, and rows of one, two and
    several register chunks of 16 x 64 columns (the last past 64 blocks,
    where the outlier rows keep their backward bits in memory)."""
    L, R = _pair(H, W, 31, 42)
    ref = orc.match(L, R, 0, 31, 7)
    m = orc.lr_check(ref["oL"], ref["mL"], ref["oR"], ref["mR"], 1)
    o = ref["oL"]
    # r <= 63 takes the bit-parallel row test, larger r the carried sweep
    for r in (1, 10, 20, 30, 63, 64, 100):
        g = np_(B.st_radial_outlier(cu(o.astype(np.int16)), cu(m), r, 2.5))
        assert np.array_equal(g, orc.radial_outlier(o, m, r, 2.5)), f"outlier r={r}"
    m2 = orc.radial_outlier(o, m, 10, 2.5)
    # radial radii on either side of 64 (one 64-column block of look-ahead)
    for args in ((50, 2, 20, 0.25), (5, 1, 3, 0.5), (0, 2, 20, 0.25), (50, 4, 0, 0.0),
                 (63, 2, 0, 0.0), (64, 2, 0, 0.0), (100, 1, 0, 0.0)):
        go, gm = B.st_fill(cu(o.astype(np.int16)), cu(m2), *args)
        ro, rm = orc.fill(o, m2, *args)
        assert np.array_equal(np_(gm), rm), f"fill mask {args}"
        assert np.array_equal(np_(go)[rm > 0], ro[rm > 0]), f"fill values {args}"


def test_fill_disk_radius_paths(B, orc):
    """Disk radii up to 63 in rows narrower than 4096 take packed row prefixes
    (count and sum modulo 2^20 in one word), up to 256 they sum in 32 bits,
    larger ones in 64: every path on the same holes, and the packed path's
    neighbours on either side of its radius limit."""
    L, R = _pair(60, 320, 31, 43)
    ref = orc.match(L, R, 0, 31, 7)
    m = orc.lr_check(ref["oL"], ref["mL"], ref["oR"], ref["mR"], 1)
    o = ref["oL"]
    m2 = orc.radial_outlier(o, m, 10, 2.5)
    # fractions near the valid share of the disks leave some holes unfilled
    for args in ((0, 2, 20, 0.25), (0, 2, 20, 0.8), (0, 2, 63, 0.8), (0, 2, 64, 0.8),
                 (0, 2, 256, 0.8), (0, 2, 257, 0.8), (0, 2, 300, 0.81), (0, 2, 256, 0.81)):
        go, gm = B.st_fill(cu(o.astype(np.int16)), cu(m2), *args)
        ro, rm = orc.fill(o, m2, *args)
        assert np.array_equal(np_(gm), rm), f"fill mask {args}"
        assert np.array_equal(np_(go)[rm > 0], ro[rm > 0]), f"fill values {args}"


def test_fill_disk_packed_extremes(B, orc):
    """The packed row prefixes at their limits: disparities of +-4096 over a
    radius-63 disk (a row segment sum near 2^19 in magnitude), a row of 4095
    pixels (row counts up to 4095 in the 12-bit field) and one of 4096, which
    takes the unpacked prefixes."""
    r = np.random.default_rng(77)
    # (shape, disparity range, valid share): 99 % valid at +-4090..4096 puts
    # row segments of ~126 valid cells, sums of ~5.2e5 < 2^19, next to holes
    for H, W, lo, hi, pv in ((140, 300, 4000, 4097, 0.4), (140, 300, -4096, -3999, 0.4),
                             (140, 300, 4090, 4097, 0.99), (140, 300, -4096, -4089, 0.99),
                             (40, 4095, -4096, 4097, 0.4), (40, 4096, -4096, 4097, 0.4)):
        o = r.integers(lo, hi, size=(H, W)).astype(np.int16)
        m = (r.random((H, W)) < pv).astype(np.uint8)
        for args in ((0, 2, 63, 0.05), (0, 2, 20, 0.25)):
            go, gm = B.st_fill(cu(o), cu(m), *args)
            ro, rm = orc.fill(o.astype(np.int32), m, *args)
            assert np.array_equal(np_(gm), rm), f"fill mask {H}x{W} {args}"
            assert np.array_equal(np_(go)[rm > 0], ro[rm > 0]), f"fill values {H}x{W} {args}"


@pytest.mark.parametrize("R,K", [(2, 1), (15, 3), (4, 2), (0, 1), (3, 0), (96, 2), (100, 2)])
def test_hc_smooth_stage(B, orc, R, K):
    r = np.random.default_rng(R * 10 + K)
    H, W = 90, 170
    s = (r.normal(40.0, 6.0, size=(H, W))).astype(np.float32)
    m = (r.random((H, W)) > 0.15).astype(np.uint8) * np.where(r.random((H, W)) > 0.5, 1, 2).astype(np.uint8)
    g = np_(B.st_hc_smooth(cu(s), cu(m), R, K, 0.1))
    ref = orc.hc_smooth(s.astype(np.float64), m, R, K, 0.1)
    v = m > 0
    assert np.isnan(g[~v]).all()
    tol = np.maximum(1e-5, np.spacing(np.abs(ref[v]).astype(np.float32)).astype(np.float64))
    assert np.all(np.abs(g[v] - ref[v]) <= tol)


def _end_to_end(B, orc, L, R, dmin, dmax, win, params_gpu, params_orc):
    """The whole GPU path stage by stage against the oracle (each oracle
    stage on the GPU's own input to it), then the final output against the
    oracle's pipeline from the images: exact outside the reach of the
    matcher's near-ties (see tests/e2e.py)."""
    g = e2e.run_debug(B, L, R, dmin, dmax, win, params_gpu)
    ref = orc.match(L, R, dmin, dmax, win, chess=bool(params_orc.chess))
    rep = e2e.stagewise(orc, L, R, dmin, dmax, win, g, params_orc, ref)
    n_cmp, n_excl = e2e.against_pipeline(orc, L, R, dmin, dmax, win, g["disp"], g["mask"],
                                         params_orc, ref)
    print(f"matching: {rep['int_disagree_px']} near-tie winners differ; final output compared "
          f"on {n_cmp} px, {n_excl} px within the near-ties' reach")


def test_end_to_end_small_workload(B, orc):
    p = synth.c1_pair()
    _end_to_end(B, orc, p["left"], p["right"], 0, 31, 7, B.preset("small"), orc.params_c1())


def test_end_to_end_full_pipeline(B, orc):
    """960x540 / 128 / 11x11 with 3 outlier-fill alternations and R=15, K=3."""
    seq = synth.c2_sequence(1)
    _end_to_end(B, orc, seq[0]["left"], seq[0]["right"], 0, 127, 11, B.preset("full"),
                orc.params_c2())


def test_end_to_end_paper_range(B, orc):
    """Signed range -20..80 through the whole pipeline."""
    p = synth.make_pair(200, 420, 80, 6106, dmin=-20)
    _end_to_end(B, orc, p["left"], p["right"], -20, 80, 11, B.preset("full"), orc.params_c2())


def test_pipeline_options(B, orc):
    """Pipeline with the left-right check and sub-pixel switched off."""
    L, R = _pair(100, 260, 31, 51)
    pg = B.preset("small", lr_check=0, subpixel=0, radial_iters=2, radial_r0=3, radial_dr=2)
    po = orc.params_c1(lr_check=0, subpixel=0, radial_iters=2, radial_r0=3, radial_dr=2)
    _end_to_end(B, orc, L, R, 0, 31, 7, pg, po)
