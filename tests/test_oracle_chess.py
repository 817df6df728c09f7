"""Pins of the oracle's chessboard window (Section II-A: the matching reads
every other pixel of the window, laid out like a chessboard).  Reading: the
cells kept are those whose offsets (u, v) from the window centre have u + v
even, so the centre is kept and an 11x11 window keeps 61 of 121 cells.

The pins: the cell count on a constant image, window sums against numpy
masks, the matching against numpy's Pearson correlation over the kept cells
(brute force on small images), the integral-image path against the direct
loops, a pair whose other-colour cells are corrupted (only pixels whose
window colour avoids them must still match exactly), and the Eq. (4)
re-search over the whole range against the winner-take-all."""
import numpy as np
import pytest


def _mask(win):
    h = win // 2
    u = np.arange(-h, h + 1)
    return (u[:, None] + u[None, :]) % 2 == 0


@pytest.mark.parametrize("win", [3, 5, 7, 11, 15])
def test_cell_count_on_constant_image(orc, win):
    img = np.ones((win + 4, win + 6), np.uint8)
    S, SS, V, ins = orc.window_stats(img, win, chess=True)
    n = (win * win + 1) // 2
    assert n == int(_mask(win).sum())
    assert np.all(S[ins == 1] == n) and np.all(SS[ins == 1] == n) and np.all(V[ins == 1] == 0)
    if win == 11:
        assert n == 61


def test_window_sums_against_numpy_mask(orc):
    r = np.random.default_rng(11)
    img = r.integers(0, 256, size=(19, 27), dtype=np.uint8)
    for win in (3, 7, 11):
        h, mk = win // 2, _mask(win)
        n = int(mk.sum())
        S, SS, V, ins = orc.window_stats(img, win, chess=True)
        for y in range(19):
            for x in range(27):
                inside = h <= y < 19 - h and h <= x < 27 - h
                assert ins[y, x] == inside
                if not inside:
                    continue
                p = img[y - h:y + h + 1, x - h:x + h + 1].astype(np.int64)[mk]
                assert S[y, x] == p.sum() and SS[y, x] == (p * p).sum()
                assert V[y, x] == n * (p * p).sum() - p.sum() ** 2


def _brute_match(L, R, dmin, dmax, win):
    """Left-reference WTA by numpy's Pearson correlation over the kept cells."""
    H, W = L.shape
    h, mk = win // 2, _mask(win)
    D = dmax - dmin + 1
    z = np.full((D, H, W), np.nan)
    for y in range(h, H - h):
        for x in range(h, W - h):
            a = L[y - h:y + h + 1, x - h:x + h + 1].astype(np.float64)[mk]
            if a.std() == 0:
                continue
            for i, d in enumerate(range(dmin, dmax + 1)):
                xr = x - d
                if xr < h or xr > W - 1 - h:
                    continue
                b = R[y - h:y + h + 1, xr - h:xr + h + 1].astype(np.float64)[mk]
                if b.std() == 0:
                    continue
                z[i, y, x] = np.corrcoef(a, b)[0, 1]
    return z


def test_match_against_pearson(orc):
    r = np.random.default_rng(5)
    H, W, win, dmin, dmax = 14, 34, 5, -2, 6
    L = r.integers(0, 256, size=(H, W), dtype=np.uint8)
    R = np.roll(L, -3, axis=1)
    R = np.clip(R.astype(int) + r.integers(-40, 41, size=(H, W)), 0, 255).astype(np.uint8)
    # a flat block gives zero-variance windows (invalid candidates)
    L[2:9, 20:28] = 77
    z = _brute_match(L, R, dmin, dmax, win)
    out = orc.match(L, R, dmin, dmax, win, chess=True)
    anyv = ~np.all(np.isnan(z), axis=0)
    assert np.array_equal(out["mL"].astype(bool), anyv)
    zz = np.where(np.isnan(z), -np.inf, z)
    best = np.argmax(zz, axis=0)  # first maximum: ties to the smallest d
    ys, xs = np.nonzero(anyv)
    for y, x in zip(ys, xs):
        col = zz[:, y, x]
        b = best[y, x]
        # the maximum is unique up to rounding of the two computations
        if np.sum(np.abs(col - col[b]) < 1e-12) == 1:
            assert out["oL"][y, x] == dmin + b
        assert abs(out["zbest"][y, x] - col[b]) < 1e-12
        k = out["oL"][y, x] - dmin
        for nb, key in ((k - 1, "zm"), (k + 1, "zp")):
            ref = z[nb, y, x] if 0 <= nb < z.shape[0] else np.nan
            got = out[key][y, x]
            assert (np.isnan(ref) and np.isnan(got)) or abs(ref - got) < 1e-12


def test_integral_path_equals_direct_loops(orc):
    r = np.random.default_rng(8)
    H, W = 40, 90
    L = r.integers(0, 256, size=(H, W), dtype=np.uint8)
    R = np.clip(np.roll(L, -7, axis=1).astype(int) + r.integers(-20, 21, size=(H, W)), 0,
                255).astype(np.uint8)
    for win in (5, 11):
        a = orc.match(L, R, 0, 15, win, chess=True)
        b = orc.match(L, R, 0, 15, win, brute=True, chess=True)
        for key in ("oL", "mL", "oR", "mR"):
            assert np.array_equal(a[key], b[key]), key
        for key in ("zbest", "zm", "zp", "zbestR"):
            assert np.array_equal(np.isnan(a[key]), np.isnan(b[key])), key
            f = ~np.isnan(a[key])
            assert np.max(np.abs(a[key][f] - b[key][f]), initial=0.0) < 1e-12, key


def _corrupted_pair(k, H=36, W=100, seed=4):
    """R = L shifted by k (even), then every right cell with x + y odd
    replaced by noise."""
    assert k % 2 == 0
    r = np.random.default_rng(seed)
    wide = r.integers(0, 256, size=(H, W + k), dtype=np.uint8)
    L, R = wide[:, :W].copy(), wide[:, k:].copy()  # L(x) = R(x - k)
    yy, xx = np.mgrid[0:H, 0:W]
    odd = (xx + yy) % 2 == 1
    R[odd] = r.integers(0, 256, size=int(odd.sum()), dtype=np.uint8)
    return L, R


def test_other_colour_is_never_read(orc):
    """A left pixel with x + y even pairs even cells of L with even cells of R
    at an even shift: its z at the true shift is exactly 1 and wins.  The
    full window sees the noise and does not reach 1."""
    k, win = 6, 11
    L, R = _corrupted_pair(k)
    H, W = L.shape
    h = win // 2
    ch = orc.match(L, R, 0, 15, win, chess=True)
    full = orc.match(L, R, 0, 15, win)
    yy, xx = np.mgrid[0:H, 0:W]
    sel = (yy >= h) & (yy < H - h) & (xx >= k + h) & (xx < W - h)
    even = sel & ((xx + yy) % 2 == 0)
    odd = sel & ((xx + yy) % 2 == 1)
    assert np.all(ch["oL"][even] == k)
    assert np.max(np.abs(ch["zbest"][even] - 1.0)) < 1e-12
    # odd-colour windows read the corrupted cells; the full window too
    assert np.all(ch["zbest"][odd] < 0.99)
    assert np.all(full["zbest"][sel] < 0.99)


def test_research_over_whole_range_equals_wta(orc):
    """eta = 0 and a window covering [dmin, dmax]: minimising 1/max(z, 1e-3)
    is maximising z wherever the best z exceeds 1e-3, so the re-search
    (direct sums) returns the winner-take-all of the matcher (integral
    images), ties to the smaller disparity on both sides."""
    r = np.random.default_rng(9)
    H, W, dmin, dmax, win = 30, 80, 0, 11, 7
    L = r.integers(0, 256, size=(H, W), dtype=np.uint8)
    R = np.clip(np.roll(L, -5, axis=1).astype(int) + r.integers(-60, 61, size=(H, W)), 0,
                255).astype(np.uint8)
    w = orc.match(L, R, dmin, dmax, win, chess=True)
    m = w["mL"].copy()
    m[w["zbest"] <= 1e-3] = 0
    d = np.full((H, W), (dmin + dmax) / 2.0)
    rng_ = (dmax - dmin) // 2 + 1
    o = orc.research(L, R, dmin, dmax, win, np.zeros((H, W), np.int32), m, d, rng_, 0.0,
                     chess=True)
    sel = m == 1
    assert sel.sum() > 500
    assert np.array_equal(o[sel], w["oL"][sel])


def test_pipeline_with_chessboard_recovers_synthetic_disparity(orc):
    """The whole path with the chessboard window (11x11 as in the paper) on a
    seeded synthetic pair still lands on the known disparity field."""
    from paper_2007_12623_amd import synth
    p = synth.c1_pair()
    disp, mask, inter = orc.pipeline(p["left"], p["right"], 0, 31, 11,
                                     orc.params_c1(chess=1), intermediates=True)
    gt = p["gt_left"]
    sel = (~np.isnan(gt)) & (inter["m_lr"] == 1)
    err = np.abs(inter["o_wta"][sel] - np.rint(gt[sel]))
    assert (err <= 1).mean() >= 0.95
    v = (mask > 0) & ~np.isnan(gt)
    assert np.nanmedian(np.abs(disp[v] - gt[v])) < 0.5
