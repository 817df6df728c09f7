"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test names what pins it: brute-force sums, numpy's Pearson correlation
(which is ZNCC of two windows), closed forms, invariants, hand-built maps and
scipy box means.  CPU only.
"""
import numpy as np
import pytest
from scipy import ndimage

from paper_2007_12623_amd import synth


def rng(s):
    return np.random.default_rng(s)


# ---------------------------------------------------------------- window sums
@pytest.mark.parametrize("shape", [(16, 16), (23, 31), (40, 40)])
@pytest.mark.parametrize("win", [3, 5, 7, 11])
def test_window_stats_integral_equals_brute(orc, shape, win):
    img = rng(shape[0] * 100 + win).integers(0, 256, size=shape, dtype=np.uint8)
    a = orc.window_stats(img, win, brute=False)
    b = orc.window_stats(img, win, brute=True)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    S, SS, V, ins = a
    h = win // 2
    # direct numpy sums over every interior window
    for y in range(h, shape[0] - h):
        for x in range(h, shape[1] - h):
            w = img[y - h:y + h + 1, x - h:x + h + 1].astype(np.int64)
            assert S[y, x] == w.sum() and SS[y, x] == (w * w).sum()
    assert ins.sum() == (shape[0] - 2 * h) * (shape[1] - 2 * h)
    assert (V[ins == 1] >= 0).all()


# ---------------------------------------------------------------- ZNCC of two windows
def test_zncc_windows_is_pearson(orc):
    r = rng(1)
    for n in (9, 49, 121, 225):
        for _ in range(50):
            a = r.integers(0, 256, size=n, dtype=np.uint8)
            b = r.integers(0, 256, size=n, dtype=np.uint8)
            ref = np.corrcoef(a.astype(np.float64), b.astype(np.float64))[0, 1]
            assert abs(orc.zncc_windows(a, b) - ref) < 1e-12


def test_zncc_invariants(orc):
    r = rng(2)
    for _ in range(200):
        a = r.integers(0, 128, size=121, dtype=np.uint8)
        b = r.integers(0, 256, size=121, dtype=np.uint8)
        z = orc.zncc_windows(a, b)
        assert -1.0 - 1e-15 <= z <= 1.0 + 1e-15
        assert orc.zncc_windows(a, a) == pytest.approx(1.0, abs=1e-15)
        assert orc.zncc_windows(b, a) == pytest.approx(z, abs=1e-15)
        assert orc.zncc_windows((a + 17).astype(np.uint8), b) == pytest.approx(z, abs=1e-12)
        assert orc.zncc_windows((2 * a).astype(np.uint8), b) == pytest.approx(z, abs=1e-12)
        assert orc.zncc_windows((255 - a).astype(np.uint8), b) == pytest.approx(-z, abs=1e-12)
    flat = np.full(121, 7, np.uint8)
    assert np.isnan(orc.zncc_windows(flat, b))


# ---------------------------------------------------------------- cost volume + WTA
def _z_direct(L, R, x, y, d, win):
    h = win // 2
    a = L[y - h:y + h + 1, x - h:x + h + 1].astype(np.float64).ravel()
    b = R[y - h:y + h + 1, x - d - h:x - d + h + 1].astype(np.float64).ravel()
    if a.std() == 0 or b.std() == 0:
        return np.nan
    return np.corrcoef(a, b)[0, 1]


@pytest.mark.parametrize("win,dmin,dmax", [(3, 0, 6), (5, -3, 4), (7, 2, 9)])
def test_match_against_direct_definition(orc, win, dmin, dmax):
    r = rng(win)
    H, W = 14, 24
    L = r.integers(0, 256, size=(H, W), dtype=np.uint8)
    R = r.integers(0, 256, size=(H, W), dtype=np.uint8)
    R[2:6, 3:9] = 50  # a flat block -> zero-variance windows
    out = orc.match(L, R, dmin, dmax, win)
    outb = orc.match(L, R, dmin, dmax, win, brute=True)
    for k in out:
        assert np.array_equal(out[k], outb[k], equal_nan=True), k
    h = win // 2
    for y in range(H):
        for x in range(W):
            zs = []
            for d in range(dmin, dmax + 1):
                ok = h <= y < H - h and h <= x < W - h and h <= x - d < W - h
                zs.append(_z_direct(L, R, x, y, d, win) if ok else np.nan)
            zs = np.array(zs)
            if np.all(np.isnan(zs)):
                assert out["mL"][y, x] == 0
                continue
            best = int(np.nanargmax(zs))  # first maximum -> smallest d
            assert out["mL"][y, x] == 1 and out["oL"][y, x] == dmin + best
            assert out["zbest"][y, x] == pytest.approx(zs[best], abs=1e-12)
            others = np.delete(zs, best)
            if np.all(np.isnan(others)):
                assert np.isinf(out["gap"][y, x])
            else:
                assert out["gap"][y, x] == pytest.approx(zs[best] - np.nanmax(others), abs=1e-12)
            zm = zs[best - 1] if best > 0 else np.nan
            zp = zs[best + 1] if best < len(zs) - 1 else np.nan
            np.testing.assert_allclose(out["zm"][y, x], zm, atol=1e-12)
            np.testing.assert_allclose(out["zp"][y, x], zp, atol=1e-12)
    # right reference: xr takes (xr + d, d)
    for y in range(H):
        for xr in range(W):
            zs = []
            for d in range(dmin, dmax + 1):
                x = xr + d
                ok = h <= y < H - h and h <= x < W - h and h <= xr < W - h
                zs.append(_z_direct(L, R, x, y, d, win) if ok else np.nan)
            zs = np.array(zs)
            if np.all(np.isnan(zs)):
                assert out["mR"][y, xr] == 0
            else:
                assert out["oR"][y, xr] == dmin + int(np.nanargmax(zs))


def test_integer_shift_recovered_exactly(orc):
    r = rng(3)
    H, W, k = 30, 60, 6
    wide = r.integers(0, 256, size=(H, W + k), dtype=np.uint8)
    L = np.ascontiguousarray(wide[:, :W])      # L(x) = T(x)
    R = np.ascontiguousarray(wide[:, k:])      # R(x) = T(x + k), so L(x) = R(x - k)
    out = orc.match(L, R, 0, 12, 7)
    h = 3
    sel = np.zeros((H, W), bool)
    sel[h:H - h, h + k:W - h] = True
    assert (out["mL"][sel] == 1).all()
    assert (out["oL"][sel] == k).all()
    assert (out["zbest"][sel] == 1.0).all()
    selr = np.zeros((H, W), bool)
    selr[h:H - h, h:W - h - k] = True
    assert (out["oR"][selr] == k).all()


def test_wta_ties_go_to_smallest_disparity(orc):
    r = rng(4)
    H, W, P, k = 20, 80, 7, 3
    base = r.integers(0, 256, size=(H, P), dtype=np.uint8)
    wide = np.tile(base, (1, (W + k) // P + 2))[:, :W + k]
    L = np.ascontiguousarray(wide[:, :W])
    R = np.ascontiguousarray(wide[:, k:])
    out = orc.match(L, R, 0, 20, 5)
    # exact ties at d = 3, 10, 17 wherever all three are valid
    h = 2
    sel = np.zeros((H, W), bool)
    sel[h:H - h, h + 17:W - h] = True
    assert (out["oL"][sel] == 3).all()
    assert (out["gap"][sel] == 0.0).all()
    selr = np.zeros((H, W), bool)
    selr[h:H - h, h:W - h - 17] = True
    assert (out["oR"][selr] == 3).all()


# ---------------------------------------------------------------- sub-pixel
def test_subpixel_parabola_vertex(orc):
    t0 = np.linspace(-0.5, 0.5, 41)
    a, c = 0.37, 0.9
    f = lambda t: c - a * (t - t0) ** 2
    o = np.full(t0.shape, 5, np.int32)
    m = np.ones(t0.shape, np.uint8)
    dl = orc.subpixel(o, m, f(-1.0), f(0.0), f(1.0), 0, 10)
    np.testing.assert_allclose(dl, t0, atol=1e-14)


def test_subpixel_edge_cases(orc):
    o = np.array([0, 10, 5, 5, 5, 5], np.int32)
    m = np.array([1, 1, 1, 1, 0, 1], np.uint8)
    zm = np.array([0.5, 0.5, np.nan, 0.7, 0.5, 0.0])
    z0 = np.array([0.9, 0.9, 0.9, 0.7, 0.9, 0.9])
    zp = np.array([0.5, 0.5, 0.5, 0.7, 0.5, 0.95])
    dl = orc.subpixel(o, m, zm, z0, zp, 0, 10)
    assert dl[0] == 0 and dl[1] == 0      # range ends
    assert dl[2] == 0                     # missing neighbour
    assert dl[3] == 0                     # flat: curvature term == 0
    assert dl[4] == 0                     # invalid pixel
    # a neighbour above z0 puts the vertex beyond +1/2: clamped
    assert dl[5] == 0.5


# ---------------------------------------------------------------- left-right check
def test_lr_check_hand_built(orc):
    H, W = 4, 30
    oL = np.full((H, W), 5, np.int32)
    mL = np.ones((H, W), np.uint8)
    oR = np.full((H, W), 5, np.int32)
    mR = np.ones((H, W), np.uint8)
    oR[:, 10:13] = 7      # |5 - 7| = 2 > tol
    oR[:, 15:17] = 6      # |5 - 6| = 1 <= tol
    mR[:, 20] = 0         # right pixel without a match
    mL[:, 28] = 0
    out = orc.lr_check(oL, mL, oR, mR, tol=1)
    exp = np.ones((H, W), np.uint8)
    exp[:, :5] = 0                # x - 5 < 0
    exp[:, 15:18] = 0             # xr = 10..12
    exp[:, 25] = 0                # xr = 20
    exp[:, 28] = 0
    assert np.array_equal(out, exp)
    assert np.array_equal(orc.lr_check(oL, mL, oR, mR, tol=2)[:, 15:18], np.ones((H, 3), np.uint8))


# ---------------------------------------------------------------- radial outliers
def test_radial_outlier_hand_built(orc):
    H, W = 40, 40
    yy, xx = np.mgrid[0:H, 0:W]
    m = np.ones((H, W), np.uint8)
    const = np.full((H, W), 9, np.int32)
    assert np.array_equal(orc.radial_outlier(const, m, 10), m)
    ramp2 = (2 * xx).astype(np.int32)
    assert np.array_equal(orc.radial_outlier(ramp2, m, 10), m)   # step 2 < 2.5 kept
    steep = (3 * xx + 6 * yy).astype(np.int32)                   # every direction steps >= 3
    assert orc.radial_outlier(steep, m, 10).sum() == 0
    spike = const.copy(); spike[20, 20] = 19
    out = orc.radial_outlier(spike, m, 10)
    assert out[20, 20] == 0 and out.sum() == H * W - 1
    # a valid pixel cut off by a ring of holes at distance 3 in every direction
    ring = m.copy()
    ring[(np.maximum(abs(yy - 20), abs(xx - 20)) == 3)] = 0
    out = orc.radial_outlier(const, ring, 10)
    assert out[20, 20] == 0 and out[20, 22] == 0 and out[5, 5] == 1
    # codes of kept pixels survive; r larger than the image in every direction removes all
    m2 = m * 2
    assert np.array_equal(orc.radial_outlier(const, m2, 10), m2)
    assert orc.radial_outlier(const, m, 40).sum() == 0


# ---------------------------------------------------------------- hole filling
def test_fill_linear_ramp_exact(orc):
    H, W = 60, 70
    yy, xx = np.mgrid[0:H, 0:W]
    f = (2 * xx - 3 * yy + 7).astype(np.int32)
    m = np.ones((H, W), np.uint8)
    r = rng(5)
    holes = r.random((H, W)) < 0.15
    holes[0, :] = holes[-1, :] = False
    holes[:, 0] = holes[:, -1] = False
    m[holes] = 0
    o = f.copy(); o[holes] = -999
    o2, m2 = orc.fill(o, m)
    assert (m2[holes] == 2).all() and (m2[~holes] == 1).all()
    assert np.array_equal(o2, f)   # line interpolants are exact on linear data


def test_fill_constant_by_disk(orc):
    H, W = 50, 50
    m = (rng(8).random((H, W)) < 0.4).astype(np.uint8)
    o = np.where(m == 1, 42, 0).astype(np.int32)
    o2, m2 = orc.fill(o, m, radial_r=0)  # radial search switched off: disk only
    filled = m2 == 2
    assert filled.sum() == (m == 0).sum() and (o2[filled] == 42).all()


def test_fill_round_half_even(orc):
    def one_hole(e, w, n, s):
        o = np.zeros((3, 3), np.int32)
        m = np.zeros((3, 3), np.uint8)
        o[1, 2], o[1, 0], o[0, 1], o[2, 1] = e, w, n, s
        m[1, 2] = m[1, 0] = m[0, 1] = m[2, 1] = 1
        o2, m2 = orc.fill(o, m, radial_r=1, disk_r=0)
        return o2[1, 1], m2[1, 1]
    assert one_hole(1, 2, 1, 2) == (2, 2)    # 1.5 -> 2
    assert one_hole(2, 3, 2, 3) == (2, 2)    # 2.5 -> 2
    assert one_hole(-1, -2, -1, -2) == (-2, 2)  # -1.5 -> -2
    assert one_hole(3, 4, 3, 3) == (3, 2)    # (3.5 + 3) / 2 = 3.25 -> 3


def test_fill_disk_threshold(orc):
    # a hole in the corner of a 21x21 map: disk cells inside the image counted exactly
    H = W = 21
    cells = sum(1 for dy in range(-20, 21) for dx in range(-20, 21)
                if dx * dx + dy * dy <= 400 and 0 <= dy < H and 0 <= dx < W)
    need = int(np.ceil(0.25 * cells))
    order = [(y, x) for y in range(H) for x in range(W) if (y, x) != (0, 0) and y * y + x * x <= 400]
    for have, expect in ((need, 2), (need - 1, 0)):
        m = np.zeros((H, W), np.uint8)
        o = np.zeros((H, W), np.int32)
        for (y, x) in order[:have]:
            m[y, x] = 1; o[y, x] = 5
        o2, m2 = orc.fill(o, m, radial_r=0)
        assert m2[0, 0] == expect


# ---------------------------------------------------------------- smoothing
def _masked_mean_scipy(f, m, R):
    k = np.ones((2 * R + 1, 2 * R + 1))
    num = ndimage.correlate(np.where(m > 0, f, 0.0), k, mode="constant", cval=0.0)
    den = ndimage.correlate((m > 0).astype(np.float64), k, mode="constant", cval=0.0)
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(m > 0, num / den, np.nan)


def test_hc_preserves_constants_and_planes(orc):
    H, W = 50, 60
    m = np.ones((H, W), np.uint8)
    r = rng(6)
    m[r.random((H, W)) < 0.1] = 0
    c = np.full((H, W), 3.25)
    out = orc.hc_smooth(c, m, 2, 3)
    np.testing.assert_allclose(out[m > 0], 3.25, atol=1e-12)
    assert np.isnan(out[m == 0]).all()
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    plane = 0.3 * xx - 0.7 * yy + 11.0
    full = np.ones((H, W), np.uint8)
    R, K = 3, 2
    out = orc.hc_smooth(plane, full, R, K)
    g = 2 * R * K + R
    np.testing.assert_allclose(out[g:H - g, g:W - g], plane[g:H - g, g:W - g], atol=1e-11)


def test_hc_one_iteration_closed_form(orc):
    H, W = 40, 45
    r = rng(7)
    s = r.normal(30.0, 5.0, size=(H, W))
    m = (r.random((H, W)) > 0.2).astype(np.uint8)
    R = 2
    A = _masked_mean_scipy(s, m, R)
    AA = _masked_mean_scipy(np.where(m > 0, A, 0.0), m, R)
    out = orc.hc_smooth(s, m, R, 1, alpha=0.1)
    np.testing.assert_allclose(out[m > 0], (2 * A - AA)[m > 0], atol=1e-10)
    # alpha enters from the second iteration on: K=2 by hand with scipy means
    alpha = 0.1
    d1 = 2 * A - AA
    b2 = A - alpha * s - (1 - alpha) * d1
    d2 = A - _masked_mean_scipy(np.where(m > 0, b2, 0.0), m, R)
    out2 = orc.hc_smooth(s, m, R, 2, alpha=alpha)
    np.testing.assert_allclose(out2[m > 0], d2[m > 0], atol=1e-10)


# ---------------------------------------------------------------- whole pipeline
def test_pipeline_recovers_synthetic_disparity(orc):
    p = synth.c1_pair()
    disp, mask, inter = orc.pipeline(p["left"], p["right"], 0, 31, 7, orc.params_c1(),
                                     intermediates=True)
    gt = p["gt_left"]
    sel = (~np.isnan(gt)) & (inter["m_lr"] == 1)
    err = np.abs(inter["o_wta"][sel] - np.rint(gt[sel]))
    assert (err <= 1).mean() >= 0.95
    v = mask > 0
    assert v.mean() > 0.8
    assert np.nanmedian(np.abs(disp[v & ~np.isnan(gt)] - gt[v & ~np.isnan(gt)])) < 0.5


def _rig_q(f, B, cx, cy):
    # reprojection matrix of a horizontal rectified rig: W = d / B
    return np.array([[1, 0, 0, -cx], [0, 1, 0, -cy], [0, 0, 0, f], [0, 0, 1.0 / B, 0]], np.float64)


def test_reproject_closed_form(orc):
    """Section II's depth from disparity: Z = f B / d, X = (x - cx) Z / f,
    Y = (y - cy) Z / f for a horizontal rig; NaN for invalid or zero
    disparity (W = 0)."""
    f, Bl, cx, cy = 800.0, 5.0, 31.5, 20.25
    rng = np.random.default_rng(4)
    H, W = 40, 64
    d = rng.uniform(2.0, 90.0, size=(H, W))
    d[3, 5] = np.nan
    d[7, 9] = 0.0
    xyz = orc.reproject(d, _rig_q(f, Bl, cx, cy))
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    ok = np.isfinite(d) & (d != 0)
    Z = f * Bl / np.where(ok, d, 1.0)
    np.testing.assert_allclose(xyz[..., 2][ok], Z[ok], rtol=1e-12)
    np.testing.assert_allclose(xyz[..., 0][ok], ((xx - cx) * Z / f)[ok], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(xyz[..., 1][ok], ((yy - cy) * Z / f)[ok], rtol=1e-12, atol=1e-12)
    assert np.isnan(xyz[3, 5]).all() and np.isnan(xyz[7, 9]).all()


def test_reproject_fronto_parallel_plane(orc):
    """A constant disparity is a plane at constant depth whose points are
    evenly spaced by Z / f per pixel."""
    f, Bl = 1000.0, 4.0
    d = np.full((8, 12), 40.0)
    xyz = orc.reproject(d, _rig_q(f, Bl, 0.0, 0.0))
    assert np.allclose(xyz[..., 2], 100.0, rtol=0, atol=1e-12)
    assert np.allclose(np.diff(xyz[..., 0], axis=1), 0.1, atol=1e-12)
    assert np.allclose(np.diff(xyz[..., 1], axis=0), 0.1, atol=1e-12)
