"""Pins of the oracle's whole-path composition (Section II, Fig. 1(a):
matching, left-right check, outlier removal / hole filling alternations,
smoothing, optionally with the Eq. (4) re-search) on pairs whose every
intermediate is known in closed form.

A pair is a noise-free integer shift k of uniform noise with one flat
square block.  Matching then gives o = k wherever candidate k is valid (its
ZNCC is exactly 1 and every other candidate's is lower) and no candidate
where the left window is all flat.  With candidates from k - 4 and a
left-right tolerance of 0, the check keeps exactly the rectangle of pixels
whose candidate k has both windows inside the image: in the four columns to
its left only smaller candidates are valid, and the right-reference winner
there is k.  Every disparity that survives is k, so outlier removal and both
fills act on validity alone (a fill value is a mean of k's) and the whole
hole-filling schedule can be replayed on a boolean map by brute force
(`_replay_masks`).  The expected maps come from that geometry, numpy's
Pearson correlation and scipy box means, never from the oracle."""
import numpy as np
import pytest
from scipy import ndimage

DIRS = [(1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (-1, -1), (1, -1), (-1, 1)]


class Geo:
    def __init__(self, k, H, W, win, fy, fx, F, seed):
        self.k, self.H, self.W, self.win, self.h = k, H, W, win, win // 2
        r = np.random.default_rng(seed)
        wide = r.integers(0, 256, size=(H, W + k), dtype=np.uint8)
        wide[fy:fy + F, fx:fx + F] = 128
        self.L, self.R = wide[:, :W].copy(), wide[:, k:].copy()
        h = self.h
        self.rect = np.zeros((H, W), bool)
        self.rect[h:H - h, h + k:W - h] = True
        self.block = np.zeros((H, W), bool)
        if F > 2 * h:
            self.block[fy + h:fy + F - h, fx + h:fx + F - h] = True
        self.matched = self.rect & ~self.block

    def pearson(self, y, x, c):
        h, W = self.h, self.W
        if not (h <= x - c <= W - 1 - h):
            return np.nan
        a = self.L[y - h:y + h + 1, x - h:x + h + 1].astype(np.float64).ravel()
        b = self.R[y - h:y + h + 1, x - c - h:x - c + h + 1].astype(np.float64).ravel()
        if a.std() == 0 or b.std() == 0:
            return np.nan
        return np.corrcoef(a, b)[0, 1]

    def parabola(self, y, x, o):
        zm, z0, zp = (self.pearson(y, x, c) for c in (o - 1, o, o + 1))
        if np.isnan(zm) or np.isnan(zp):
            return 0.0
        den = 2.0 * (zm - 2.0 * z0 + zp)
        return float(np.clip((zm - zp) / den, -0.5, 0.5)) if den < 0 else 0.0


GA = Geo(5, 48, 110, 7, 18, 40, 11, 5)     # 5 x 5 flat hole block, thin frame
GB = Geo(12, 48, 110, 15, 16, 50, 19, 6)   # 5 x 5 flat hole block, thick frame
GC = Geo(5, 30, 36, 7, 0, 0, 0, 7)         # no flat block; smaller than 41 x 41


def _shifted(valid, dy, dx):
    """out[y, x] = valid[y + dy, x + dx], False outside the image."""
    H, W = valid.shape
    pad = np.zeros((H + 2 * abs(dy), W + 2 * abs(dx)), bool)
    pad[abs(dy):abs(dy) + H, abs(dx):abs(dx) + W] = valid
    return pad[abs(dy) + dy:abs(dy) + dy + H, abs(dx) + dx:abs(dx) + dx + W]


def _hit_within(valid, dy, dx, R):
    """True where some step s <= R along (dx, dy) lands on a valid pixel
    inside the image."""
    hit = np.zeros(valid.shape, bool)
    for s in range(1, R + 1):
        hit |= _shifted(valid, s * dy, s * dx)
    return hit


def _run_ok(valid, dy, dx, r):
    """True where all r steps along (dx, dy) are inside the image and valid."""
    ok = np.ones(valid.shape, bool)
    for s in range(1, r + 1):
        ok &= _shifted(valid, s * dy, s * dx)
    return ok


def _disk_fill(valid, radius=20, frac=0.25):
    H, W = valid.shape
    dy, dx = np.mgrid[-radius:radius + 1, -radius:radius + 1]
    keep = (dx * dx + dy * dy) <= radius * radius
    kern = keep.astype(np.float64)
    cnt = ndimage.correlate(valid.astype(np.float64), kern, mode="constant", cval=0.0)
    cells = ndimage.correlate(np.ones((H, W)), kern, mode="constant", cval=0.0)
    return valid | ((cnt > 0) & (cnt >= np.ceil(frac * cells - 1e-9)))


def _replay_masks(valid0, iters, r0=10, dr=10, fill_r=50, lines=2):
    """The outlier / fill schedule on a map whose every disparity is equal:
    returns the final 0/1/2 mask."""
    code = valid0.astype(np.uint8)
    sched = [None] if iters == 0 else [r0 + i * dr for i in range(iters)]
    for r in sched:
        valid = code > 0
        if r is not None:
            passes = np.zeros_like(valid)
            for dx, dy in DIRS:
                passes |= _run_ok(valid, dy, dx, r)
            code = np.where(valid & passes, code, 0).astype(np.uint8)
            valid = code > 0
        nl = np.zeros(valid.shape, np.int64)
        for i in range(4):
            (ax, ay), (bx, by) = DIRS[2 * i], DIRS[2 * i + 1]
            nl += _hit_within(valid, ay, ax, fill_r) & _hit_within(valid, by, bx, fill_r)
        rad = valid | (nl >= lines)
        full = _disk_fill(rad)
        code = np.where(valid, code, np.where(full, 2, 0)).astype(np.uint8)
    return code


def _masked_mean(f, m, R):
    k = np.ones((2 * R + 1, 2 * R + 1))
    num = ndimage.correlate(np.where(m > 0, f, 0.0), k, mode="constant", cval=0.0)
    den = ndimage.correlate((m > 0).astype(np.float64), k, mode="constant", cval=0.0)
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(m > 0, num / den, np.nan)


def _delta(g):
    out = np.zeros((g.H, g.W))
    for y, x in zip(*np.nonzero(g.matched)):
        assert g.pearson(y, x, g.k) == pytest.approx(1.0, abs=1e-12)
        out[y, x] = g.parabola(y, x, g.k)
    return out


def _margin_offsets(g):
    """Parabola offsets of the WTA winners in the four columns left of the
    rectangle (candidates k-4 .. k-1 only), which the left-right check
    removes."""
    out = []
    for y in range(g.h, g.H - g.h):
        for x in range(g.h + g.k - 4, g.h + g.k):
            zs = {c: g.pearson(y, x, c) for c in range(g.k - 4, g.k)}
            zs = {c: z for c, z in zs.items() if not np.isnan(z)}
            o = max(zs, key=lambda c: (zs[c], -c))
            if g.k - 4 < o:
                out.append(g.parabola(y, x, o))
    return np.array(out)


@pytest.mark.parametrize("g", [GA, GB, GC], ids=["win7", "win15", "small"])
@pytest.mark.parametrize("smooth", [0, 1, 3])
def test_pipeline_closed_form_plain(orc, g, smooth):
    """research = 0, candidates k-4 .. k+4, tolerance 0, 3 alternations.
    smooth = 0: the output is s itself - o + delta on matched pixels, o on
    filled ones (the winners removed by the left-right check have non-zero
    offsets, which must not reach s); smooth > 0: Eqs. (1)-(3) on that s over
    the final mask, by hand with scipy box means."""
    k = g.k
    mask_ref = _replay_masks(g.matched, 3)
    delta = _delta(g)
    assert np.abs(delta[g.matched]).max() > 0.01
    assert np.abs(_margin_offsets(g)).max() > 0.01
    s = np.where(mask_ref == 1, k + delta, np.where(mask_ref == 2, float(k), np.nan))
    Rs, alpha = 4, 0.1
    want = s
    if smooth:
        a = _masked_mean(s, mask_ref, Rs)
        d = s
        for _ in range(smooth):
            b = a - alpha * s - (1 - alpha) * d
            d = a - _masked_mean(np.where(mask_ref > 0, b, 0.0), mask_ref, Rs)
        want = d
    p = orc.params_c2(lr_tol=0, smooth_radius=Rs, smooth_iters=smooth, smooth_alpha=alpha)
    disp, mask, inter = orc.pipeline(g.L, g.R, k - 4, k + 4, g.win, p, intermediates=True)
    assert np.array_equal(inter["m_lr"], g.matched.astype(np.uint8))
    assert (inter["o_wta"][g.matched] == k).all()
    np.testing.assert_allclose(inter["delta"][g.matched], delta[g.matched], rtol=0, atol=1e-9)
    assert np.array_equal(mask, mask_ref)
    assert (inter["o_post"] == k).all()
    np.testing.assert_allclose(disp, want, rtol=0, atol=1e-9)


def test_outlier_radius_grows(orc):
    """On the 30 x 36 pair no direction from the central columns has 20
    steps inside the image: the second alternation (r = 20) removes matched
    pixels there, which the first (r = 10) kept, and its fill refills them
    (code 2)."""
    g = GC
    ref = _replay_masks(g.matched, 3)
    assert ((ref == 2) & g.matched).any()
    assert (_replay_masks(g.matched, 1)[g.matched] == 1).all()
    p = orc.params_c2(lr_tol=0, smooth_iters=0)
    disp, mask = orc.pipeline(g.L, g.R, g.k - 4, g.k + 4, g.win, p)
    assert np.array_equal(mask, ref)


def test_alternations_are_counted(orc):
    """The thick frame of the 15 x 15 pair is not filled in one alternation
    (the disk around an image corner holds no matched pixel); three
    alternations fill it, a single one leaves holes."""
    g = GB
    one, three = _replay_masks(g.matched, 1), _replay_masks(g.matched, 3)
    assert (one == 0).any() and (three > 0).all()
    for iters, ref in ((1, one), (3, three), (2, _replay_masks(g.matched, 2))):
        p = orc.params_c2(lr_tol=0, radial_iters=iters, smooth_iters=0)
        disp, mask = orc.pipeline(g.L, g.R, g.k - 4, g.k + 4, g.win, p)
        assert np.array_equal(mask, ref), iters
        assert np.isnan(disp[mask == 0]).all()
        assert (disp[mask == 2] == g.k).all()


@pytest.mark.parametrize("g", [GA, GB], ids=["win7", "win15"])
def test_pipeline_closed_form_single_fill_pass(orc, g):
    """radial_iters = 0: one fill pass and no outlier removal."""
    p = orc.params_c1(lr_tol=0, smooth_iters=0)
    disp, mask = orc.pipeline(g.L, g.R, g.k - 4, g.k + 4, g.win, p)
    assert np.array_equal(mask, _replay_masks(g.matched, 0))


@pytest.mark.parametrize("g", [GA, GB], ids=["win7", "win15"])
def test_pipeline_closed_form_research(orc, g):
    """research = 1 with candidates k .. k+7: o = k is the re-search's
    choice on the rectangle (ZNCC 1 and no smoothing cost at d = k), and no
    candidate is defined on the frame or on the flat block, so d = k
    wherever the final mask is set."""
    mask_ref = _replay_masks(g.matched, 3)
    p = orc.params_c2(research=1, smooth_radius=4, smooth_iters=3)
    disp, mask, inter = orc.pipeline(g.L, g.R, g.k, g.k + 7, g.win, p, intermediates=True)
    assert np.array_equal(inter["m_lr"], g.matched.astype(np.uint8))
    assert np.array_equal(mask, mask_ref)
    assert (disp[mask > 0] == float(g.k)).all()
    assert np.isnan(disp[mask == 0]).all()
