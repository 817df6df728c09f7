"""Pins of the Eq. (4) re-search (Section II-C) in the oracle: limits where
the cost reduces to a known answer, a brute-force textbook-ZNCC argmin, and
the reduction of Eqs. (1)-(4) to the plain smoothing when no re-search runs."""
import numpy as np
import pytest

from paper_2007_12623_amd import synth


def _shift_pair(k, H=40, W=90, seed=3):
    r = np.random.default_rng(seed)
    wide = r.integers(0, 256, size=(H, W + k), dtype=np.uint8)
    return wide[:, :W].copy(), wide[:, k:].copy()


def test_large_eta_rounds_d(orc):
    """eta -> infinity: the smoothing term decides; o = the integer nearest d."""
    p = synth.make_pair(50, 120, 31, 21)
    L, R = p["left"], p["right"]
    r = np.random.default_rng(1)
    d = r.uniform(8.0, 24.0, size=L.shape)
    d = np.where(np.abs(d - np.floor(d) - 0.5) < 0.05, d + 0.2, d)  # keep off .5
    m = np.zeros(L.shape, np.uint8)
    m[10:40, 40:110] = 1
    o0 = np.full(L.shape, 7, np.int32)
    o = orc.research(L, R, 0, 31, 7, o0, m, d, 5, 1e9)
    sel = m == 1
    assert np.array_equal(o[sel], np.rint(d[sel]).astype(np.int32))
    assert np.array_equal(o[~sel], o0[~sel])


def test_zero_eta_finds_exact_shift(orc):
    """eta = 0 on a noise-free integer shift: z = 1 only at the shift, and
    1/z is smallest there."""
    k = 6
    L, R = _shift_pair(k)
    H, W = L.shape
    m = np.zeros((H, W), np.uint8)
    m[5:35, 20:80] = 1
    d = np.full((H, W), k + 3.3)
    o = orc.research(L, R, 0, 20, 9, np.zeros((H, W), np.int32), m, d, 5, 0.0)
    assert (o[m == 1] == k).all()


def test_cost_argmin_brute_force(orc):
    """The chosen candidate minimises 1/max(z, 1e-3) + eta (c - d)^2 with z
    the textbook ZNCC of the two windows."""
    p = synth.make_pair(40, 100, 31, 5)
    L, R = p["left"].astype(np.float64), p["right"].astype(np.float64)
    win, h, eta = 7, 3, 0.01
    r = np.random.default_rng(9)
    d = r.uniform(3.0, 28.0, size=L.shape)
    m = np.ones(L.shape, np.uint8)
    o = orc.research(p["left"], p["right"], 0, 31, win, np.zeros(L.shape, np.int32), m, d, 5, eta)
    for (y, x) in [(10, 40), (20, 60), (30, 80), (15, 35), (25, 95)]:
        best, arg = np.inf, None
        for c in range(max(0, int(np.ceil(d[y, x] - 5))), min(31, int(np.floor(d[y, x] + 5))) + 1):
            xr = x - c
            if not (h <= x <= L.shape[1] - 1 - h and h <= xr <= L.shape[1] - 1 - h):
                continue
            a = L[y - h:y + h + 1, x - h:x + h + 1].ravel()
            b = R[y - h:y + h + 1, xr - h:xr + h + 1].ravel()
            z = np.corrcoef(a, b)[0, 1]
            cost = 1.0 / max(z, 1e-3) + eta * (c - d[y, x]) ** 2
            if cost < best - 1e-12:
                best, arg = cost, c
        assert o[y, x] == arg, (y, x)


def test_one_iteration_is_plain_smoothing(orc):
    """K = 1: no re-search runs before the output, so Eqs. (1)-(4) give the
    improved Laplacian smoothing of o."""
    p = synth.make_pair(40, 80, 31, 8)
    r = np.random.default_rng(2)
    o = r.integers(5, 25, size=(40, 80)).astype(np.int32)
    m = (r.random((40, 80)) > 0.2).astype(np.uint8)
    d, oo = orc.hc_research(p["left"], p["right"], 0, 31, 7, o, m, 3, 1, 0.1, 0.01, 5)
    ref = orc.hc_smooth(o.astype(np.float64), m, 3, 1, 0.1)
    v = m == 1
    np.testing.assert_allclose(d[v], ref[v], rtol=0, atol=1e-12)
    assert np.isnan(d[~v]).all() and np.array_equal(oo, o)


def test_exact_shift_is_a_fixed_point(orc):
    """A noise-free integer shift with o = k everywhere: smoothing keeps
    d = k and the re-search keeps o = k."""
    k = 4
    L, R = _shift_pair(k, 50, 100, 11)
    m = np.zeros(L.shape, np.uint8)
    m[6:44, 12:94] = 1
    o = np.where(m == 1, k, 0).astype(np.int32)
    d, oo = orc.hc_research(L, R, 0, 15, 7, o, m, 4, 3, 0.1, 0.01, 5)
    np.testing.assert_allclose(d[m == 1], k, atol=1e-12)
    assert (oo[m == 1] == k).all()


def _masked_mean(f, m, R):
    """Mean of f over the pixels with m != 0 in the (2R+1)^2 square around
    each pixel (scipy box sums; NaN where m == 0)."""
    from scipy import ndimage
    k = np.ones((2 * R + 1, 2 * R + 1))
    num = ndimage.correlate(np.where(m > 0, f, 0.0), k, mode="constant", cval=0.0)
    den = ndimage.correlate((m > 0).astype(np.float64), k, mode="constant", cval=0.0)
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(m > 0, num / den, np.nan)


def _pearson(L, R, y, x, c, h):
    a = L[y - h:y + h + 1, x - h:x + h + 1].astype(np.float64).ravel()
    b = R[y - h:y + h + 1, x - c - h:x - c + h + 1].astype(np.float64).ravel()
    return np.corrcoef(a, b)[0, 1]


@pytest.mark.parametrize("K", [2, 3, 4])
def test_coupled_loop_closed_form(orc, K):
    """Eqs. (1)-(4) with K >= 2 on a noise-free integer shift k, starting
    from o = k except on two small patches (k + 2 and k - 2).

    The first pass is the plain K = 1 step, d^1 = 2 A(o) - A(A(o)) (A the
    masked box mean, here from scipy), which lies within 1 of k everywhere.
    A re-search of range 1 around d^1 then contains k, where the ZNCC is
    exactly 1 and every other candidate scores far lower, so every pixel
    takes o = k.  From then on Eq. (1) gives a = A(o) = k and Eqs. (2)-(3)
    reduce to d^j = alpha k + (1 - alpha) A(d^{j-1}).  An oracle whose
    Eq. (1) kept averaging the initial o, which re-searched around d^{j-1}
    (on a patch, k + 2 +- 1 does not contain k), or which skipped the
    re-search, ends elsewhere."""
    from scipy import ndimage  # noqa: F401  (used through _masked_mean)
    k, H, W, win, Rs, alpha, eta = 5, 48, 110, 7, 4, 0.1, 0.01
    h = win // 2
    L, R = _shift_pair(k, H, W, 23)
    m = np.zeros((H, W), np.uint8)
    m[6:H - 6, 12:W - 8] = 1
    o0 = np.where(m == 1, k, 0).astype(np.int32)
    o0[20:23, 40:43] = k + 2
    o0[30:32, 80:82] = k - 2
    v = m == 1
    d1 = 2 * _masked_mean(o0.astype(np.float64), m, Rs) - _masked_mean(
        np.where(v, _masked_mean(o0.astype(np.float64), m, Rs), 0.0), m, Rs)
    # premises: the first re-search window around d^1 holds k on every pixel,
    # and on the patches the window around the initial o does not
    assert np.abs(d1[v] - k).max() < 1.0
    assert np.abs(o0[20:23, 40:43] - k).min() == 2
    # premise: every wrong candidate near k scores far below the true shift
    for (y, x) in [(21, 41), (30, 80), (10, 20), (40, 100)]:
        for c in (k - 3, k - 2, k - 1, k + 1, k + 2, k + 3):
            assert _pearson(L, R, y, x, c, h) < 0.5
        assert _pearson(L, R, y, x, k, h) == pytest.approx(1.0, abs=1e-12)
    d = d1
    for _ in range(K - 1):
        d = alpha * k + (1 - alpha) * _masked_mean(np.where(v, d, 0.0), m, Rs)
    got_d, got_o = orc.hc_research(L, R, 0, 20, win, o0, m, Rs, K, alpha, eta, 1)
    np.testing.assert_allclose(got_d[v], d[v], rtol=0, atol=1e-12)
    assert np.isnan(got_d[~v]).all()
    assert (got_o[v] == k).all()
    assert np.array_equal(got_o[~v], o0[~v])


def test_no_candidate_keeps_o(orc):
    """A pixel whose re-search window holds no candidate with a defined ZNCC
    keeps its disparity: range 0 around a non-integer d is empty."""
    p = synth.make_pair(30, 80, 15, 4)
    m = np.ones((30, 80), np.uint8)
    o0 = np.full((30, 80), 6, np.int32)
    d = np.full((30, 80), 7.5)
    o = orc.research(p["left"], p["right"], 0, 15, 5, o0, m, d, 0, 0.01)
    assert (o == 6).all()


def test_resume_from_a_state(orc):
    """d_init resumes the loop from a state (o, d): one iteration gives
    d = a - A(a - alpha o - (1 - alpha) d_init), a = A(o) (Eqs. (1)-(3) by
    hand with scipy box means), and no re-search runs (K = 1)."""
    p = synth.make_pair(40, 90, 31, 12)
    r = np.random.default_rng(5)
    o = r.integers(5, 25, size=(40, 90)).astype(np.int32)
    m = (r.random((40, 90)) > 0.25).astype(np.uint8)
    d0 = o + r.uniform(-1.5, 1.5, size=(40, 90))
    Rs, alpha = 3, 0.1
    v = m == 1
    a = _masked_mean(o.astype(np.float64), m, Rs)
    b = a - alpha * o - (1 - alpha) * d0
    want = a - _masked_mean(np.where(v, b, 0.0), m, Rs)
    got, oo = orc.hc_research(p["left"], p["right"], 0, 31, 7, o, m, Rs, 1, alpha, 0.01, 5,
                              d_init=d0)
    np.testing.assert_allclose(got[v], want[v], rtol=0, atol=1e-11)
    assert np.array_equal(oo, o)
