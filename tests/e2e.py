"""Whole-path checks shared by the GPU tests (no arithmetic of the method:
every expected value comes from the oracle).

stagewise(): each oracle stage runs on the GPU's own input to that stage and
must give the GPU's output - masks and integer maps bit-exact, smoothed
disparities within max(1e-5, 1 ulp) - so that a matcher near-tie, where two
candidates are equal up to rounding, cannot spread through the later stages
unseen.

against_pipeline(): the GPU's final output against the oracle's pipeline run
from the images.  Where matching has a near-tie (an oracle top-2 gap at or
below the bar) either winner is correct, and the later stages carry the
difference only so far: the left-right check reads the right-reference map
up to the disparity range away, each alternation reads up to its outlier
radius plus both fill radii, and the smoothing R per box pass.  Outside the
near-tie pixels dilated by that reach the two outputs must agree exactly
(masks) and within the smoothing bar (disparities)."""
import numpy as np

from gpu_util import cu, dilate, np_, tie_mask


def run_debug(B, L, R, dmin, dmax, win, params, handle=None):
    """stereo_match with debug_outputs = 1; returns the output and every
    intermediate as numpy arrays."""
    import torch
    H, W = L.shape
    h = handle or B.Handle(0)
    try:
        params.debug_outputs = 1
        disp, mask = B.stereo_match(cu(L), cu(R), dmin, dmax, win, params, handle=h)
        out = {"disp": np_(disp), "mask": np_(mask)}

        def get(name, dt):
            return np_(B.stereo_debug_get(name, (H, W), dt, handle=h))
        out["o_wta"] = get("o_wta", torch.int16).astype(np.int32)
        out["m_wta"] = get("m_wta", torch.uint8)
        out["o_r"] = get("o_r", torch.int16).astype(np.int32)
        out["m_r"] = get("m_r", torch.uint8)
        out["delta"] = get("delta", torch.float32).astype(np.float64)
        out["zbest"] = get("zbest", torch.float64)
        out["m_lr"] = get("m_lr", torch.uint8)
        out["o_post"] = get("o_post", torch.int16).astype(np.int32)
        out["m_post"] = get("m_post", torch.uint8)
    finally:
        if handle is None:
            h.close()
    return out


def smooth_bar(ref):
    return np.maximum(1e-5, np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64))


def stagewise(orc, L, R, dmin, dmax, win, g, po, ref, tie_bar=1e-5):
    """Stage-by-stage parity of one debug run `g` (see run_debug) with the
    oracle; `ref` is orc.match of the same pair.  Returns the error report
    of the matching stage (counts and maxima against the oracle)."""
    chess = bool(po.chess)
    rep = {}
    # matching: validity exact, winners exact away from near-ties
    assert np.array_equal(g["m_wta"], ref["mL"]), "left validity"
    assert np.array_equal(g["m_r"], ref["mR"]), "right validity"
    vl, vr = ref["mL"] == 1, ref["mR"] == 1
    sel = vl & ~tie_mask(ref["gap"], tie_bar)
    selr = vr & ~tie_mask(ref["gapR"], tie_bar)
    bad = int((g["o_wta"][sel] != ref["oL"][sel]).sum())
    badr = int((g["o_r"][selr] != ref["oR"][selr]).sum())
    assert bad == 0, f"{bad} left disparities differ beyond the tie bar {tie_bar}"
    assert badr == 0, f"{badr} right disparities differ beyond the tie bar {tie_bar}"
    dis = vl & (g["o_wta"] != ref["oL"])
    disr = vr & (g["o_r"] != ref["oR"])
    rep["valid_px"] = int(vl.sum())
    rep["int_disagree_px"] = int(dis.sum())
    rep["int_disagree_frac"] = float(dis.sum() / max(1, vl.sum()))
    rep["int_disagree_above_bar_px"] = bad
    rep["right_int_disagree_px"] = int(disr.sum())
    agree = vl & ~dis
    dl = g["delta"]
    if po.subpixel:
        # the exact z at the GPU's winner (computed by the sub-pixel step):
        # equal to the oracle's where the winners agree, and below it by less
        # than the tie bar where they do not
        dz = np.abs(g["zbest"][vl] - ref["zbest"][vl])
        np.testing.assert_allclose(g["zbest"][agree], ref["zbest"][agree], rtol=0, atol=1e-12)
        assert (dz <= tie_bar + 1e-12).all()
        rep["max_abs_dz"] = float(dz.max()) if dz.size else 0.0
        rep["mean_abs_dz"] = float(dz.mean()) if dz.size else 0.0
        # sub-pixel offsets where the winners agree
        dref = orc.subpixel(ref["oL"], ref["mL"], ref["zm"], ref["zbest"], ref["zp"], dmin, dmax)
        dd = np.abs(dl[agree] - dref[agree])
        assert dd.size == 0 or dd.max() <= 1e-5
        rep["max_abs_ddelta"] = float(dd.max()) if dd.size else 0.0
    else:
        dl = np.zeros_like(dl)
    # left-right check on the GPU's two winner maps
    mlr_ref = orc.lr_check(g["o_wta"], g["m_wta"], g["o_r"], g["m_r"], po.lr_tol) \
        if po.lr_check else g["m_wta"]
    assert np.array_equal(g["m_lr"], mlr_ref), "left-right mask"
    # outlier removal / hole filling alternations from the GPU's checked map
    o, m = g["o_wta"].copy(), g["m_lr"].copy()
    fill = dict(radial_r=po.fill_radial_r, min_lines=po.fill_min_lines, disk_r=po.fill_disk_r,
                min_frac=float(np.float32(po.fill_disk_frac)))
    if po.radial_iters <= 0:
        o, m = orc.fill(o, m, **fill)
    for it in range(po.radial_iters):
        m = orc.radial_outlier(o, m, po.radial_r0 + it * po.radial_dr, po.radial_thresh)
        o, m = orc.fill(o, m, **fill)
    assert np.array_equal(g["m_post"], m), f"masks differ on {(g['m_post'] != m).sum()} px"
    assert np.array_equal(g["o_post"][m > 0], o[m > 0])
    # smoothing of o + delta (research runs are checked by their own test)
    if not po.research:
        s = np.where(m == 1, o + dl, o.astype(np.float64))
        if po.smooth_iters > 0:
            dref = orc.hc_smooth(s, m, po.smooth_radius, po.smooth_iters,
                                 float(np.float32(po.smooth_alpha)))
        else:
            dref = np.where(m > 0, s, np.nan)
        assert np.array_equal(g["mask"], m)
        v = m > 0
        assert np.isnan(g["disp"][~v]).all()
        err = np.abs(g["disp"][v] - dref[v])
        nbad = int((err > smooth_bar(dref[v])).sum())
        assert nbad == 0, f"{nbad} disparities differ, max {err.max():.3g}"
    return rep


def reach(po, dmin, dmax, win):
    """How far a changed matching decision can move later outputs (pixels)."""
    r = (dmax - dmin + 1) + po.lr_tol + win
    if po.radial_iters <= 0:
        r += po.fill_radial_r + po.fill_disk_r
    for it in range(po.radial_iters):
        r += po.radial_r0 + it * po.radial_dr + po.fill_radial_r + po.fill_disk_r
    r += po.smooth_radius * (po.smooth_iters + 1)
    if po.research:
        r += (po.research_range + win) * po.smooth_iters
    return r


def against_pipeline(orc, L, R, dmin, dmax, win, disp, mask, po, ref, rref=None, tie_bar=1e-5):
    """Final GPU output against the oracle's pipeline from the images (see
    the module docstring).  `ref` is orc.match of the pair (for the gaps),
    `rref` the oracle pipeline's (disp, mask) if already computed.  Returns
    (pixels compared, pixels excluded as near-tie reach)."""
    rdisp, rmask = rref if rref is not None else orc.pipeline(L, R, dmin, dmax, win, po)
    seed = (ref["mL"] == 1) & tie_mask(ref["gap"], tie_bar)
    tr = (ref["mR"] == 1) & tie_mask(ref["gapR"], tie_bar)
    if tr.any():
        # a right-reference tie at xr reaches the left pixels xr + dmin .. xr + dmax
        ys, xs = np.nonzero(tr)
        for d in range(dmin, dmax + 1):
            xx = xs + d
            ok = (xx >= 0) & (xx < L.shape[1])
            seed[ys[ok], xx[ok]] = True
    excl = dilate(seed, reach(po, dmin, dmax, win)) if seed.any() else np.zeros_like(seed)
    keep = ~excl
    nm = int((mask[keep] != rmask[keep]).sum())
    assert nm == 0, f"final masks differ on {nm} px outside the near-tie reach"
    v = keep & (rmask > 0)
    assert np.isnan(disp[keep & (rmask == 0)]).all()
    err = np.abs(disp[v] - rdisp[v])
    nbad = int((err > smooth_bar(rdisp[v])).sum())
    assert nbad == 0, f"{nbad} final disparities differ outside the near-tie reach, max {err.max():.3g}"
    return int(keep.sum()), int(excl.sum())


def match_banded(orc, L, R, dmin, dmax, win, rows=64, chess=False):
    """orc.match over row bands (bounded memory for the full cost volume),
    concatenated."""
    H = L.shape[0]
    parts = [orc.match(L, R, dmin, dmax, win, rows=(y, min(y + rows, H)), chess=chess)
             for y in range(0, H, rows)]
    return {k: np.concatenate([p[k] for p in parts], axis=0) for k in parts[0]}
