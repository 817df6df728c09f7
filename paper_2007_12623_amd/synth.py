"""Seeded synthetic stereo inputs shaped like the paper's laparoscopy video.

This module only draws inputs: textures, a known disparity field and the
right image warped from the left one.  It holds none of the matching method's
arithmetic, so the CPU oracle and the HIP path can both be fed from it.

The paper measures on 960x540 stereo laparoscope video with candidate
disparities -20..80 (Section IV-A) and on 320x240 Hamlyn frames (Table I);
those recordings are not available, so seeded synthetic pairs of the same
shapes stand in for them.

Recipe (all draws from ``numpy.random.default_rng(seed)``):

* texture: for sigma in (1, 4, 16) a uniform [0,1) field is blurred with a
  separable Gaussian (truncate 4 sigma, reflect border) and standardised; the
  three fields are summed, min-max scaled to [0, 255] and rounded half to
  even.  The canvas is padded by ``PAD`` pixels on every side (and by the
  disparity range on the right) so that per-frame shifts and the warp stay
  inside it;
* two non-overlapping 40x40 low-texture patches: the patch mean rounded to an
  integer plus uniform integer noise in {-2..2}, clipped to [0, 255];
* disparity field on the right-image grid: two slanted planes split by a
  vertical seam at 40-60 % of the width (slopes |a|, |b| <= 0.03 px/px) plus a
  spherical bump of radius 0.15*min(W, H) and height 0.2*range, mapped
  affinely onto [1, dmax-2] so that both parabola neighbours exist;
* right image: R(xr, y) = round_half_even(clip(lerp_x(L, xr + D(xr, y))
  + N(0, 2^2), 0, 255));
* left ground truth by fixed-point inversion x = xr + D(xr) (20 iterations);
  unconverged pixels and pixels whose source falls outside the image have no
  ground truth (NaN);
* sequences: frame f shifts texture and field by a cumulative integer
  translation whose per-frame increments are uniform in {-4..4}^2.
"""
from __future__ import annotations

import numpy as np
from scipy.ndimage import gaussian_filter

PAD = 128
SIGMAS = (1.0, 4.0, 16.0)
NOISE_STD = 2.0
PATCH = 40

# Seeds of the five standard workloads.
SEED_C1 = 1001
SEED_C2 = 2002
SEED_C3 = 3003
SEED_C4 = 4004
SEED_C5 = 5005
SEED_PAPER = 6006

C4_SHAPES = ((240, 320), (480, 640), (540, 960), (720, 1280))  # (H, W)


def _texture_canvas(rng: np.random.Generator, Hc: int, Wc: int) -> np.ndarray:
    acc = np.zeros((Hc, Wc), dtype=np.float64)
    for s in SIGMAS:
        u = rng.random((Hc, Wc))
        b = gaussian_filter(u, sigma=s, mode="reflect", truncate=4.0)
        b = (b - b.mean()) / b.std()
        acc += b
    acc = (acc - acc.min()) / (acc.max() - acc.min()) * 255.0
    return np.rint(acc)  # numpy rint rounds half to even


def _flat_patches(rng, canvas, H, W, oy, ox):
    """Two non-overlapping low-texture patches (40x40, or a quarter of the
    smaller image side for images under 80 px) inside the image window whose
    top-left canvas corner is (oy, ox)."""
    ps = PATCH if min(H, W) >= 2 * PATCH else max(2, min(H, W) // 4)
    placed = []
    tries = 0
    while len(placed) < 2 and tries < 1000:
        tries += 1
        py = int(rng.integers(0, H - ps + 1))
        px = int(rng.integers(0, W - ps + 1))
        if any(abs(py - qy) < ps and abs(px - qx) < ps for qy, qx in placed):
            continue
        placed.append((py, px))
    for py, px in placed:
        sl = (slice(oy + py, oy + py + ps), slice(ox + px, ox + px + ps))
        m = np.rint(canvas[sl].mean())
        noise = rng.integers(-2, 3, size=(ps, ps))
        canvas[sl] = np.clip(m + noise, 0, 255)
    return placed


def _disparity_field(rng, Hc, Wc, H, W, dmax, oy, ox, dmin=0):
    """Field over the whole canvas; image pixel (x, y) sits at (ox+x, oy+y)."""
    yy, xx = np.mgrid[0:Hc, 0:Wc].astype(np.float64)
    xi = xx - ox
    yi = yy - oy
    seam = W * rng.uniform(0.4, 0.6)
    a1, b1, a2, b2 = rng.uniform(-0.03, 0.03, size=4)
    c1, c2 = rng.uniform(0.0, 1.0, size=2) * 0.3 * dmax
    f = np.where(xi < seam, a1 * xi + b1 * yi + c1, a2 * xi + b2 * yi + c2)
    rho = 0.15 * min(W, H)
    cy = rng.uniform(0.3, 0.7) * H
    cx = rng.uniform(0.3, 0.7) * W
    r2 = (xi - cx) ** 2 + (yi - cy) ** 2
    f = f + 0.2 * dmax * np.sqrt(np.maximum(0.0, 1.0 - r2 / rho**2))
    # affine map so that the image window spans [dmin+1, dmax-2]
    win = f[oy:oy + H, ox:ox + W]
    lo, hi = win.min(), win.max()
    span = max(hi - lo, 1e-9)
    d = (dmin + 1.0) + (f - lo) / span * (dmax - dmin - 3.0)
    return np.clip(d, dmin + 1.0, dmax - 2.0)


def _lerp_rows(rows: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Linear interpolation of each row of ``rows`` at fractional columns u."""
    W = rows.shape[1]
    u = np.clip(u, 0.0, W - 1.0)
    i0 = np.floor(u).astype(np.int64)
    i0 = np.minimum(i0, W - 2)
    t = u - i0
    r = np.arange(rows.shape[0])[:, None]
    return rows[r, i0] * (1.0 - t) + rows[r, i0 + 1] * t


class Scene:
    """A seeded texture canvas plus disparity field; frames are crops."""

    def __init__(self, H: int, W: int, dmax: int, seed: int, dmin: int = 0):
        assert -PAD < dmin < dmax
        self.H, self.W, self.dmax, self.dmin, self.seed = H, W, dmax, dmin, seed
        self.rng = np.random.default_rng(seed)
        self.Hc = H + 2 * PAD
        self.Wc = W + 2 * PAD + dmax + 2
        self.oy = PAD
        self.ox = PAD
        canvas = _texture_canvas(self.rng, self.Hc, self.Wc)
        self.patches = _flat_patches(self.rng, canvas, H, W, self.oy, self.ox)
        self.canvas = canvas
        self.field = _disparity_field(self.rng, self.Hc, self.Wc, H, W, dmax,
                                      self.oy, self.ox, dmin)

    def frame(self, ty: int = 0, tx: int = 0, noise_rng=None):
        """Left/right uint8 images and ground truth for a shift (ty, tx)."""
        H, W = self.H, self.W
        rng = noise_rng if noise_rng is not None else self.rng
        y0, x0 = self.oy + ty, self.ox + tx
        rows = self.canvas[y0:y0 + H, :]
        left = self.canvas[y0:y0 + H, x0:x0 + W].astype(np.uint8)
        d_right = self.field[y0:y0 + H, x0:x0 + W].copy()
        xr = np.arange(W, dtype=np.float64)[None, :]
        src = x0 + xr + d_right
        val = _lerp_rows(rows, src) + rng.normal(0.0, NOISE_STD, size=(H, W))
        right = np.rint(np.clip(val, 0.0, 255.0)).astype(np.uint8)
        gt_right = np.where(xr + d_right <= W - 1, d_right, np.nan)
        # left ground truth: x = xr + D(xr)  =>  xr = x - D(xr)
        fld = self.field[y0:y0 + H, :]
        x = np.arange(W, dtype=np.float64)[None, :].repeat(H, 0)
        guess = x - fld[:, x0:x0 + W]
        for _ in range(20):
            guess = x - _lerp_rows(fld, x0 + guess)
        resid = guess + _lerp_rows(fld, x0 + guess) - x
        ok = (np.abs(resid) < 1e-3) & (guess >= 0.0) & (guess <= W - 1.0)
        gt_left = np.where(ok, x - guess, np.nan)
        return {"left": np.ascontiguousarray(left),
                "right": np.ascontiguousarray(right),
                "gt_right": gt_right, "gt_left": gt_left}


def make_pair(H: int, W: int, dmax: int, seed: int, dmin: int = 0):
    """One seeded pair (frame 0 of a scene); disparities in [dmin+1, dmax-2]."""
    return Scene(H, W, dmax, seed, dmin).frame(0, 0)


def make_sequence(H: int, W: int, dmax: int, seed: int, n_frames: int):
    """n_frames pairs of one scene under a cumulative random integer drift."""
    sc = Scene(H, W, dmax, seed)
    rng = np.random.default_rng(seed + 7919)
    ty = tx = 0
    out = []
    for f in range(n_frames):
        if f > 0:
            dy, dx = rng.integers(-4, 5, size=2)
            ty = int(np.clip(ty + dy, -PAD + 4, PAD - 4))
            tx = int(np.clip(tx + dx, -PAD + 4, PAD - 4))
        fr = sc.frame(ty, tx, noise_rng=rng)
        fr["shift"] = (ty, tx)
        out.append(fr)
    return out


def c1_pair():
    """320x240, disparities 0..31, 7x7 window."""
    return make_pair(240, 320, 31, SEED_C1)


def c2_sequence(n_frames: int = 30):
    """960x540, disparities 0..127, 11x11 window, drifting sequence."""
    return make_sequence(540, 960, 127, SEED_C2, n_frames)


def c5_sequence(n_frames: int = 30):
    """1920x1080, disparities 0..255, 15x15 window, drifting sequence."""
    return make_sequence(1080, 1920, 255, SEED_C5, n_frames)


def paper_pair():
    """960x540 with the paper's candidate range -20..80 (101 values), 11x11
    window (Section IV's recordings; Section II-A's window)."""
    return make_pair(540, 960, 80, SEED_PAPER, dmin=-20)


def c4_layout(seed: int = SEED_C4, n_pairs: int = 64):
    """Shapes, disparity counts and windows of the uneven batch."""
    rng = np.random.default_rng(seed)
    lay = []
    for _ in range(n_pairs):
        H, W = C4_SHAPES[int(rng.integers(0, len(C4_SHAPES)))]
        D = int(rng.integers(32, 193))
        win = int((7, 11)[int(rng.integers(0, 2))])
        lay.append({"H": H, "W": W, "dmin": 0, "dmax": D - 1, "win": win})
    return lay


def c4_batch(seed: int = SEED_C4, n_pairs: int = 64):
    """64 pairs of seeded random shapes, disparity ranges and windows."""
    lay = c4_layout(seed, n_pairs)
    out = []
    for i, p in enumerate(lay):
        fr = make_pair(p["H"], p["W"], p["dmax"], seed * 1000 + i)
        fr.update(p)
        out.append(fr)
    return out
