/*
 * CPU oracle for the dense ZNCC stereo path of Zhou & Jagadeesan,
 * "Real-time Dense Reconstruction of Tissue Surface from Stereo Optical
 * Video" (arXiv 2007.12623).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code with the HIP library.
 *
 * Plain and slow on purpose: FP64 for real numbers, int64 for integer sums,
 * row-major loops, a full cost volume, Jacobi updates.  Each function names
 * the passage of the paper it follows.  Choices the paper leaves open are
 * fixed as follows (the same readings are listed in the design notes):
 *   - left pixel x at disparity d matches right pixel x - d; d may be negative;
 *   - a candidate is valid only if both windows lie inside the image and both
 *     have non-zero variance; there is no border padding;
 *   - exact WTA ties go to the smallest disparity (left and right reference);
 *   - the sub-pixel offset is a 3-point parabola on z, clamped to +-1/2;
 *   - the radial outlier test walks the full radius, needs every step inside
 *     the image and valid, and compares consecutive disparities with a strict
 *     "< threshold";
 *   - the radial fill needs >= min_lines complete lines (a line is a pair of
 *     opposite directions that both hit), the disk fill >= ceil(frac*cells)
 *     valid cells; fill values are exact rationals rounded half to even;
 *   - improved Laplacian smoothing averages over valid pixels of a square
 *     (2R+1)^2 window including the centre.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL -1
#define OR_ENOMEM -2

static inline int64_t ii_at(const int64_t *ii, int Wp1, int y, int x) {
  return ii[(int64_t)y * Wp1 + x];
}

/* int64 integral image of f over an H x W grid: ii[(y+1)*(W+1)+(x+1)] =
 * sum_{y'<=y, x'<=x} f(y', x'). */
static void integral(const int64_t *f, int H, int W, int64_t *ii) {
  int Wp1 = W + 1;
  memset(ii, 0, sizeof(int64_t) * (size_t)Wp1);
  for (int y = 0; y < H; ++y) {
    int64_t row = 0;
    ii[(int64_t)(y + 1) * Wp1] = 0;
    for (int x = 0; x < W; ++x) {
      row += f[(int64_t)y * W + x];
      ii[(int64_t)(y + 1) * Wp1 + x + 1] = ii[(int64_t)y * Wp1 + x + 1] + row;
    }
  }
}

/* Sum of f over the square window of half-size h centred on (x, y); the
 * window must lie inside the grid. */
static int64_t box(const int64_t *ii, int W, int y, int x, int h) {
  int Wp1 = W + 1;
  return ii_at(ii, Wp1, y + h + 1, x + h + 1) - ii_at(ii, Wp1, y - h, x + h + 1) -
         ii_at(ii, Wp1, y + h + 1, x - h) + ii_at(ii, Wp1, y - h, x - h);
}

static int inside(int H, int W, int h, int y, int x) {
  return y >= h && y <= H - 1 - h && x >= h && x <= W - 1 - h;
}

/*
 * Window statistics (Section II-A: ZNCC over a square window, 11x11 in the
 * paper).  For every pixel whose window lies inside the image:
 *   S = sum I, SS = sum I^2, varN = n*SS - S^2 (n = win^2), exactly.
 * brute != 0 sums the window directly instead of through integral images.
 * chess != 0: the chessboard window of the paper's matching (every other
 * pixel): only offsets (u, v) from the centre with u + v even, n =
 * (win^2 + 1) / 2, summed directly.
 */
int or_window_stats(const uint8_t *img, int H, int W, int pitch, int win, int brute, int chess,
                    int64_t *S, int64_t *SS, int64_t *varN, uint8_t *ins) {
  if (win < 1 || (win & 1) == 0 || H < 1 || W < 1 || pitch < W) return OR_EINVAL;
  int h = win / 2;
  int64_t n = chess ? ((int64_t)win * win + 1) / 2 : (int64_t)win * win;
  if (chess) brute = 1;
  int64_t *f1 = NULL, *f2 = NULL, *i1 = NULL, *i2 = NULL;
  if (!brute) {
    f1 = malloc(sizeof(int64_t) * (size_t)H * W);
    f2 = malloc(sizeof(int64_t) * (size_t)H * W);
    i1 = malloc(sizeof(int64_t) * (size_t)(H + 1) * (W + 1));
    i2 = malloc(sizeof(int64_t) * (size_t)(H + 1) * (W + 1));
    if (!f1 || !f2 || !i1 || !i2) { free(f1); free(f2); free(i1); free(i2); return OR_ENOMEM; }
    for (int y = 0; y < H; ++y)
      for (int x = 0; x < W; ++x) {
        int64_t v = img[(int64_t)y * pitch + x];
        f1[(int64_t)y * W + x] = v;
        f2[(int64_t)y * W + x] = v * v;
      }
    integral(f1, H, W, i1);
    integral(f2, H, W, i2);
  }
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      int64_t k = (int64_t)y * W + x;
      if (!inside(H, W, h, y, x)) {
        S[k] = SS[k] = varN[k] = 0; ins[k] = 0; continue;
      }
      int64_t s = 0, ss = 0;
      if (brute) {
        for (int v = -h; v <= h; ++v)
          for (int u = -h; u <= h; ++u) {
            if (chess && ((u + v) & 1)) continue;
            int64_t p = img[(int64_t)(y + v) * pitch + x + u];
            s += p; ss += p * p;
          }
      } else {
        s = box(i1, W, y, x, h);
        ss = box(i2, W, y, x, h);
      }
      S[k] = s; SS[k] = ss; varN[k] = n * ss - s * s; ins[k] = 1;
    }
  free(f1); free(f2); free(i1); free(i2);
  return OR_OK;
}

/*
 * Zero-mean normalised cross-correlation of two windows of n samples, as
 * textbook definition (Section I-A cites it for its robustness to
 * illumination; Section II-A uses it as the matching cost): the covariance of
 * the mean-subtracted windows over the product of their norms.  NaN when a
 * window has zero variance.
 */
double or_zncc_windows(const uint8_t *a, const uint8_t *b, int n) {
  double ma = 0, mb = 0;
  for (int i = 0; i < n; ++i) { ma += a[i]; mb += b[i]; }
  ma /= n; mb /= n;
  double sab = 0, saa = 0, sbb = 0;
  for (int i = 0; i < n; ++i) {
    double da = a[i] - ma, db = b[i] - mb;
    sab += da * db; saa += da * da; sbb += db * db;
  }
  if (saa == 0.0 || sbb == 0.0) return NAN;
  return sab / sqrt(saa * sbb);
}

/*
 * Dense ZNCC matching by brute force over every candidate disparity
 * (Section II-A: every pixel tests every candidate), followed by
 * winner-take-all in the left and the right reference.
 *
 * For rows y in [y0, y1) (outputs are (y1-y0) x W, row-major):
 *   z(x,y,d) = (n*S_LR - S_L*S_R) / sqrt(varN_L * varN_R)
 * with S_LR = sum_W L(x+u,y+v) R(x+u-d,y+v) in int64 (integral image of the
 * product per d, or direct loops when brute != 0).  The whole cost volume is
 * kept in memory.  chess != 0: the window is the chessboard of the paper's
 * matching (Section II-A: every other pixel of the window), the cells with
 * u + v even, and n = (win^2 + 1) / 2; the sums then come from integral
 * images of the product masked to one checker colour, picked by the colour
 * of the centre (x + y).
 *   oL, mL      : argmax_d z (ties -> smallest d), mask 1 if any valid d
 *   zbest, gap  : best z and best - (max over other valid d) (inf if none)
 *   zm, zp      : z at oL-1 and oL+1 (NaN if out of range or invalid)
 *   oR, mR, ... : for right pixel xr, argmax_d z(xr+d, y, d)
 */
int or_match(const uint8_t *L, const uint8_t *R, int H, int W, int pitch, int dmin, int dmax,
             int win, int y0, int y1, int brute, int chess,
             int32_t *oL, uint8_t *mL, double *zbest, double *gap, double *zm, double *zp,
             int32_t *oR, uint8_t *mR, double *zbestR, double *gapR) {
  if (win < 1 || (win & 1) == 0 || dmax < dmin || y0 < 0 || y1 > H || y1 < y0 || pitch < W)
    return OR_EINVAL;
  int h = win / 2;
  int64_t n = chess ? ((int64_t)win * win + 1) / 2 : (int64_t)win * win;
  int D = dmax - dmin + 1;
  int rows = y1 - y0;
  size_t plane = (size_t)rows * W;
  int64_t *SL = malloc(sizeof(int64_t) * (size_t)H * W), *SSL = malloc(sizeof(int64_t) * (size_t)H * W);
  int64_t *VL = malloc(sizeof(int64_t) * (size_t)H * W), *SR = malloc(sizeof(int64_t) * (size_t)H * W);
  int64_t *SSR = malloc(sizeof(int64_t) * (size_t)H * W), *VR = malloc(sizeof(int64_t) * (size_t)H * W);
  uint8_t *IL = malloc((size_t)H * W), *IR = malloc((size_t)H * W);
  double *vol = malloc(sizeof(double) * plane * (size_t)D);
  if (!SL || !SSL || !VL || !SR || !SSR || !VR || !IL || !IR || !vol) {
    free(SL); free(SSL); free(VL); free(SR); free(SSR); free(VR); free(IL); free(IR); free(vol);
    return OR_ENOMEM;
  }
  or_window_stats(L, H, W, pitch, win, brute, chess, SL, SSL, VL, IL);
  or_window_stats(R, H, W, pitch, win, brute, chess, SR, SSR, VR, IR);

  /* rows of the product image needed: [y0-h, y1+h) clipped to the image */
  int py0 = y0 - h < 0 ? 0 : y0 - h;
  int py1 = y1 + h > H ? H : y1 + h;
  int PH = py1 - py0;

#pragma omp parallel
  {
    int64_t *prod = brute ? NULL : malloc(sizeof(int64_t) * (size_t)(PH > 0 ? PH : 1) * W);
    int64_t *ii = brute ? NULL : malloc(sizeof(int64_t) * (size_t)(PH + 1) * (W + 1));
    int64_t *ii1 = (brute || !chess) ? NULL : malloc(sizeof(int64_t) * (size_t)(PH + 1) * (W + 1));
#pragma omp for schedule(dynamic)
    for (int di = 0; di < D; ++di) {
      int d = dmin + di;
      if (!brute) {
        /* colour c of the chessboard: pass 0 keeps (x + y) even cells, pass 1 odd */
        for (int pass = 0; pass < (chess ? 2 : 1); ++pass) {
          for (int y = py0; y < py1; ++y)
            for (int x = 0; x < W; ++x) {
              int xr = x - d;
              int64_t v = 0;
              if (xr >= 0 && xr < W && (!chess || ((x + y) & 1) == pass))
                v = (int64_t)L[(int64_t)y * pitch + x] * (int64_t)R[(int64_t)y * pitch + xr];
              prod[(int64_t)(y - py0) * W + x] = v;
            }
          integral(prod, PH, W, pass ? ii1 : ii);
        }
      }
      double *zd = vol + plane * (size_t)di;
      for (int y = y0; y < y1; ++y)
        for (int x = 0; x < W; ++x) {
          double z = NAN;
          int xr = x - d;
          int64_t kl = (int64_t)y * W + x, kr = (int64_t)y * W + xr;
          if (inside(H, W, h, y, x) && xr >= h && xr <= W - 1 - h && VL[kl] > 0 && VR[kr] > 0) {
            int64_t slr = 0;
            if (brute) {
              for (int v = -h; v <= h; ++v)
                for (int u = -h; u <= h; ++u) {
                  if (chess && ((u + v) & 1)) continue;
                  slr += (int64_t)L[(int64_t)(y + v) * pitch + x + u] *
                         (int64_t)R[(int64_t)(y + v) * pitch + x + u - d];
                }
            } else {
              slr = box(chess && ((x + y) & 1) ? ii1 : ii, W, y - py0, x, h);
            }
            int64_t num = n * slr - SL[kl] * SR[kr];
            z = (double)num / sqrt((double)VL[kl] * (double)VR[kr]);
          }
          zd[(size_t)(y - y0) * W + x] = z;
        }
    }
    free(prod); free(ii); free(ii1);
  }

  /* left reference WTA */
#pragma omp parallel for
  for (int y = y0; y < y1; ++y)
    for (int x = 0; x < W; ++x) {
      size_t k = (size_t)(y - y0) * W + x;
      int best = -1; double bz = -INFINITY;
      for (int di = 0; di < D; ++di) {
        double z = vol[plane * di + k];
        if (!isnan(z) && z > bz) { bz = z; best = di; }
      }
      if (best < 0) {
        oL[k] = 0; mL[k] = 0; zbest[k] = NAN; gap[k] = NAN; zm[k] = NAN; zp[k] = NAN;
        continue;
      }
      double second = -INFINITY;
      for (int di = 0; di < D; ++di) {
        double z = vol[plane * di + k];
        if (di != best && !isnan(z) && z > second) second = z;
      }
      oL[k] = dmin + best; mL[k] = 1; zbest[k] = bz;
      gap[k] = isinf(second) ? INFINITY : bz - second;
      zm[k] = best > 0 ? vol[plane * (best - 1) + k] : NAN;
      zp[k] = best < D - 1 ? vol[plane * (best + 1) + k] : NAN;
    }

  /* right reference WTA: right pixel xr takes candidates (xr + d, d) */
#pragma omp parallel for
  for (int y = y0; y < y1; ++y)
    for (int xr = 0; xr < W; ++xr) {
      size_t k = (size_t)(y - y0) * W + xr;
      int best = -1; double bz = -INFINITY;
      for (int di = 0; di < D; ++di) {
        int x = xr + dmin + di;
        if (x < 0 || x >= W) continue;
        double z = vol[plane * di + (size_t)(y - y0) * W + x];
        if (!isnan(z) && z > bz) { bz = z; best = di; }
      }
      if (best < 0) { oR[k] = 0; mR[k] = 0; zbestR[k] = NAN; gapR[k] = NAN; continue; }
      double second = -INFINITY;
      for (int di = 0; di < D; ++di) {
        int x = xr + dmin + di;
        if (x < 0 || x >= W || di == best) continue;
        double z = vol[plane * di + (size_t)(y - y0) * W + x];
        if (!isnan(z) && z > second) second = z;
      }
      oR[k] = dmin + best; mR[k] = 1; zbestR[k] = bz;
      gapR[k] = isinf(second) ? INFINITY : bz - second;
    }

  free(SL); free(SSL); free(VL); free(SR); free(SSR); free(VR); free(IL); free(IR); free(vol);
  return OR_OK;
}

/*
 * Sub-pixel offset of the WTA disparity by a 3-point parabola through
 * (o-1, zm), (o, z0), (o+1, zp).  The paper obtains continuous disparities
 * only from its refinement (Section II-C); the parabola is the fit this path
 * adds.  delta = (zm - zp) / (2 (zm - 2 z0 + zp)), clamped to [-1/2, 1/2];
 * delta = 0 when o is at either end of the range, a neighbour is missing
 * (NaN), or the curvature term is >= 0.
 */
void or_subpixel(int64_t count, const int32_t *o, const uint8_t *m, const double *zm,
                 const double *z0, const double *zp, int dmin, int dmax, double *delta) {
  for (int64_t k = 0; k < count; ++k) {
    double dl = 0.0;
    if (m[k] && o[k] > dmin && o[k] < dmax && !isnan(zm[k]) && !isnan(zp[k])) {
      double den = 2.0 * (zm[k] - 2.0 * z0[k] + zp[k]);
      if (den < 0.0) {
        dl = (zm[k] - zp[k]) / den;
        if (dl > 0.5) dl = 0.5;
        if (dl < -0.5) dl = -0.5;
      }
    }
    delta[k] = dl;
  }
}

/*
 * Left-right consistency.  Section II-B treats a left pixel that cannot find
 * its corresponding right pixel as a hole; a pixel is kept when its match in
 * the right image points back to it:  xr = x - oL(x) in the image, oR(xr)
 * defined and |oL(x) - oR(xr)| <= tol.  Output mask 1 = kept, 0 = hole.
 */
void or_lr_check(int H, int W, const int32_t *oL, const uint8_t *mL, const int32_t *oR,
                 const uint8_t *mR, int tol, uint8_t *out) {
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      int64_t k = (int64_t)y * W + x;
      uint8_t keep = 0;
      if (mL[k]) {
        int xr = x - oL[k];
        if (xr >= 0 && xr < W) {
          int64_t kr = (int64_t)y * W + xr;
          if (mR[kr] && abs(oL[k] - oR[kr]) <= tol) keep = 1;
        }
      }
      out[k] = keep;
    }
}

static const int DIR8[8][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}, {1, 1}, {-1, -1}, {1, -1}, {-1, 1}};
/* DIR8[2i] and DIR8[2i+1] are opposite: the four lines of the radial fill. */

/*
 * Radial outlier removal (Section II-B): along each of the 8 radial
 * directions within radius r, neighbouring disparities must differ by less
 * than the threshold (2.5 in the paper); a pixel for which no direction
 * satisfies this is an outlier.  Jacobi: reads (o, m), writes mout.
 * Mask codes of kept pixels are preserved; removed pixels get 0.
 */
void or_radial_outlier(int H, int W, const int32_t *o, const uint8_t *m, int r, double thresh,
                       uint8_t *mout) {
#pragma omp parallel for
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      int64_t k = (int64_t)y * W + x;
      if (!m[k]) { mout[k] = 0; continue; }
      int any = 0;
      for (int dir = 0; dir < 8 && !any; ++dir) {
        int ux = DIR8[dir][0], uy = DIR8[dir][1];
        int pass = 1;
        for (int s = 1; s <= r; ++s) {
          int qx = x + s * ux, qy = y + s * uy;
          if (qx < 0 || qx >= W || qy < 0 || qy >= H) { pass = 0; break; }
          int64_t q = (int64_t)qy * W + qx;
          int64_t qp = (int64_t)(qy - uy) * W + (qx - ux);
          if (!m[q]) { pass = 0; break; }
          if (!(fabs((double)o[q] - (double)o[qp]) < thresh)) { pass = 0; break; }
        }
        any = pass;
      }
      mout[k] = any ? m[k] : 0;
    }
}

/* floor division and round-half-to-even of num/den (den > 0) */
static int64_t floordiv(int64_t a, int64_t b) {
  int64_t q = a / b, r = a % b;
  if (r != 0 && ((r < 0) != (b < 0))) --q;
  return q;
}
static int64_t round_half_even(int64_t num, int64_t den) {
  int64_t q = floordiv(num, den);
  int64_t r = num - q * den; /* 0 <= r < den */
  if (2 * r > den) return q + 1;
  if (2 * r == den) return (q & 1) ? q + 1 : q;
  return q;
}

/*
 * Hole filling (Section II-B), two methods applied in turn, each a Jacobi
 * step over the map it receives:
 *  (i) radial: search the 8 radial directions up to radial_r (50 px in the
 *      paper) for the first valid pixel; a line (two opposite directions)
 *      with both ends found gives (v_a s_b + v_b s_a) / (s_a + s_b); with at
 *      least min_lines complete lines the hole takes the mean of the line
 *      values;
 * (ii) disk: within radius disk_r (20 px in the paper), if the number of
 *      valid pixels is at least ceil(min_frac * in-image disk cells) the hole
 *      takes their mean.
 * Fill values are exact rationals rounded half to even.  Filled pixels get
 * mask code 2.  o and m are updated in place.
 */
int or_fill(int H, int W, int32_t *o, uint8_t *m, int radial_r, int min_lines, int disk_r,
            double min_frac) {
  int64_t N = (int64_t)H * W;
  int32_t *o1 = malloc(sizeof(int32_t) * (size_t)N);
  uint8_t *m1 = malloc((size_t)N);
  if (!o1 || !m1) { free(o1); free(m1); return OR_ENOMEM; }
  memcpy(o1, o, sizeof(int32_t) * (size_t)N);
  memcpy(m1, m, (size_t)N);
  /* (i) radial, reads (o, m), writes (o1, m1) */
#pragma omp parallel for
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      int64_t k = (int64_t)y * W + x;
      if (m[k]) continue;
      int64_t v[8], s[8];
      int hit[8];
      for (int dir = 0; dir < 8; ++dir) {
        hit[dir] = 0;
        for (int st = 1; st <= radial_r; ++st) {
          int qx = x + st * DIR8[dir][0], qy = y + st * DIR8[dir][1];
          if (qx < 0 || qx >= W || qy < 0 || qy >= H) break;
          int64_t q = (int64_t)qy * W + qx;
          if (m[q]) { hit[dir] = 1; v[dir] = o[q]; s[dir] = st; break; }
        }
      }
      int64_t num = 0, den = 1;
      int lines = 0;
      for (int l = 0; l < 4; ++l) {
        int a = 2 * l, b = 2 * l + 1;
        if (!(hit[a] && hit[b])) continue;
        int64_t ln = v[a] * s[b] + v[b] * s[a];
        int64_t ld = s[a] + s[b];
        num = num * ld + ln * den; /* num/den += ln/ld */
        den = den * ld;
        ++lines;
      }
      if (lines >= min_lines && lines > 0) {
        o1[k] = (int32_t)round_half_even(num, den * lines);
        m1[k] = 2;
      }
    }
  /* (ii) disk, reads (o1, m1), writes (o, m) */
  memcpy(o, o1, sizeof(int32_t) * (size_t)N);
  memcpy(m, m1, (size_t)N);
  int64_t R2 = (int64_t)disk_r * disk_r;
#pragma omp parallel for
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      int64_t k = (int64_t)y * W + x;
      if (m1[k]) continue;
      int64_t cells = 0, cnt = 0, sum = 0;
      for (int dy = -disk_r; dy <= disk_r; ++dy)
        for (int dx = -disk_r; dx <= disk_r; ++dx) {
          if ((int64_t)dx * dx + (int64_t)dy * dy > R2) continue;
          int qx = x + dx, qy = y + dy;
          if (qx < 0 || qx >= W || qy < 0 || qy >= H) continue;
          ++cells;
          int64_t q = (int64_t)qy * W + qx;
          if (m1[q]) { ++cnt; sum += o1[q]; }
        }
      double need = ceil(min_frac * (double)cells);
      if (cnt > 0 && (double)cnt >= need) {
        o[k] = (int32_t)round_half_even(sum, cnt);
        m[k] = 2;
      }
    }
  free(o1); free(m1);
  return OR_OK;
}

/* masked mean over the square window of half-size R, valid pixels only */
static void masked_mean(int H, int W, const double *f, const uint8_t *m, int R, double *out) {
#pragma omp parallel for
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      int64_t k = (int64_t)y * W + x;
      if (!m[k]) { out[k] = NAN; continue; }
      double s = 0.0;
      int64_t c = 0;
      for (int dy = -R; dy <= R; ++dy) {
        int qy = y + dy;
        if (qy < 0 || qy >= H) continue;
        for (int dx = -R; dx <= R; ++dx) {
          int qx = x + dx;
          if (qx < 0 || qx >= W) continue;
          int64_t q = (int64_t)qy * W + qx;
          if (m[q]) { s += f[q]; ++c; }
        }
      }
      out[k] = s / (double)c;
    }
}

/*
 * Improved Laplacian smoothing (Section II-C, Eqs. (1)-(3), after Vollmer):
 *   d^0 = s;  for k = 1..K:
 *     a   = average of s over the valid neighbours          (Eq. 1)
 *     b   = a - alpha*s - (1 - alpha)*d^{k-1}              (Eq. 2)
 *     d^k = a - average of b over the valid neighbours      (Eq. 3)
 * Eq. (1) averages the discrete disparities o; with the re-search of Eq. (4)
 * left out they stay fixed, so a is the same in every iteration and s (the
 * integer disparity plus its sub-pixel offset) plays the role of o.
 * Invalid pixels are NaN in the output.
 */
int or_hc_smooth(int H, int W, const double *s, const uint8_t *m, int R, int K, double alpha,
                 double *out) {
  int64_t N = (int64_t)H * W;
  double *a = malloc(sizeof(double) * (size_t)N), *b = malloc(sizeof(double) * (size_t)N);
  double *ab = malloc(sizeof(double) * (size_t)N), *dprev = malloc(sizeof(double) * (size_t)N);
  if (!a || !b || !ab || !dprev) { free(a); free(b); free(ab); free(dprev); return OR_ENOMEM; }
  for (int64_t k = 0; k < N; ++k) dprev[k] = m[k] ? s[k] : NAN;
  masked_mean(H, W, s, m, R, a);
  for (int it = 0; it < K; ++it) {
    for (int64_t k = 0; k < N; ++k)
      b[k] = m[k] ? a[k] - alpha * s[k] - (1.0 - alpha) * dprev[k] : 0.0;
    masked_mean(H, W, b, m, R, ab);
    for (int64_t k = 0; k < N; ++k) dprev[k] = m[k] ? a[k] - ab[k] : NAN;
  }
  memcpy(out, dprev, sizeof(double) * (size_t)N);
  free(a); free(b); free(ab); free(dprev);
  return OR_OK;
}

/*
 * Exact ZNCC of the left window at (x, y) and the right window at (x - d, y)
 * by direct sums (Section II-A): (n*S_LR - S_L*S_R) / sqrt(varN_L * varN_R)
 * with int64 sums (chess: the chessboard cells u + v even, n = (win^2+1)/2).
 * Returns NAN when either window leaves the image or has zero variance (the
 * candidate is not valid).
 */
static double zncc_at(const uint8_t *L, const uint8_t *R, int H, int W, int pitch, int win,
                      int chess, int y, int x, int d) {
  int h = win / 2, xr = x - d;
  if (!inside(H, W, h, y, x) || xr < h || xr > W - 1 - h) return NAN;
  int64_t n = chess ? ((int64_t)win * win + 1) / 2 : (int64_t)win * win;
  int64_t sl = 0, sll = 0, sr = 0, srr = 0, slr = 0;
  for (int v = -h; v <= h; ++v)
    for (int u = -h; u <= h; ++u) {
      if (chess && ((u + v) & 1)) continue;
      int64_t a = L[(int64_t)(y + v) * pitch + x + u], b = R[(int64_t)(y + v) * pitch + xr + u];
      sl += a; sll += a * a; sr += b; srr += b * b; slr += a * b;
    }
  int64_t vl = n * sll - sl * sl, vr = n * srr - sr * sr;
  if (vl <= 0 || vr <= 0) return NAN;
  return (double)(n * slr - sl * sr) / sqrt((double)vl * (double)vr);
}

/*
 * The re-search of Eq. (4) (Section II-C) for every valid pixel: among the
 * integer candidates o* in [d - range, d + range] (and in [dmin, dmax]) whose
 * ZNCC is defined, take the one minimising
 *     f_zncc(o*) + eta * (o* - d)^2,   f_zncc = 1 / max(z, 1e-3)
 * (the paper's reciprocal ZNCC, held finite where z <= 0); ties go to the
 * smaller o*.  A pixel without any defined candidate keeps its o.
 * o_in / o_out: H*W int32 (may alias), m: mask, d: H*W.
 */
void or_research(const uint8_t *L, const uint8_t *R, int H, int W, int pitch, int win, int chess,
                 int dmin, int dmax, const int32_t *o_in, const uint8_t *m, const double *d,
                 int range, double eta, int32_t *o_out) {
#pragma omp parallel for
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      int64_t k = (int64_t)y * W + x;
      int32_t o = o_in[k];
      if (m[k]) {
        double lo = ceil(d[k] - range), hi = floor(d[k] + range);
        if (lo < dmin) lo = dmin;
        if (hi > dmax) hi = dmax;
        double best = INFINITY;
        for (int c = (int)lo; c <= (int)hi; ++c) {
          double z = zncc_at(L, R, H, W, pitch, win, chess, y, x, c);
          if (isnan(z)) continue;
          double cost = 1.0 / (z > 1e-3 ? z : 1e-3) + eta * (c - d[k]) * (c - d[k]);
          if (cost < best) { best = cost; o = c; }
        }
      }
      o_out[k] = o;
    }
}

/*
 * The refinement of Section II-C with the discrete disparities updated in
 * every iteration (Eqs. (1)-(4)):  d^0 = o;  for k = 1..K:
 *     a   = average of o over the valid neighbours          (Eq. 1)
 *     b   = a - alpha*o - (1 - alpha)*d^{k-1}              (Eq. 2)
 *     d^k = a - average of b over the valid neighbours      (Eq. 3)
 *     o   = re-search around d^k                            (Eq. 4; k < K,
 *           the last update could not change d^K)
 * o (int32, in/out: the final discrete disparities), out = d^K (NaN where
 * invalid).  d_init (may be NULL): d^0 instead of o, so that the loop can be
 * resumed from any iteration's state (o, d).
 */
int or_hc_research(const uint8_t *L, const uint8_t *R, int H, int W, int pitch, int win, int chess,
                   int dmin, int dmax, int32_t *o, const uint8_t *m, int Rs, int K, double alpha,
                   double eta, int range, const double *d_init, double *out) {
  int64_t N = (int64_t)H * W;
  double *od = malloc(sizeof(double) * (size_t)N), *a = malloc(sizeof(double) * (size_t)N);
  double *b = malloc(sizeof(double) * (size_t)N), *ab = malloc(sizeof(double) * (size_t)N);
  double *dprev = malloc(sizeof(double) * (size_t)N);
  if (!od || !a || !b || !ab || !dprev) {
    free(od); free(a); free(b); free(ab); free(dprev);
    return OR_ENOMEM;
  }
  for (int64_t k = 0; k < N; ++k) dprev[k] = m[k] ? (d_init ? d_init[k] : (double)o[k]) : NAN;
  for (int it = 0; it < K; ++it) {
    for (int64_t k = 0; k < N; ++k) od[k] = (double)o[k];
    masked_mean(H, W, od, m, Rs, a);
    for (int64_t k = 0; k < N; ++k)
      b[k] = m[k] ? a[k] - alpha * od[k] - (1.0 - alpha) * dprev[k] : 0.0;
    masked_mean(H, W, b, m, Rs, ab);
    for (int64_t k = 0; k < N; ++k) dprev[k] = m[k] ? a[k] - ab[k] : NAN;
    if (it < K - 1)
      or_research(L, R, H, W, pitch, win, chess, dmin, dmax, o, m, dprev, range, eta, o);
  }
  if (K == 0)
    for (int64_t k = 0; k < N; ++k) dprev[k] = m[k] ? (double)o[k] : NAN;
  memcpy(out, dprev, sizeof(double) * (size_t)N);
  free(od); free(a); free(b); free(ab); free(dprev);
  return OR_OK;
}

/*
 * Disparity to 3-D points (Section II: after stereo calibration the depths
 * follow directly from the disparities; the paper's conversion is the one of
 * Matlab's reconstructScene).  Q is the 4x4 reprojection matrix of the
 * rectified pair, row-major: [X Y Z W]^T = Q [x y d 1]^T and the point is
 * (X/W, Y/W, Z/W).  A NaN disparity or W == 0 gives a NaN point.
 * xyz: H*W*3, interleaved.
 */
void or_reproject(int H, int W, const double *disp, const double *Q, double *xyz) {
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      int64_t k = (int64_t)y * W + x;
      double d = disp[k];
      double v[4] = {(double)x, (double)y, d, 1.0}, r[4];
      for (int i = 0; i < 4; ++i) {
        r[i] = 0.0;
        for (int j = 0; j < 4; ++j) r[i] += Q[4 * i + j] * v[j];
      }
      int ok = !isnan(d) && r[3] != 0.0;
      for (int c = 0; c < 3; ++c) xyz[3 * k + c] = ok ? r[c] / r[3] : NAN;
    }
}

/* Parameters of the whole pipeline (paper constants in the comments). */
typedef struct {
  int32_t subpixel;       /* 1 */
  int32_t lr_check;       /* 1 */
  int32_t lr_tol;         /* 1 px */
  int32_t radial_iters;   /* 3 alternations (Section II-B) */
  int32_t radial_r0;      /* 10 px */
  int32_t radial_dr;      /* 10 px */
  double radial_thresh;   /* 2.5 */
  int32_t fill_radial_r;  /* 50 px */
  int32_t fill_min_lines; /* 2 */
  int32_t fill_disk_r;    /* 20 px */
  double fill_disk_frac;  /* 0.25 */
  int32_t smooth_radius;  /* 15 px (Section II-C) */
  int32_t smooth_iters;   /* 3 */
  double smooth_alpha;    /* 0.1 */
  int32_t research;       /* 1: Eq. (4) re-search inside the smoothing */
  int32_t research_range; /* 5 px */
  double research_eta;    /* 0.01 */
  int32_t chess;          /* 1: chessboard window (Section II-A) */
} or_params;

/*
 * The whole stereo path of Section II (Fig. 1a): ZNCC matching and WTA, the
 * sub-pixel offset, the left-right check, then either one fill pass
 * (radial_iters == 0) or radial_iters alternations of outlier removal with
 * radius r0 + k*dr and hole filling (Section II-B), then improved Laplacian
 * smoothing (Section II-C).  Each step reads the previous step's whole map.
 * Outputs: disparity (NaN where invalid), mask (0 invalid, 1 matched,
 * 2 filled); optional intermediates may be NULL.
 */
int or_pipeline(const uint8_t *L, const uint8_t *R, int H, int W, int pitch, int dmin, int dmax,
                int win, const or_params *p, double *disp, uint8_t *mask,
                int32_t *o_wta, uint8_t *m_wta, double *delta_out, int32_t *o_post,
                uint8_t *m_lr) {
  int64_t N = (int64_t)H * W;
  int32_t *oL = malloc(sizeof(int32_t) * (size_t)N), *oR = malloc(sizeof(int32_t) * (size_t)N);
  uint8_t *mL = malloc((size_t)N), *mR = malloc((size_t)N), *mm = malloc((size_t)N);
  uint8_t *m2 = malloc((size_t)N);
  double *zb = malloc(sizeof(double) * (size_t)N), *gp = malloc(sizeof(double) * (size_t)N);
  double *zm = malloc(sizeof(double) * (size_t)N), *zp = malloc(sizeof(double) * (size_t)N);
  double *zbR = malloc(sizeof(double) * (size_t)N), *gpR = malloc(sizeof(double) * (size_t)N);
  double *dl = malloc(sizeof(double) * (size_t)N), *s = malloc(sizeof(double) * (size_t)N);
  int rc = OR_ENOMEM;
  if (!oL || !oR || !mL || !mR || !mm || !m2 || !zb || !gp || !zm || !zp || !zbR || !gpR || !dl || !s)
    goto done;
  rc = or_match(L, R, H, W, pitch, dmin, dmax, win, 0, H, 0, p->chess, oL, mL, zb, gp, zm, zp, oR,
                mR, zbR, gpR);
  if (rc) goto done;
  if (o_wta) memcpy(o_wta, oL, sizeof(int32_t) * (size_t)N);
  if (m_wta) memcpy(m_wta, mL, (size_t)N);
  if (p->subpixel) or_subpixel(N, oL, mL, zm, zb, zp, dmin, dmax, dl);
  else for (int64_t k = 0; k < N; ++k) dl[k] = 0.0;
  if (delta_out) memcpy(delta_out, dl, sizeof(double) * (size_t)N);
  if (p->lr_check) or_lr_check(H, W, oL, mL, oR, mR, p->lr_tol, mm);
  else memcpy(mm, mL, (size_t)N);
  if (m_lr) memcpy(m_lr, mm, (size_t)N);
  if (p->radial_iters <= 0) {
    rc = or_fill(H, W, oL, mm, p->fill_radial_r, p->fill_min_lines, p->fill_disk_r, p->fill_disk_frac);
    if (rc) goto done;
  } else {
    for (int it = 0; it < p->radial_iters; ++it) {
      or_radial_outlier(H, W, oL, mm, p->radial_r0 + it * p->radial_dr, p->radial_thresh, m2);
      memcpy(mm, m2, (size_t)N);
      rc = or_fill(H, W, oL, mm, p->fill_radial_r, p->fill_min_lines, p->fill_disk_r, p->fill_disk_frac);
      if (rc) goto done;
    }
  }
  if (o_post) memcpy(o_post, oL, sizeof(int32_t) * (size_t)N);
  for (int64_t k = 0; k < N; ++k) s[k] = mm[k] == 1 ? (double)oL[k] + dl[k] : (double)oL[k];
  if (p->research) {
    rc = or_hc_research(L, R, H, W, pitch, win, p->chess, dmin, dmax, oL, mm, p->smooth_radius,
                        p->smooth_iters, p->smooth_alpha, p->research_eta, p->research_range, NULL,
                        disp);
    if (rc) goto done;
  } else if (p->smooth_iters > 0) {
    rc = or_hc_smooth(H, W, s, mm, p->smooth_radius, p->smooth_iters, p->smooth_alpha, disp);
    if (rc) goto done;
  } else {
    for (int64_t k = 0; k < N; ++k) disp[k] = mm[k] ? s[k] : NAN;
  }
  memcpy(mask, mm, (size_t)N);
  rc = OR_OK;
done:
  free(oL); free(oR); free(mL); free(mR); free(mm); free(m2); free(zb); free(gp); free(zm);
  free(zp); free(zbR); free(gpR); free(dl); free(s);
  return rc;
}

/*
 * Photometric energy of a continuous disparity field (the differentiable
 * refinement added on top of the paper's Section II-C):
 *   E(d) = sum_{p in Omega} (1 - Z_p(d)) + lambda * TV(d)
 * R_w(q) = linear interpolation of the right image along row q_y at
 *          u = q_x - d(q), u clamped to [0, W-1];
 * Z_p    = ZNCC (textbook mean form) of the left window and the R_w window
 *          around p; 0 when the R_w window has zero variance;
 * Omega  = pixels with valid != 0 whose whole window lies in the image, is
 *          valid, and has non-zero left variance;
 * TV     = sum of |d(q+e) - d(q)| over right and down neighbour pairs that
 *          are both valid.
 * Z (H*W, NaN outside Omega) may be NULL.  Returns E.
 */
double or_refine_energy(const uint8_t *L, const uint8_t *R, int H, int W, int pitch, int win,
                        const double *d, const uint8_t *valid, double lambda, double *Z) {
  int h = win / 2;
  int n = win * win;
  double *rw = malloc(sizeof(double) * (size_t)H * W);
  if (!rw) return NAN;
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      double u = (double)x - d[(int64_t)y * W + x];
      if (u < 0.0) u = 0.0;
      if (u > W - 1.0) u = W - 1.0;
      int i0 = (int)floor(u);
      double t = u - i0;
      double r0 = R[(int64_t)y * pitch + i0];
      double r1 = i0 + 1 < W ? R[(int64_t)y * pitch + i0 + 1] : r0;
      rw[(int64_t)y * W + x] = r0 * (1.0 - t) + r1 * t;
    }
  double E = 0.0;
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      int64_t k = (int64_t)y * W + x;
      if (Z) Z[k] = NAN;
      if (!valid[k] || !inside(H, W, h, y, x)) continue;
      int all = 1;
      double ma = 0, mb = 0;
      for (int v = -h; v <= h && all; ++v)
        for (int u = -h; u <= h; ++u) {
          int64_t q = (int64_t)(y + v) * W + x + u;
          if (!valid[q]) { all = 0; break; }
          ma += L[(int64_t)(y + v) * pitch + x + u];
          mb += rw[q];
        }
      if (!all) continue;
      ma /= n; mb /= n;
      double sab = 0, saa = 0, sbb = 0;
      for (int v = -h; v <= h; ++v)
        for (int u = -h; u <= h; ++u) {
          double a = L[(int64_t)(y + v) * pitch + x + u] - ma;
          double b = rw[(int64_t)(y + v) * W + x + u] - mb;
          sab += a * b; saa += a * a; sbb += b * b;
        }
      if (saa == 0.0) continue;
      double z = sbb == 0.0 ? 0.0 : sab / sqrt(saa * sbb);
      if (Z) Z[k] = z;
      E += 1.0 - z;
    }
  double tv = 0.0;
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      int64_t k = (int64_t)y * W + x;
      if (!valid[k]) continue;
      if (x + 1 < W && valid[k + 1]) tv += fabs(d[k + 1] - d[k]);
      if (y + 1 < H && valid[k + W]) tv += fabs(d[k + W] - d[k]);
    }
  free(rw);
  return E + lambda * tv;
}

/*
 * The part of the refinement energy that depends on d(q): the windows of
 * Omega that contain q (their ZNCC reads R_w(q)) and the TV pairs that
 * contain q.  E(d) - E_local(d, q) does not depend on d(q), so central
 * differences of E_local at q equal those of E; it makes the check of a
 * full-size gradient cheap.  Same definitions as or_refine_energy.
 */
double or_refine_energy_local(const uint8_t *L, const uint8_t *R, int H, int W, int pitch,
                              int win, const double *d, const uint8_t *valid, double lambda,
                              int qx, int qy) {
  int h = win / 2;
  int n = win * win;
  double E = 0.0;
  for (int py = qy - h; py <= qy + h; ++py)
    for (int px = qx - h; px <= qx + h; ++px) {
      if (py < 0 || py >= H || px < 0 || px >= W) continue;
      if (!valid[(int64_t)py * W + px] || !inside(H, W, h, py, px)) continue;
      int all = 1;
      double ma = 0, mb = 0;
      double bw[15 * 15];
      for (int v = -h; v <= h && all; ++v)
        for (int u = -h; u <= h; ++u) {
          int64_t q = (int64_t)(py + v) * W + px + u;
          if (!valid[q]) { all = 0; break; }
          double uu = (double)(px + u) - d[q];
          if (uu < 0.0) uu = 0.0;
          if (uu > W - 1.0) uu = W - 1.0;
          int i0 = (int)floor(uu);
          double t = uu - i0;
          double r0 = R[(int64_t)(py + v) * pitch + i0];
          double r1 = i0 + 1 < W ? R[(int64_t)(py + v) * pitch + i0 + 1] : r0;
          double rw = r0 * (1.0 - t) + r1 * t;
          bw[(v + h) * win + (u + h)] = rw;
          ma += L[(int64_t)(py + v) * pitch + px + u];
          mb += rw;
        }
      if (!all) continue;
      ma /= n; mb /= n;
      double sab = 0, saa = 0, sbb = 0;
      for (int v = -h; v <= h; ++v)
        for (int u = -h; u <= h; ++u) {
          double a = L[(int64_t)(py + v) * pitch + px + u] - ma;
          double b = bw[(v + h) * win + (u + h)] - mb;
          sab += a * b; saa += a * a; sbb += b * b;
        }
      if (saa == 0.0) continue;
      E += 1.0 - (sbb == 0.0 ? 0.0 : sab / sqrt(saa * sbb));
    }
  int64_t k = (int64_t)qy * W + qx;
  if (valid[k]) {
    if (qx + 1 < W && valid[k + 1]) E += lambda * fabs(d[k + 1] - d[k]);
    if (qy + 1 < H && valid[k + W]) E += lambda * fabs(d[k + W] - d[k]);
    if (qx > 0 && valid[k - 1]) E += lambda * fabs(d[k] - d[k - 1]);
    if (qy > 0 && valid[k - W]) E += lambda * fabs(d[k] - d[k - W]);
  }
  return E;
}
