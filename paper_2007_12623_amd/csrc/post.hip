// Post-processing of the WTA disparities (Section II-B and II-C of the paper)
// and the exact sub-pixel step.  Every kernel is a Jacobi step: it reads
// whole input maps and writes new ones, one thread per pixel, so results do
// not depend on scheduling.  Integer results are exact; smoothing runs in
// FP64.  Each kernel serves one pair (descriptor by value) or a batch (table
// in device memory, pair = blockIdx.z).
#include <algorithm>

#include "common.h"

namespace st {

#define PAIR const PostPair &P = B ? many[blockIdx.z] : one
#define PIX                                                     \
  const int x = blockIdx.x * blockDim.x + threadIdx.x;         \
  const int y = blockIdx.y;                                     \
  if (x >= P.W || y >= P.H) return;                             \
  const int W = P.W, H = P.H;                                   \
  const size_t k = (size_t)y * W + x;                           \
  (void)H

__device__ __forceinline__ long long floordiv_ll(long long a, long long b) {
  long long q = a / b, r = a % b;
  if (r != 0 && ((r < 0) != (b < 0))) --q;
  return q;
}
// round(num/den) to nearest, ties to even; den > 0
__device__ __forceinline__ long long round_half_even(long long num, long long den) {
  const long long q = floordiv_ll(num, den);
  const long long r = num - q * den;
  if (2 * r > den) return q + 1;
  if (2 * r == den) return (q & 1) ? q + 1 : q;
  return q;
}

// ---------------------------------------------------------------- decode
// Merged keys -> WTA disparities and masks (ob[0], mb[0], oR, mR); the keys
// are cleared for the next matcher run.
template <bool B>
__global__ void decode_kernel(PostPair one, const PostPair *many) {
  PAIR;
  PIX;
  const uint32_t a = P.keyL[k], b = P.keyR[k];
  P.ob[0][k] = a ? (int16_t)(P.dmin + 255 - (int)(a & 255u)) : 0;
  P.mb[0][k] = a ? 1 : 0;
  P.oR[k] = b ? (int16_t)(P.dmin + 255 - (int)(b & 255u)) : 0;
  P.mR[k] = b ? 1 : 0;
  P.keyL[k] = 0;
  P.keyR[k] = 0;
}

__global__ void fill_u32_kernel(uint32_t *p, int N, uint32_t v) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < N) p[k] = v;
}

// ---------------------------------------------------------------- sub-pixel
// Exact ZNCC at o-1, o, o+1 (int32 window sums of L*R, int64 numerator
// n*S_LR - S_L*S_R, FP64 normalisation), then the parabola offset
// delta = (zm - zp) / (2 (zm - 2 z0 + zp)) clamped to [-1/2, 1/2]; 0 at the
// ends of the range, when a neighbour is missing or the curvature is >= 0.
// A block covers 128 pixels of one row: it stages the window rows of the left
// image and the right columns its disparities reach in LDS once, then every
// thread slides a 3-value window over the right row for the three sums.
constexpr int SP_TX = 128, SP_MAXWIN = 15;
template <bool B>
__global__ __launch_bounds__(SP_TX) void subpixel_kernel(PostPair one, const PostPair *many) {
  PAIR;
  __shared__ uint8_t Ls[SP_MAXWIN][SP_TX + 16];
  __shared__ uint8_t Rs[SP_MAXWIN][SP_TX + 256 + 24];
  __shared__ int s_omin, s_omax;
  const int tx = threadIdx.x;
  const int x0 = blockIdx.x * SP_TX, y = blockIdx.y;
  if (x0 >= P.W || y >= P.H) return;  // uniform per block
  const int W = P.W, H = P.H, win = P.win, h = win / 2;
  const int x = x0 + tx;
  const bool in = x < W;
  const size_t k = (size_t)y * W + x;
  const bool valid = in && P.mb[0][k];
  const int o = valid ? (int)P.ob[0][k] : 0;
  if (tx == 0) {
    s_omin = 1 << 30;
    s_omax = -(1 << 30);
  }
  __syncthreads();
  if (valid) {
    atomicMin(&s_omin, o);
    atomicMax(&s_omax, o);
  }
  __syncthreads();
  const int omin = s_omin, omax = s_omax;
  const double qn = __builtin_nan("");
  if (omin <= omax) {
    const int LW = SP_TX + 2 * h, RW = SP_TX + (omax - omin) + 2 + 2 * h;
    const int lx0 = x0 - h, rx0 = x0 - omax - 1 - h;
    for (int i = tx; i < win * LW; i += SP_TX) {
      const int r = i / LW, c = i - r * LW;
      const int gy = y - h + r, gx = lx0 + c;
      Ls[r][c] = (gy >= 0 && gy < H && gx >= 0 && gx < W) ? P.left[(size_t)gy * P.pitch + gx] : 0;
    }
    for (int i = tx; i < win * RW; i += SP_TX) {
      const int r = i / RW, c = i - r * RW;
      const int gy = y - h + r, gx = rx0 + c;
      Rs[r][c] = (gy >= 0 && gy < H && gx >= 0 && gx < W) ? P.right[(size_t)gy * P.pitch + gx] : 0;
    }
  }
  __syncthreads();
  if (!in) return;
  if (!valid) {
    if (P.zbest) P.zbest[k] = qn;
    if (P.zm) P.zm[k] = qn;
    if (P.zp) P.zp[k] = qn;
    P.delta[k] = 0.0f;
    return;
  }
  // Rs[v][q] holds R(y - h + v, x - h + u - o) for q = tx + u + omax + 1 - o
  int sm = 0, s0 = 0, sp = 0;  // sums at d = o - 1, o, o + 1
  const int qb = tx + omax + 1 - o;
  for (int v = 0; v < win; ++v) {
    const uint8_t *lr = &Ls[v][tx];
    const uint8_t *rr = &Rs[v][qb];
    int rprev = rr[-1], rcur = rr[0];
    for (int u = 0; u < win; ++u) {
      const int rnext = rr[u + 1];
      const int l = lr[u];
      sp += l * rprev;
      s0 += l * rcur;
      sm += l * rnext;
      rprev = rcur;
      rcur = rnext;
    }
  }
  const long long n = (long long)win * win;
  const long long sl = P.SL[k];
  const long long varL = n * (long long)P.SSL[k] - sl * sl;
  const int slr[3] = {sm, s0, sp};
  double z[3];
  for (int q = 0; q < 3; ++q) {
    const int d = o + q - 1;
    const int xr = x - d;
    z[q] = qn;
    if (d < P.dmin || d > P.dmax || xr < h || xr > W - 1 - h) continue;
    const size_t kr = (size_t)y * W + xr;
    const long long sr = P.SR[kr];
    const long long varR = n * (long long)P.SSR[kr] - sr * sr;
    if (varR <= 0) continue;
    const long long num = n * (long long)slr[q] - sl * sr;
    z[q] = (double)num / sqrt((double)varL * (double)varR);
  }
  if (P.zbest) P.zbest[k] = z[1];
  if (P.zm) P.zm[k] = z[0];
  if (P.zp) P.zp[k] = z[2];
  double dl = 0.0;
  if (o > P.dmin && o < P.dmax && !__builtin_isnan(z[0]) && !__builtin_isnan(z[2])) {
    const double den = 2.0 * (z[0] - 2.0 * z[1] + z[2]);
    if (den < 0.0) {
      dl = (z[0] - z[2]) / den;
      dl = dl > 0.5 ? 0.5 : (dl < -0.5 ? -0.5 : dl);
    }
  }
  P.delta[k] = (float)dl;
}

// ---------------------------------------------------------------- LR check
// (ob[0], mb[0]) and (oR, mR) -> (ob[dst], mb[dst]): kept when the right
// pixel x - oL points back within tol.
template <bool B>
__global__ void lr_check_kernel(PostPair one, const PostPair *many, int tol, int dst) {
  PAIR;
  PIX;
  const int16_t *oL = P.ob[0];
  uint8_t keep = 0;
  if (P.mb[0][k]) {
    const int xr = x - oL[k];
    if (xr >= 0 && xr < W) {
      const size_t kr = (size_t)y * W + xr;
      const int diff = (int)oL[k] - (int)P.oR[kr];
      if (P.mR[kr] && (diff < 0 ? -diff : diff) <= tol) keep = 1;
    }
  }
  P.ob[dst][k] = oL[k];
  P.mb[dst][k] = keep;
}

__constant__ int c_dir8[8][2] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}, {1, 1}, {-1, -1}, {1, -1}, {-1, 1}};

// ---------------------------------------------------------------- radial line scans
// The 8 radial directions come in 4 line types: rows, columns, diagonals
// (x - y const) and anti-diagonals (x + y const); c_dir8[2t] steps forward
// along a line of type t, c_dir8[2t+1] backward.  A thread owns one segment
// of SEG positions of one line and scans it, plus a look-ahead of `reach`
// positions, in both directions; segments are independent.
constexpr int SEG = 64;

struct LineGeom {
  int x, y, dx, dy, len;
};

__device__ __forceinline__ int nlines(int t, int H, int W) {
  return t == 0 ? H : (t == 1 ? W : W + H - 1);
}
__device__ __forceinline__ int maxlen(int t, int H, int W) {
  return t == 0 ? W : (t == 1 ? H : min(W, H));
}
__device__ __forceinline__ LineGeom line_geom(int t, int l, int H, int W) {
  LineGeom g;
  if (t == 0) { g.x = 0; g.y = l; g.dx = 1; g.dy = 0; g.len = W; }
  else if (t == 1) { g.x = l; g.y = 0; g.dx = 0; g.dy = 1; g.len = H; }
  else if (t == 2) {  // x - y = l - (H - 1), step (1, 1)
    const int c = l - (H - 1);
    g.x = max(0, c); g.y = max(0, -c); g.dx = 1; g.dy = 1;
    g.len = min(W - g.x, H - g.y);
  } else {            // x + y = l, step (1, -1)
    g.x = max(0, l - (H - 1)); g.y = min(l, H - 1); g.dx = 1; g.dy = -1;
    g.len = min(W - g.x, g.y + 1);
  }
  return g;
}

// Thread index -> (line type, line, segment); false when out of range.
__device__ __forceinline__ bool scan_task(int idx, int H, int W, int &t, int &l, int &sg) {
  for (t = 0; t < 4; ++t) {
    const int nl = nlines(t, H, W), ns = ceil_div(maxlen(t, H, W), SEG);
    if (idx < nl * ns) {
      sg = idx / nl;
      l = idx - sg * nl;
      return true;
    }
    idx -= nl * ns;
  }
  return false;
}

__device__ __forceinline__ int scan_tasks(int H, int W) {
  int n = 0;
  for (int t = 0; t < 4; ++t) n += nlines(t, H, W) * ceil_div(maxlen(t, H, W), SEG);
  return n;
}

// Outlier runs: for direction u, run(p) = number of consecutive steps
// p -> p+u -> ... that land on valid pixels whose disparity differs from the
// previous one by less than thresh.  p passes u when run(p) >= r.  Writes
// pass[t][p] = bit 0 (forward direction) | bit 1 (backward direction).
template <bool B>
__global__ void outlier_scan_kernel(PostPair one, const PostPair *many, int r, float thresh, int src) {
  PAIR;
  const int H = P.H, W = P.W;
  int t, l, sg;
  if (!scan_task(blockIdx.x * blockDim.x + threadIdx.x, H, W, t, l, sg)) return;
  const LineGeom g = line_geom(t, l, H, W);
  const int a = sg * SEG;
  if (a >= g.len) return;
  const int b = min(g.len, a + SEG);
  const int16_t *o = P.ob[src];
  const uint8_t *m = P.mb[src];
  const size_t N = (size_t)W * H;
  uint8_t *pass = P.pass + (size_t)t * N;
  const int lstep = g.dy * W + g.dx;
  const long long base = (long long)g.y * W + g.x;
  // forward: walk from the far end of the look-ahead towards a
  {
    const int e = min(g.len - 1, b - 1 + r);
    int run = 0, onext = 0;
    bool vnext = false;
    for (int p = e; p >= a; --p) {
      const long long k = base + (long long)p * lstep;
      const int op = o[k];
      if (p < e) {
        const int dv = onext - op;
        run = (vnext && (float)(dv < 0 ? -dv : dv) < thresh) ? min(run + 1, r) : 0;
      }
      if (p < b) pass[k] = run >= r ? 1 : 0;
      onext = op;
      vnext = m[k] != 0;
    }
  }
  // backward
  {
    const int e = max(0, a - r);
    int run = 0, oprev = 0;
    bool vprev = false;
    for (int p = e; p < b; ++p) {
      const long long k = base + (long long)p * lstep;
      const int op = o[k];
      if (p > e) {
        const int dv = oprev - op;
        run = (vprev && (float)(dv < 0 ? -dv : dv) < thresh) ? min(run + 1, r) : 0;
      }
      if (p >= a && run >= r) pass[k] |= 2;
      oprev = op;
      vprev = m[k] != 0;
    }
  }
}

// A valid pixel stays when some direction passes (Section II-B).
template <bool B>
__global__ void outlier_combine_kernel(PostPair one, const PostPair *many, int src, int dst) {
  PAIR;
  PIX;
  const size_t N = (size_t)W * H;
  const uint8_t mk = P.mb[src][k];
  P.ob[dst][k] = P.ob[src][k];
  const bool any = (P.pass[k] | P.pass[N + k] | P.pass[2 * N + k] | P.pass[3 * N + k]) != 0;
  P.mb[dst][k] = (mk && any) ? mk : 0;
}

// Nearest valid pixel within R steps in each direction of a line type:
// hits[2t (+1)][p] = (steps << 16) | (uint16 disparity), 0 when none.
template <bool B>
__global__ void fill_scan_kernel(PostPair one, const PostPair *many, int R, int src) {
  PAIR;
  const int H = P.H, W = P.W;
  int t, l, sg;
  if (!scan_task(blockIdx.x * blockDim.x + threadIdx.x, H, W, t, l, sg)) return;
  const LineGeom g = line_geom(t, l, H, W);
  const int a = sg * SEG;
  if (a >= g.len) return;
  const int b = min(g.len, a + SEG);
  const int16_t *o = P.ob[src];
  const uint8_t *m = P.mb[src];
  const size_t N = (size_t)W * H;
  uint32_t *hf = P.hits + (size_t)(2 * t) * N, *hb = P.hits + (size_t)(2 * t + 1) * N;
  const int lstep = g.dy * W + g.dx;
  const long long base = (long long)g.y * W + g.x;
  {
    const int e = min(g.len - 1, b - 1 + R);
    int q = -1;
    uint32_t vq = 0;
    for (int p = e; p >= a; --p) {
      const long long k = base + (long long)p * lstep;
      if (p < b) hf[k] = (q >= 0 && q - p <= R) ? ((uint32_t)(q - p) << 16) | vq : 0u;
      if (m[k]) { q = p; vq = (uint16_t)o[k]; }
    }
  }
  {
    const int e = max(0, a - R);
    int q = -1;
    uint32_t vq = 0;
    for (int p = e; p < b; ++p) {
      const long long k = base + (long long)p * lstep;
      if (p >= a) hb[k] = (q >= 0 && p - q <= R) ? ((uint32_t)(p - q) << 16) | vq : 0u;
      if (m[k]) { q = p; vq = (uint16_t)o[k]; }
    }
  }
}

// (i) radial fill from the scanned hits: complete lines (both opposite
// directions hit) give (va*sb + vb*sa)/(sa+sb); with >= min_lines complete
// lines the hole takes their mean, an exact rational rounded half to even;
// code 2.
template <bool B>
__global__ void fill_radial_kernel(PostPair one, const PostPair *many, int min_lines, int src,
                                   int dst) {
  PAIR;
  PIX;
  const int16_t *o = P.ob[src];
  const uint8_t *m = P.mb[src];
  P.ob[dst][k] = o[k];
  P.mb[dst][k] = m[k];
  if (m[k]) return;
  const size_t N = (size_t)W * H;
  long long num = 0, den = 1;
  int lines = 0;
  for (int ln = 0; ln < 4; ++ln) {
    const uint32_t ha = P.hits[(size_t)(2 * ln) * N + k], hb = P.hits[(size_t)(2 * ln + 1) * N + k];
    if (!ha || !hb) continue;
    const long long sa = ha >> 16, sb = hb >> 16;
    const long long va = (int16_t)(ha & 0xFFFFu), vb = (int16_t)(hb & 0xFFFFu);
    const long long lnum = va * sb + vb * sa;
    const long long ld = sa + sb;
    num = num * ld + lnum * den;
    den = den * ld;
    ++lines;
  }
  if (lines >= min_lines && lines > 0) {
    P.ob[dst][k] = (int16_t)round_half_even(num, den * lines);
    P.mb[dst][k] = 2;
  }
}

// Row prefix sums of the valid count and of the valid disparities of
// (ob[src], mb[src]): pc[y][x+1] = sum_{x' <= x} [m != 0]; pc[y][0] = 0.
template <bool B>
__global__ __launch_bounds__(256) void row_prefix_kernel(PostPair one, const PostPair *many,
                                                         int src) {
  PAIR;
  __shared__ int sc[256], ss[256];
  const int y = blockIdx.x;
  if (y >= P.H) return;
  const int W = P.W;
  const int16_t *o = P.ob[src];
  const uint8_t *m = P.mb[src];
  const int t = threadIdx.x;
  const int per = ceil_div(W, 256);
  const int x0 = min(t * per, W), x1 = min(x0 + per, W);
  int c = 0, s = 0;
  for (int x = x0; x < x1; ++x) {
    const size_t k = (size_t)y * W + x;
    if (m[k]) { ++c; s += o[k]; }
  }
  sc[t] = c;
  ss[t] = s;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    int ac = 0, as = 0;
    if (t >= off) { ac = sc[t - off]; as = ss[t - off]; }
    __syncthreads();
    sc[t] += ac;
    ss[t] += as;
    __syncthreads();
  }
  int bc = t ? sc[t - 1] : 0, bs = t ? ss[t - 1] : 0;
  int32_t *pcr = P.pc + (size_t)y * (W + 1), *psr = P.ps + (size_t)y * (W + 1);
  if (t == 0) { pcr[0] = 0; psr[0] = 0; }
  for (int x = x0; x < x1; ++x) {
    const size_t k = (size_t)y * W + x;
    if (m[k]) { ++bc; bs += o[k]; }
    pcr[x + 1] = bc;
    psr[x + 1] = bs;
  }
}

__device__ __forceinline__ int isqrt_floor(int v) {
  int w = (int)sqrt((double)v);
  while ((w + 1) * (w + 1) <= v) ++w;
  while (w * w > v) --w;
  return w;
}

// (ii) disk: holes with at least ceil(frac * in-image disk cells) valid
// pixels within radius R take their mean, rounded half to even; code 2.
// Disk sums come from the row prefix sums, one segment per disk row.
template <bool B>
__global__ void fill_disk_kernel(PostPair one, const PostPair *many, int R, float frac, int src,
                                 int dst) {
  PAIR;
  PIX;
  const int16_t *o = P.ob[src];
  const uint8_t *m = P.mb[src];
  P.ob[dst][k] = o[k];
  P.mb[dst][k] = m[k];
  if (m[k]) return;
  long long cells = 0, cnt = 0, sum = 0;
  for (int dy = -R; dy <= R; ++dy) {
    const int qy = y + dy;
    if (qy < 0 || qy >= H) continue;
    const int w = isqrt_floor(R * R - dy * dy);
    const int xl = max(0, x - w), xh = min(W - 1, x + w);
    if (xl > xh) continue;
    cells += xh - xl + 1;
    const int32_t *pcr = P.pc + (size_t)qy * (W + 1), *psr = P.ps + (size_t)qy * (W + 1);
    cnt += pcr[xh + 1] - pcr[xl];
    sum += psr[xh + 1] - psr[xl];
  }
  const double need = ceil((double)frac * (double)cells);
  if (cnt > 0 && (double)cnt >= need) {
    P.ob[dst][k] = (int16_t)round_half_even(sum, cnt);
    P.mb[dst][k] = 2;
  }
}

// ---------------------------------------------------------------- smoothing (FP64)
// Planes of P.f: 0 s, 1 s*m / b, 2 box(m), 3 column pass, 4 a = A(s), 5 d.
enum { F_S = 0, F_IN = 1, F_CNT = 2, F_TMP = 3, F_A = 4, F_D = 5 };

// s = o + delta for matched pixels (code 1), o for filled ones (code 2), or
// the given s_in; plane F_IN <- s*m, F_D <- m (ones, used for the counts).
template <bool B>
__global__ void hc_init_kernel(PostPair one, const PostPair *many, int src, int use_delta) {
  PAIR;
  PIX;
  const size_t N = (size_t)W * H;
  const uint8_t mk = P.mb[src][k];
  double v = 0.0;
  if (mk) {
    if (P.s_in) v = (double)P.s_in[k];
    else v = (mk == 1 && use_delta) ? (double)P.ob[src][k] + (double)P.delta[k] : (double)P.ob[src][k];
  }
  P.f[F_S * N + k] = v;
  P.f[F_IN * N + k] = mk ? v : 0.0;
  P.f[F_D * N + k] = mk ? 1.0 : 0.0;
}

// Box sums over a (2R+1) window along columns: a thread owns one column and
// a segment of seg rows, seeds the window sum, then slides it.
template <bool B>
__global__ void box_v_kernel(PostPair one, const PostPair *many, int R, int seg, int in, int out) {
  PAIR;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y0 = blockIdx.y * seg;
  const int H = P.H, W = P.W;
  if (x >= W || y0 >= H) return;
  const size_t N = (size_t)W * H;
  const double *fi = P.f + in * N;
  double *fo = P.f + out * N;
  double s = 0.0;
  for (int v = y0 - R; v <= y0 + R; ++v)
    if (v >= 0 && v < H) s += fi[(size_t)v * W + x];
  const int y1 = min(y0 + seg, H);
  for (int y = y0; y < y1; ++y) {
    fo[(size_t)y * W + x] = s;
    const int a = y + R + 1, b = y - R;
    if (a < H) s += fi[(size_t)a * W + x];
    if (b >= 0) s -= fi[(size_t)b * W + x];
  }
}

template <bool B>
__global__ void box_h_kernel(PostPair one, const PostPair *many, int R, int seg, int in, int out) {
  PAIR;
  const int y = blockIdx.x * blockDim.x + threadIdx.x;
  const int x0 = blockIdx.y * seg;
  const int H = P.H, W = P.W;
  if (y >= H || x0 >= W) return;
  const size_t N = (size_t)W * H;
  const double *row = P.f + in * N + (size_t)y * W;
  double *fo = P.f + out * N + (size_t)y * W;
  double s = 0.0;
  for (int u = x0 - R; u <= x0 + R; ++u)
    if (u >= 0 && u < W) s += row[u];
  const int x1 = min(x0 + seg, W);
  for (int x = x0; x < x1; ++x) {
    fo[x] = s;
    const int a = x + R + 1, b = x - R;
    if (a < W) s += row[a];
    if (b >= 0) s -= row[b];
  }
}

// Row box sums through LDS: one block per row stages the row, takes an
// inclusive prefix sum and writes out(x) = P(min(x+R, W-1)) - P(x-R-1),
// with coalesced loads and stores.  Rows up to BOXH_MAXW wide.
constexpr int BOXH_MAXW = 4096;
template <bool B>
__global__ __launch_bounds__(256) void box_h_lds_kernel(PostPair one, const PostPair *many, int R,
                                                        int in, int out) {
  PAIR;
  __shared__ double row[BOXH_MAXW];
  __shared__ double part[256];
  const int y = blockIdx.x;
  const int H = P.H, W = P.W;
  if (y >= H) return;
  const size_t N = (size_t)W * H;
  const double *src = P.f + in * N + (size_t)y * W;
  double *dst = P.f + out * N + (size_t)y * W;
  const int t = threadIdx.x;
  for (int x = t; x < W; x += 256) row[x] = src[x];
  __syncthreads();
  // each thread scans a contiguous segment, then the segment totals
  const int per = ceil_div(W, 256);
  const int x0 = min(t * per, W), x1 = min(x0 + per, W);
  double acc = 0.0;
  for (int x = x0; x < x1; ++x) {
    acc += row[x];
    row[x] = acc;
  }
  part[t] = acc;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const double v = t >= off ? part[t - off] : 0.0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  const double base = t ? part[t - 1] : 0.0;
  for (int x = x0; x < x1; ++x) row[x] += base;
  __syncthreads();
  for (int x = t; x < W; x += 256) {
    const int a = min(x + R, W - 1), b = x - R - 1;
    dst[x] = row[a] - (b >= 0 ? row[b] : 0.0);
  }
}

// a = A(s) = box(s m) / box(m) on valid pixels (Eq. 1)
template <bool B>
__global__ void hc_a_kernel(PostPair one, const PostPair *many, int src) {
  PAIR;
  PIX;
  const size_t N = (size_t)W * H;
  P.f[F_A * N + k] = P.mb[src][k] ? P.f[F_IN * N + k] / P.f[F_CNT * N + k] : 0.0;
}

// b = a - alpha*s - (1-alpha)*d_prev on valid pixels, 0 elsewhere (Eq. 2);
// d_prev is s in the first iteration.
template <bool B>
__global__ void hc_b_kernel(PostPair one, const PostPair *many, int src, double alpha, int first) {
  PAIR;
  PIX;
  const size_t N = (size_t)W * H;
  const double s = P.f[F_S * N + k];
  const double dp = first ? s : P.f[F_D * N + k];
  P.f[F_IN * N + k] = P.mb[src][k] ? P.f[F_A * N + k] - alpha * s - (1.0 - alpha) * dp : 0.0;
}

// d = a - A(b) (Eq. 3)
template <bool B>
__global__ void hc_d_kernel(PostPair one, const PostPair *many, int src) {
  PAIR;
  PIX;
  const size_t N = (size_t)W * H;
  P.f[F_D * N + k] = P.mb[src][k] ? P.f[F_A * N + k] - P.f[F_IN * N + k] / P.f[F_CNT * N + k] : 0.0;
}

template <bool B>
__global__ void hc_out_kernel(PostPair one, const PostPair *many, int src, int plane) {
  PAIR;
  PIX;
  const size_t N = (size_t)W * H;
  const uint8_t mk = P.mb[src][k];
  P.disparity[k] = mk ? (float)P.f[plane * N + k] : __builtin_nanf("");
  if (P.valid_mask) P.valid_mask[k] = mk;
}

// ---------------------------------------------------------------- host side
static inline dim3 pixgrid(const PostLaunch &L) { return dim3(ceil_div(L.maxW, 128), L.maxH, L.npairs); }

#define LAUNCH(kern, grid, block, ...)                                                   \
  do {                                                                                   \
    if (L.many)                                                                          \
      hipLaunchKernelGGL(kern<true>, grid, block, 0, L.s, L.one, L.many, ##__VA_ARGS__); \
    else                                                                                 \
      hipLaunchKernelGGL(kern<false>, grid, block, 0, L.s, L.one, L.many, ##__VA_ARGS__); \
  } while (0)

hipError_t post_decode(const PostLaunch &L) {
  LAUNCH(decode_kernel, pixgrid(L), dim3(128));
  return hipGetLastError();
}
hipError_t post_subpixel(const PostLaunch &L) {
  LAUNCH(subpixel_kernel, dim3(ceil_div(L.maxW, SP_TX), L.maxH, L.npairs), dim3(SP_TX));
  return hipGetLastError();
}
hipError_t post_lr(const PostLaunch &L, int tol, int dst) {
  LAUNCH(lr_check_kernel, pixgrid(L), dim3(128), tol, dst);
  return hipGetLastError();
}
static dim3 scangrid(const PostLaunch &L) {
  int n = 0;
  for (int t = 0; t < 4; ++t) {
    const int nl = t == 0 ? L.maxH : (t == 1 ? L.maxW : L.maxW + L.maxH - 1);
    const int ml = t == 0 ? L.maxW : (t == 1 ? L.maxH : std::min(L.maxW, L.maxH));
    n += nl * ceil_div(ml, SEG);
  }
  return dim3(ceil_div(n, 64), 1, L.npairs);
}

hipError_t post_outlier(const PostLaunch &L, int r, float thresh, int src, int dst) {
  LAUNCH(outlier_scan_kernel, scangrid(L), dim3(64), r, thresh, src);
  LAUNCH(outlier_combine_kernel, pixgrid(L), dim3(128), src, dst);
  return hipGetLastError();
}
// radial fill src -> tmp, disk fill tmp -> dst (dst may equal src)
hipError_t post_fill(const PostLaunch &L, int radial_r, int min_lines, int disk_r, float frac,
                     int src, int tmp, int dst) {
  LAUNCH(fill_scan_kernel, scangrid(L), dim3(64), radial_r, src);
  LAUNCH(fill_radial_kernel, pixgrid(L), dim3(128), min_lines, src, tmp);
  LAUNCH(row_prefix_kernel, dim3(L.maxH, 1, L.npairs), dim3(256), tmp);
  LAUNCH(fill_disk_kernel, pixgrid(L), dim3(128), disk_r, frac, tmp, dst);
  return hipGetLastError();
}

static void box2d(const PostLaunch &L, int R, int in, int out) {
  const int seg = 32;
  LAUNCH(box_v_kernel, dim3(ceil_div(L.maxW, 64), ceil_div(L.maxH, seg), L.npairs), dim3(64), R,
         seg, in, F_TMP);
  if (L.maxW <= BOXH_MAXW)
    LAUNCH(box_h_lds_kernel, dim3(L.maxH, 1, L.npairs), dim3(256), R, F_TMP, out);
  else
    LAUNCH(box_h_kernel, dim3(ceil_div(L.maxH, 64), ceil_div(L.maxW, seg), L.npairs), dim3(64), R,
           seg, F_TMP, out);
}

// Improved Laplacian smoothing of (ob[src], delta, mb[src]) or s_in; writes
// disparity (NaN where invalid) and valid_mask.
hipError_t post_hc(const PostLaunch &L, int src, int R, int K, float alpha, int use_delta) {
  LAUNCH(hc_init_kernel, pixgrid(L), dim3(128), src, use_delta);
  box2d(L, R, F_D, F_CNT);  // counts of valid pixels
  box2d(L, R, F_IN, F_IN);  // box(s m)
  LAUNCH(hc_a_kernel, pixgrid(L), dim3(128), src);
  for (int it = 0; it < K; ++it) {
    LAUNCH(hc_b_kernel, pixgrid(L), dim3(128), src, (double)alpha, it == 0 ? 1 : 0);
    box2d(L, R, F_IN, F_IN);
    LAUNCH(hc_d_kernel, pixgrid(L), dim3(128), src);
  }
  LAUNCH(hc_out_kernel, pixgrid(L), dim3(128), src, K > 0 ? (int)F_D : (int)F_S);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, int N, uint32_t v, hipStream_t s) {
  hipLaunchKernelGGL(fill_u32_kernel, dim3(ceil_div(N, 256)), dim3(256), 0, s, p, N, v);
  return hipGetLastError();
}

}  // namespace st
