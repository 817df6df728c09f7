// Post-processing of the WTA disparities (Section II-B and II-C of the paper)
// and the exact sub-pixel step.  Every kernel is a Jacobi step: it reads
// whole input maps and writes new ones, one thread per pixel, so results do
// not depend on scheduling.  Integer results are exact; smoothing runs in
// FP64.  Each kernel serves one pair (descriptor by value) or a batch (table
// in device memory, pair = blockIdx.z).
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
template <bool B>
__global__ void subpixel_kernel(PostPair one, const PostPair *many) {
  PAIR;
  PIX;
  const double qn = __builtin_nan("");
  if (!P.mb[0][k]) {
    if (P.zbest) P.zbest[k] = qn;
    if (P.zm) P.zm[k] = qn;
    if (P.zp) P.zp[k] = qn;
    P.delta[k] = 0.0f;
    return;
  }
  const int win = P.win, h = win / 2;
  const long long n = (long long)win * win;
  const int o = P.ob[0][k];
  const long long sl = P.SL[k];
  const long long varL = n * (long long)P.SSL[k] - sl * sl;
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
    int slr = 0;
    for (int v = -h; v <= h; ++v) {
      const uint8_t *lr = P.left + (size_t)(y + v) * P.pitch + x - h;
      const uint8_t *rr = P.right + (size_t)(y + v) * P.pitch + xr - h;
      for (int u = 0; u < win; ++u) slr += (int)lr[u] * (int)rr[u];
    }
    const long long num = n * (long long)slr - sl * sr;
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

// ---------------------------------------------------------------- radial outliers
// A valid pixel is kept if along at least one of the 8 radial directions
// all of the next r pixels are inside the image and valid, and consecutive
// disparities differ by less than thresh (Section II-B).
template <bool B>
__global__ void radial_outlier_kernel(PostPair one, const PostPair *many, int r, float thresh,
                                      int src, int dst) {
  PAIR;
  PIX;
  const int16_t *o = P.ob[src];
  const uint8_t *m = P.mb[src];
  const uint8_t mk = m[k];
  P.ob[dst][k] = o[k];
  if (!mk) { P.mb[dst][k] = 0; return; }
  bool any = false;
  for (int dir = 0; dir < 8 && !any; ++dir) {
    const int ux = c_dir8[dir][0], uy = c_dir8[dir][1];
    const int ex = x + r * ux, ey = y + r * uy;
    if (ex < 0 || ex >= W || ey < 0 || ey >= H) continue;
    int prev = o[k];
    bool pass = true;
    for (int s = 1; s <= r; ++s) {
      const size_t q = (size_t)(y + s * uy) * W + (x + s * ux);
      if (!m[q]) { pass = false; break; }
      const int v = o[q];
      const int dv = v - prev;
      if (!((float)(dv < 0 ? -dv : dv) < thresh)) { pass = false; break; }
      prev = v;
    }
    any = pass;
  }
  P.mb[dst][k] = any ? mk : 0;
}

// ---------------------------------------------------------------- hole filling
// (i) radial: first valid pixel within R steps along each of the 8
// directions; complete lines (both opposite directions hit) give
// (va*sb + vb*sa)/(sa+sb); with >= min_lines complete lines the hole takes
// their mean, an exact rational rounded half to even; code 2.
template <bool B>
__global__ void fill_radial_kernel(PostPair one, const PostPair *many, int R, int min_lines,
                                   int src, int dst) {
  PAIR;
  PIX;
  const int16_t *o = P.ob[src];
  const uint8_t *m = P.mb[src];
  P.ob[dst][k] = o[k];
  P.mb[dst][k] = m[k];
  if (m[k]) return;
  int v[8], s[8];
  bool hit[8];
  for (int dir = 0; dir < 8; ++dir) {
    hit[dir] = false;
    v[dir] = 0;
    s[dir] = 0;
    const int ux = c_dir8[dir][0], uy = c_dir8[dir][1];
    for (int st = 1; st <= R; ++st) {
      const int qx = x + st * ux, qy = y + st * uy;
      if (qx < 0 || qx >= W || qy < 0 || qy >= H) break;
      const size_t q = (size_t)qy * W + qx;
      if (m[q]) { hit[dir] = true; v[dir] = o[q]; s[dir] = st; break; }
    }
  }
  long long num = 0, den = 1;
  int lines = 0;
  for (int l = 0; l < 4; ++l) {
    const int a = 2 * l, b = 2 * l + 1;
    if (!(hit[a] && hit[b])) continue;
    const long long ln = (long long)v[a] * s[b] + (long long)v[b] * s[a];
    const long long ld = s[a] + s[b];
    num = num * ld + ln * den;
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
  LAUNCH(subpixel_kernel, pixgrid(L), dim3(128));
  return hipGetLastError();
}
hipError_t post_lr(const PostLaunch &L, int tol, int dst) {
  LAUNCH(lr_check_kernel, pixgrid(L), dim3(128), tol, dst);
  return hipGetLastError();
}
hipError_t post_outlier(const PostLaunch &L, int r, float thresh, int src, int dst) {
  LAUNCH(radial_outlier_kernel, pixgrid(L), dim3(128), r, thresh, src, dst);
  return hipGetLastError();
}
// radial fill src -> tmp, disk fill tmp -> dst (dst may equal src)
hipError_t post_fill(const PostLaunch &L, int radial_r, int min_lines, int disk_r, float frac,
                     int src, int tmp, int dst) {
  LAUNCH(fill_radial_kernel, pixgrid(L), dim3(128), radial_r, min_lines, src, tmp);
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
