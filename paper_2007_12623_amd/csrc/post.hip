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
// Per-pixel kernels: a block of PIX_T threads covers PIX_SEG columns of one
// row, PIX_SEG / PIX_T pixels per thread at stride PIX_T (coalesced).  Few,
// fat blocks: with one short-lived block per 128 pixels these kernels were
// limited by the rate at which waves are launched, not by work.
constexpr int PIX_T = 256, PIX_SEG = 1024;
template <class F>
__device__ __forceinline__ void for_pixels(const PostPair &P, F f) {
  const int y = blockIdx.y;
  if (y >= P.H) return;
  const int x1 = min(P.W, (int)(blockIdx.x + 1) * PIX_SEG);
  for (int x = blockIdx.x * PIX_SEG + threadIdx.x; x < x1; x += PIX_T) f(x, y, (size_t)y * P.W + x);
}

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
__global__ void decode_kernel(PostPair one, const PostPair *__restrict__ many) {
  PAIR;
  const int W = P.W, H = P.H;
  (void)W;
  (void)H;
  for_pixels(P, [&](int x, int y, size_t k) {
    const uint32_t a = P.keyL[k], b = P.keyR[k];
    P.ob[0][k] = a ? (int16_t)(P.dmin + 255 - (int)(a & 255u)) : 0;
    P.mb[0][k] = a ? 1 : 0;
    P.oR[k] = b ? (int16_t)(P.dmin + 255 - (int)(b & 255u)) : 0;
    P.mR[k] = b ? 1 : 0;
    P.keyL[k] = 0;
    P.keyR[k] = 0;
  });
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
// image and the right columns its disparities reach in LDS once; every thread
// then reads its window rows as packed bytes and forms the three sums with
// v_dot4_u32_u8 (4 products per instruction, exact in 32 bits).
constexpr int SP_TX = 128, SP_MAXWIN = 15;
constexpr int SP_LROW = SP_TX + 24, SP_RROW = SP_TX + 256 + 32;

// Copy the bytes [off, off + len) of the image buffer base[0, span) (byte
// offsets relative to base; off may be negative) to an LDS row as whole
// dwords starting at the dword-aligned address at or below base + off, one
// dword per thread (len + 3 < 4 * SP_TX); the byte offset of base + off in
// the LDS row is (base + off) & 3.  The range of dwords wholly inside the
// buffer is worked out once per row (uniform); the at most two dwords that
// straddle its ends are assembled byte by byte; bytes outside come out 0.
__device__ __forceinline__ void stage_row(uint8_t *dst, const GLOBAL uint8_t *base, long long off,
                                          int len, long long span, int tid) {
  const int mis = (int)(((uintptr_t)base + (uintptr_t)off) & 3);
  const long long a0 = off - mis;  // offset of dword 0
  const int nd = (mis + len + 3) >> 2;
  const int ilo = a0 >= 0 ? 0 : (int)((-a0 + 3) >> 2);
  const int ihi = span - a0 >= 4 ? (int)min((span - a0) >> 2, (long long)nd) : 0;
  if (tid >= nd) return;
  const GLOBAL uint32_t *row = (const GLOBAL uint32_t *)(base + a0);
  uint32_t v;
  if (tid >= ilo && tid < ihi) {
    v = row[(unsigned)tid];
  } else {
    v = 0;
    const long long b = a0 + 4 * (long long)tid;
    for (int j = 0; j < 4; ++j)
      if (b + j >= 0 && b + j < span) v |= (uint32_t)base[b + j] << (8 * j);
  }
  ((uint32_t *)dst)[tid] = v;
}

// Byte mask of window row v for the chessboard window (cells u + v even,
// counted from the window's corner, which has the parity of the centre):
// bytes 0 and 2 of every dword in even rows, 1 and 3 in odd rows.
__device__ __forceinline__ uint32_t chess_mask(int chess, int v) {
  return chess ? ((v & 1) ? 0xFF00FF00u : 0x00FF00FFu) : 0xFFFFFFFFu;
}

// Sums over one staged window of L(u) R(u + e) for e = 0, 1, 2, i.e. at the
// disparities o + 1, o, o - 1.  ND dwords hold the win bytes of an L row
// (the bytes past win, and the other chessboard colour, are masked to 0);
// the R row starts at byte rs.
template <int ND>
__device__ __forceinline__ void sp_sums(const uint8_t (*Ls)[SP_LROW], const uint8_t (*Rs)[SP_RROW],
                                        const int *misL, const int *misR, int win, int chess,
                                        int tx, int rs0, int &sp, int &s0, int &sm) {
  const uint32_t lmask = (win & 3) ? (1u << (8 * (win & 3))) - 1u : 0xFFFFFFFFu;
  uint32_t a0 = 0, a1 = 0, a2 = 0;
  for (int v = 0; v < win; ++v) {
    const uint32_t cm = chess_mask(chess, v);
    const int lb = tx + misL[v], rs = rs0 + misR[v];
    const int la = lb & ~3, lsh = lb & 3, ra = rs & ~3, rsh = rs & 3;
    const bool up1 = rsh + 1 >= 4, up2 = rsh + 2 >= 4;
    const int sh1 = (rsh + 1) & 3, sh2 = (rsh + 2) & 3;
    const uint32_t *lw = (const uint32_t *)&Ls[v][la];
    const uint32_t *rw = (const uint32_t *)&Rs[v][ra];
    uint32_t lt[ND + 1], rt[ND + 2];
#pragma unroll
    for (int i = 0; i <= ND; ++i) lt[i] = lw[i];
#pragma unroll
    for (int i = 0; i < ND + 2; ++i) rt[i] = rw[i];
    uint32_t l[ND];
#pragma unroll
    for (int i = 0; i < ND; ++i) l[i] = __builtin_amdgcn_alignbyte(lt[i + 1], lt[i], lsh) & cm;
    l[ND - 1] &= lmask;
    // R windows shifted by e bytes: alignbyte within a dword pair, and the
    // next pair when rsh + e reaches 4
    uint32_t A1[ND + 1], A2[ND + 1];
#pragma unroll
    for (int i = 0; i <= ND; ++i) {
      A1[i] = __builtin_amdgcn_alignbyte(rt[i + 1], rt[i], sh1);
      A2[i] = __builtin_amdgcn_alignbyte(rt[i + 1], rt[i], sh2);
    }
#pragma unroll
    for (int i = 0; i < ND; ++i) {
      a0 = __builtin_amdgcn_udot4(l[i], __builtin_amdgcn_alignbyte(rt[i + 1], rt[i], rsh), a0, false);
      a1 = __builtin_amdgcn_udot4(l[i], up1 ? A1[i + 1] : A1[i], a1, false);
      a2 = __builtin_amdgcn_udot4(l[i], up2 ? A2[i + 1] : A2[i], a2, false);
    }
  }
  sp = (int)a0;
  s0 = (int)a1;
  sm = (int)a2;
}

template <bool B>
__global__ __launch_bounds__(SP_TX) void subpixel_kernel(PostPair one, const PostPair *__restrict__ many) {
  PAIR;
  __shared__ __align__(16) uint8_t Ls[SP_MAXWIN][SP_LROW];
  __shared__ __align__(16) uint8_t Rs[SP_MAXWIN][SP_RROW];
  __shared__ int s_omin, s_omax, misL[SP_MAXWIN], misR[SP_MAXWIN];
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
    // Ls[r][misL[r] + c] = L(y-h+r, x0-h+c), Rs[r][misR[r] + c] = R(y-h+r, x0-omax-1-h+c).
    // Bytes of columns outside the image only enter sums whose z is
    // discarded (a valid pixel's windows at o lie inside the image).
    const int LW = SP_TX + 2 * h, RW = SP_TX + (omax - omin) + 2 + 2 * h;
    const int lx0 = x0 - h, rx0 = x0 - omax - 1 - h;
    const GLOBAL uint8_t *Lg = gro(P.left), *Rg = gro(P.right);
    const long long span = (long long)(H - 1) * P.pitch + W;
#pragma unroll
    for (int r = 0; r < SP_MAXWIN; ++r) {
      if (r < win) {
        const long long row = (long long)(y - h + r) * P.pitch;  // inside: the block has a valid pixel
        stage_row(Ls[r], Lg, row + lx0, LW, span, tx);
        stage_row(Rs[r], Rg, row + rx0, RW, span, tx);
        if (tx == 0) {
          misL[r] = (int)(((uintptr_t)Lg + (uintptr_t)(row + lx0)) & 3);
          misR[r] = (int)(((uintptr_t)Rg + (uintptr_t)(row + rx0)) & 3);
        }
      }
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
  // window column u of the thread at d = o + 1 - e is Rs[v][rs + e + u]
  const int rs = tx + omax - o;
  int sm = 0, s0 = 0, sp = 0;  // sums at d = o - 1, o, o + 1
  switch ((win + 3) >> 2) {
    case 1: sp_sums<1>(Ls, Rs, misL, misR, win, P.chess, tx, rs, sp, s0, sm); break;
    case 2: sp_sums<2>(Ls, Rs, misL, misR, win, P.chess, tx, rs, sp, s0, sm); break;
    case 3: sp_sums<3>(Ls, Rs, misL, misR, win, P.chess, tx, rs, sp, s0, sm); break;
    default: sp_sums<4>(Ls, Rs, misL, misR, win, P.chess, tx, rs, sp, s0, sm); break;
  }
  const long long n = P.chess ? ((long long)win * win + 1) / 2 : (long long)win * win;
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
__global__ void lr_check_kernel(PostPair one, const PostPair *__restrict__ many, int tol, int dst) {
  PAIR;
  const int W = P.W, H = P.H;
  (void)W;
  (void)H;
  for_pixels(P, [&](int x, int y, size_t k) {
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
  });
}


// ---------------------------------------------------------------- radial line scans
// The 8 radial directions come in 4 line types: rows, columns, diagonals
// (x - y const) and anti-diagonals (x + y const), each a pair of opposite
// directions.  Per pixel and direction the scans give
//   outlier: whether the r steps from the pixel all land on valid pixels,
//            each within thresh of the previous one (plane pass[t], bit 0
//            forward, bit 1 backward);
//   fill:    the nearest valid pixel within R steps, as (steps << 16) |
//            uint16 disparity, 0 when there is none (planes hits[2t],
//            hits[2t+1]).
// Rows: a wave covers 64 columns of a row, lanes are columns, and ballot
// masks give the next break or valid pixel; the look-ahead runs over the
// following 64-column blocks until every lane is settled.  Columns and
// diagonals: a thread scans SEG rows of one line (plus the look-ahead) and
// the lanes of a wave are neighbouring lines, so each step reads
// consecutive columns of one row.
constexpr int SEG = 32;

__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }
__device__ __forceinline__ int ctz64(uint64_t v) { return __builtin_ctzll(v); }
__device__ __forceinline__ int top64(uint64_t v) { return 63 - __builtin_clzll(v); }

// forward / backward step failure of the outlier test at column p of a row:
// the neighbour is outside, invalid or too far in disparity
__device__ __forceinline__ bool step_breaks(const GLOBAL int16_t *o, const GLOBAL uint8_t *m, int p,
                                            int q, int W, float thresh) {
  if (q < 0 || q >= W || p < 0 || p >= W) return true;
  if (!m[q]) return true;
  const int dv = o[q] - o[p];
  return !((float)(dv < 0 ? -dv : dv) < thresh);
}

template <bool B>
__global__ __launch_bounds__(256) void outlier_rows_kernel(PostPair one, const PostPair *__restrict__ many, int r,
                                                          float thresh, int src) {
  PAIR;
  const int H = P.H, W = P.W;
  // a block holds 4 waves, one row each (no block-level synchronisation)
  const int lane = threadIdx.x & 63, y = blockIdx.y * 4 + (threadIdx.x >> 6), xb = blockIdx.x * 64;
  if (y >= H || xb >= W) return;  // whole wave
  const GLOBAL int16_t *o = gro(P.ob[src]) + (size_t)y * W;
  const GLOBAL uint8_t *m = gro(P.mb[src]) + (size_t)y * W;
  const int x = xb + lane;
  // forward: distance to the first break at or after x must reach r
  int df = 0;
  bool open = true;
  for (int k = 0; ; ++k) {
    const int p0 = xb + 64 * k;
    const uint64_t bm = ballot64(step_breaks(o, m, p0 + lane, p0 + lane + 1, W, thresh));
    if (open) {
      const uint64_t rest = k == 0 ? bm >> lane << lane : bm;  // breaks at >= x
      if (rest) { df = p0 + ctz64(rest) - x; open = false; }
      else if (p0 + 64 - x >= r) { df = r; open = false; }
    }
    if (!__any(open)) break;
  }
  // backward: distance from the last break at or before x
  int db = 0;
  open = true;
  for (int k = 0; ; ++k) {
    const int p0 = xb - 64 * k;
    const uint64_t bm = ballot64(step_breaks(o, m, p0 + lane, p0 + lane - 1, W, thresh));
    if (open) {
      const uint64_t low = k == 0 ? (lane == 63 ? bm : bm & ((2ull << lane) - 1)) : bm;  // <= x
      if (low) { db = x - (p0 + top64(low)); open = false; }
      else if (x - (p0 - 1) >= r) { db = r; open = false; }
    }
    if (!__any(open)) break;
  }
  if (x < W && m[x]) P.pass[(size_t)y * W + x] = (df >= r ? 1 : 0) | (db >= r ? 2 : 0);
}

template <bool B>
__global__ __launch_bounds__(256) void fill_rows_kernel(PostPair one, const PostPair *__restrict__ many, int R,
                                                       int src) {
  PAIR;
  const int H = P.H, W = P.W;
  // a block holds 4 waves, one row each (no block-level synchronisation)
  const int lane = threadIdx.x & 63, y = blockIdx.y * 4 + (threadIdx.x >> 6), xb = blockIdx.x * 64;
  if (y >= H || xb >= W) return;  // whole wave
  const GLOBAL int16_t *o = gro(P.ob[src]) + (size_t)y * W;
  const GLOBAL uint8_t *m = gro(P.mb[src]) + (size_t)y * W;
  const int x = xb + lane;
  int qf = -1, qb = -1;
  bool open = true;
  for (int k = 0; ; ++k) {
    const int p0 = xb + 64 * k, p = p0 + lane;
    const uint64_t vm = ballot64(p < W && m[p]);
    if (open) {
      const uint64_t rest = k == 0 ? (lane == 63 ? 0ull : vm >> (lane + 1) << (lane + 1)) : vm;  // > x
      if (rest) { qf = p0 + ctz64(rest); open = false; }
      else if (p0 + 64 - x > R || p0 + 64 >= W) open = false;
    }
    if (!__any(open)) break;
  }
  open = true;
  for (int k = 0; ; ++k) {
    const int p0 = xb - 64 * k, p = p0 + lane;
    const uint64_t vm = ballot64(p >= 0 && p < W && m[p]);
    if (open) {
      const uint64_t low = k == 0 ? vm & ((1ull << lane) - 1) : vm;  // < x
      if (low) { qb = p0 + top64(low); open = false; }
      else if (x - (p0 - 1) > R || p0 <= 0) open = false;
    }
    if (!__any(open)) break;
  }
  if (x >= W || m[x]) return;
  const size_t N = (size_t)W * H, k = (size_t)y * W + x;
  P.hits[k] = (qf >= 0 && qf - x <= R) ? ((uint32_t)(qf - x) << 16) | (uint16_t)o[qf] : 0u;
  P.hits[N + k] = (qb >= 0 && x - qb <= R) ? ((uint32_t)(x - qb) << 16) | (uint16_t)o[qb] : 0u;
}

// Columns (t = 1), diagonals (t = 2, x = y + l - (H-1)) and anti-diagonals
// (t = 3, x = l - y), stepped in increasing y.  Line l crosses rows
// [ylo, yhi); its pixel in row y has the flat index y * (W + dx) + c0.
struct VLine {
  int ylo, yhi, st, c0;
};
__device__ __forceinline__ VLine vline(int t, int l, int H, int W) {
  VLine v;
  if (t == 1) { v.ylo = 0; v.yhi = H; v.st = W; v.c0 = l; }
  else if (t == 2) {
    const int c = l - (H - 1);
    v.ylo = max(0, -c); v.yhi = min(H, W - c); v.st = W + 1; v.c0 = c;
  } else {
    v.ylo = max(0, l - (W - 1)); v.yhi = min(H, l + 1); v.st = W - 1; v.c0 = l;
  }
  return v;
}
__device__ __forceinline__ int vlines(int t, int H, int W) { return t == 1 ? W : W + H - 1; }

// Thread index -> (line type 1..3, line, row segment); false past the end.
__device__ __forceinline__ bool vscan_task(int idx, int H, int W, int &t, int &l, int &sg) {
  const int ns = ceil_div(H, SEG);
  for (t = 1; t < 4; ++t) {
    const int nl = vlines(t, H, W);
    if (idx < nl * ns) {
      sg = idx / nl;
      l = idx - sg * nl;
      return true;
    }
    idx -= nl * ns;
  }
  return false;
}

// Each scan first runs through the look-ahead rows (state only), then through
// its own rows, writing results only where a later kernel reads them: pass
// for valid pixels, hits for holes.  The loops are branch-free so that the
// loads of an unrolled group issue together.
template <bool B>
__global__ void outlier_vscan_kernel(PostPair one, const PostPair *__restrict__ many, int r,
                                     float thresh, int src) {
  PAIR;
  const int H = P.H, W = P.W;
  int t, l, sg;
  if (!vscan_task(blockIdx.x * blockDim.x + threadIdx.x, H, W, t, l, sg)) return;
  const VLine L = vline(t, l, H, W);
  const int a = max(L.ylo, sg * SEG), b = min(L.yhi, sg * SEG + SEG);
  if (a >= b) return;
  const GLOBAL int16_t *__restrict__ o = gro(P.ob[src]);
  const GLOBAL uint8_t *__restrict__ m = gro(P.mb[src]);
  GLOBAL uint8_t *__restrict__ pass = grw(P.pass) + (size_t)t * W * H;
  // run = consecutive good steps from y along the scan direction, capped at r
  auto step = [&](int op, int onb, bool vnb, int run) {
    const int dv = onb - op;
    const bool good = vnb & ((float)(dv < 0 ? -dv : dv) < thresh);
    return good ? min(run + 1, r) : 0;
  };
  {  // forward (+y), walked from the end of the look-ahead back to a
    const int e = min(L.yhi - 1, b - 1 + r);
    int k = e * L.st + L.c0;
    int on = o[k], run = 0;
    bool vn = m[k] != 0;
    if (e < b && vn) pass[k] = 0;
    int y = e - 1;
    k -= L.st;
#pragma unroll 8
    for (; y >= b; --y, k -= L.st) {
      const int op = o[k];
      const bool v = m[k] != 0;
      run = step(op, on, vn, run);
      on = op;
      vn = v;
    }
#pragma unroll 8
    for (; y >= a; --y, k -= L.st) {
      const int op = o[k];
      const bool v = m[k] != 0;
      run = step(op, on, vn, run);
      on = op;
      vn = v;
      if (v) pass[k] = run >= r ? 1 : 0;
    }
  }
  {  // backward (-y); when e == a the first row has no step (run 0 < r)
    const int e = max(L.ylo, a - r);
    int k = e * L.st + L.c0;
    int on = o[k], run = 0;
    bool vn = m[k] != 0;
    int y = e + 1;
    k += L.st;
#pragma unroll 8
    for (; y < a; ++y, k += L.st) {
      const int op = o[k];
      const bool v = m[k] != 0;
      run = step(op, on, vn, run);
      on = op;
      vn = v;
    }
#pragma unroll 8
    for (; y < b; ++y, k += L.st) {
      const int op = o[k];
      const bool v = m[k] != 0;
      run = step(op, on, vn, run);
      on = op;
      vn = v;
      if (v && run >= r) pass[k] |= 2;
    }
  }
}

template <bool B>
__global__ void fill_vscan_kernel(PostPair one, const PostPair *__restrict__ many, int R, int src) {
  PAIR;
  const int H = P.H, W = P.W;
  int t, l, sg;
  if (!vscan_task(blockIdx.x * blockDim.x + threadIdx.x, H, W, t, l, sg)) return;
  const VLine L = vline(t, l, H, W);
  const int a = max(L.ylo, sg * SEG), b = min(L.yhi, sg * SEG + SEG);
  if (a >= b) return;
  const GLOBAL int16_t *__restrict__ o = gro(P.ob[src]);
  const GLOBAL uint8_t *__restrict__ m = gro(P.mb[src]);
  const size_t N = (size_t)W * H;
  GLOBAL uint32_t *__restrict__ hf = grw(P.hits) + (size_t)(2 * t) * N;
  GLOBAL uint32_t *__restrict__ hb = grw(P.hits) + (size_t)(2 * t + 1) * N;
  {  // nearest valid pixel in +y
    const int e = min(L.yhi - 1, b - 1 + R);
    int q = -1;
    uint32_t vq = 0;
    int y = e, k = e * L.st + L.c0;
#pragma unroll 8
    for (; y >= b; --y, k -= L.st) {
      const bool v = m[k] != 0;
      const uint32_t ov = (uint16_t)o[k];
      q = v ? y : q;
      vq = v ? ov : vq;
    }
#pragma unroll 8
    for (; y >= a; --y, k -= L.st) {
      const bool v = m[k] != 0;
      const uint32_t ov = (uint16_t)o[k];
      if (!v) hf[k] = (q >= 0 && q - y <= R) ? ((uint32_t)(q - y) << 16) | vq : 0u;
      q = v ? y : q;
      vq = v ? ov : vq;
    }
  }
  {  // nearest valid pixel in -y
    const int e = max(L.ylo, a - R);
    int q = -1;
    uint32_t vq = 0;
    int y = e, k = e * L.st + L.c0;
#pragma unroll 8
    for (; y < a; ++y, k += L.st) {
      const bool v = m[k] != 0;
      const uint32_t ov = (uint16_t)o[k];
      q = v ? y : q;
      vq = v ? ov : vq;
    }
#pragma unroll 8
    for (; y < b; ++y, k += L.st) {
      const bool v = m[k] != 0;
      const uint32_t ov = (uint16_t)o[k];
      if (!v) hb[k] = (q >= 0 && y - q <= R) ? ((uint32_t)(y - q) << 16) | vq : 0u;
      q = v ? y : q;
      vq = v ? ov : vq;
    }
  }
}

// A valid pixel stays when some direction passes (Section II-B).
template <bool B>
__global__ void outlier_combine_kernel(PostPair one, const PostPair *__restrict__ many, int src, int dst) {
  PAIR;
  const int W = P.W, H = P.H;
  (void)W;
  (void)H;
  for_pixels(P, [&](int x, int y, size_t k) {
    const size_t N = (size_t)W * H;
    const uint8_t mk = P.mb[src][k];
    P.ob[dst][k] = P.ob[src][k];
    const bool any = (P.pass[k] | P.pass[N + k] | P.pass[2 * N + k] | P.pass[3 * N + k]) != 0;
    P.mb[dst][k] = (mk && any) ? mk : 0;
  });
}

// (i) radial fill from the scanned hits: complete lines (both opposite
// directions hit) give (va*sb + vb*sa)/(sa+sb); with >= min_lines complete
// lines the hole takes their mean, an exact rational rounded half to even;
// code 2.  Fused with the row prefix sums of the result that the disk fill
// reads: pc[y][x+1] = number of valid pixels x' <= x in row y, ps[y][x+1]
// the sum of their disparities.  One block per row; the row goes in chunks
// of 256 columns with a block scan (wave scans plus wave totals in LDS).
template <bool B>
__global__ __launch_bounds__(256) void fill_radial_kernel(PostPair one, const PostPair *__restrict__ many,
                                                          int min_lines, int src, int dst) {
  PAIR;
  __shared__ int wc[4], wsum[4];
  const int y = blockIdx.x;
  if (y >= P.H) return;  // uniform per block
  const int W = P.W, H = P.H, t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const size_t N = (size_t)W * H;
  const GLOBAL int16_t *o = gro(P.ob[src]);
  const GLOBAL uint8_t *m = gro(P.mb[src]);
  const GLOBAL uint32_t *hits = gro(P.hits);
  GLOBAL int32_t *pcr = grw(P.pc) + (size_t)y * (W + 1);
  GLOBAL int32_t *psr = grw(P.ps) + (size_t)y * (W + 1);
  if (t == 0) {
    pcr[0] = 0;
    psr[0] = 0;
  }
  int carry_c = 0, carry_s = 0;
  for (int x0 = 0; x0 < W; x0 += 256) {
    const int x = x0 + t;
    int ov = 0, mv = 0;
    if (x < W) {
      const size_t k = (size_t)y * W + x;
      ov = o[k];
      mv = m[k];
      if (!mv) {
        long long num = 0, den = 1;
        int lines = 0;
        for (int ln = 0; ln < 4; ++ln) {
          const uint32_t ha = hits[(size_t)(2 * ln) * N + k], hb = hits[(size_t)(2 * ln + 1) * N + k];
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
          ov = (int)round_half_even(num, den * lines);
          mv = 2;
        }
      }
      grw(P.ob[dst])[k] = (int16_t)ov;
      grw(P.mb[dst])[k] = (uint8_t)mv;
    }
    int c = mv ? 1 : 0, sv = mv ? ov : 0;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int uc = __shfl_up(c, off, 64), us = __shfl_up(sv, off, 64);
      if (lane >= off) {
        c += uc;
        sv += us;
      }
    }
    if (lane == 63) {
      wc[wave] = c;
      wsum[wave] = sv;
    }
    __syncthreads();
    int bc = carry_c, bs = carry_s;
    for (int w = 0; w < wave; ++w) {
      bc += wc[w];
      bs += wsum[w];
    }
    if (x < W) {
      pcr[x + 1] = bc + c;
      psr[x + 1] = bs + sv;
    }
    for (int w = 0; w < 4; ++w) {
      carry_c += wc[w];
      carry_s += wsum[w];
    }
    __syncthreads();  // wc / wsum are rewritten by the next chunk
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
// Disk sums come from the row prefix sums, one segment per disk row; the
// half-widths floor(sqrt(R^2 - dy^2)) of the disk rows are tabulated once
// per block (for |dy| <= DISK_TAB) instead of per pixel and row.
constexpr int DISK_TAB = 512;

template <bool B>
__global__ __launch_bounds__(PIX_T) void fill_disk_kernel(PostPair one, const PostPair *__restrict__ many, int R,
                                                        float frac, int src, int dst) {
  PAIR;
  __shared__ int hw[2 * DISK_TAB + 1];
  const int RT = min(R, DISK_TAB);
  for (int i = threadIdx.x; i <= 2 * RT; i += blockDim.x) {
    const int dy = i - RT;
    hw[i] = isqrt_floor(R * R - dy * dy);
  }
  __syncthreads();
  const int W = P.W, H = P.H;
  (void)W;
  (void)H;
  for_pixels(P, [&](int x, int y, size_t k) {
    const GLOBAL int16_t *o = gro(P.ob[src]);
    const GLOBAL uint8_t *m = gro(P.mb[src]);
    grw(P.ob[dst])[k] = o[k];
    grw(P.mb[dst])[k] = m[k];
    if (m[k]) return;
    long long cells = 0, cnt = 0, sum = 0;
    const int ya = max(-R, -y), yb = min(R, H - 1 - y);
    const GLOBAL int32_t *__restrict__ pc = gro(P.pc);
    const GLOBAL int32_t *__restrict__ ps = gro(P.ps);
#pragma unroll 8
    for (int dy = ya; dy <= yb; ++dy) {
      const int qy = y + dy;
      const int w = (dy >= -RT && dy <= RT) ? hw[dy + RT] : isqrt_floor(R * R - dy * dy);
      const int xl = max(0, x - w), xh = min(W - 1, x + w);
      cells += xh - xl + 1;
      const size_t rb = (size_t)qy * (W + 1);
      cnt += pc[rb + xh + 1] - pc[rb + xl];
      sum += ps[rb + xh + 1] - ps[rb + xl];
    }
    const double need = ceil((double)frac * (double)cells);
    if (cnt > 0 && (double)cnt >= need) {
      grw(P.ob[dst])[k] = (int16_t)round_half_even(sum, cnt);
      grw(P.mb[dst])[k] = 2;
    }
  });
}

// ---------------------------------------------------------------- smoothing (FP64)
// Planes of P.f: 0 s, 1 s*m / b, 2 box(m), 3 column pass, 4 a = A(s), 5 d.
enum { F_S = 0, F_IN = 1, F_CNT = 2, F_TMP = 3, F_A = 4, F_D = 5 };

// s = o + delta for matched pixels (code 1), o for filled ones (code 2), or
// the given s_in; plane F_IN <- s*m, F_D <- m (ones, used for the counts).
__device__ __forceinline__ double hc_s_at(const PostPair &P, size_t k, uint8_t mk, int osrc,
                                          int use_delta) {
  if (P.s_in) return (double)gro(P.s_in)[k];
  const double o = (double)gro(P.ob[osrc])[k];
  return (mk == 1 && use_delta) ? o + (double)gro(P.delta)[k] : o;
}

template <bool B>
__global__ void hc_init_kernel(PostPair one, const PostPair *__restrict__ many, int src, int osrc,
                               int use_delta, int counts) {
  PAIR;
  const int W = P.W, H = P.H;
  (void)W;
  (void)H;
  for_pixels(P, [&](int x, int y, size_t k) {
    const size_t N = (size_t)W * H;
    const uint8_t mk = P.mb[src][k];
    const double v = mk ? hc_s_at(P, k, mk, osrc, use_delta) : 0.0;
    P.f[F_S * N + k] = v;
    P.f[F_IN * N + k] = v;
    if (counts) P.f[F_D * N + k] = mk ? 1.0 : 0.0;
  });
}

// Box sums over a (2R+1) window along columns: a thread owns one column and
// a segment of seg rows, seeds the window sum, then slides it.
template <bool B>
__global__ void box_v_kernel(PostPair one, const PostPair *__restrict__ many, int R, int seg, int in, int out) {
  PAIR;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y0 = blockIdx.y * seg;
  const int H = P.H, W = P.W;
  if (x >= W || y0 >= H) return;
  const size_t N = (size_t)W * H;
  const GLOBAL double *__restrict__ fi = gro(P.f) + in * N;
  GLOBAL double *__restrict__ fo = grw(P.f) + out * N;
  double s = 0.0;
  const int va = max(0, y0 - R), vb = min(H - 1, y0 + R);
#pragma unroll 8
  for (int v = va; v <= vb; ++v) s += fi[(size_t)v * W + x];
  const int y1 = min(y0 + seg, H);
#pragma unroll 4
  for (int y = y0; y < y1; ++y) {
    fo[(size_t)y * W + x] = s;
    const int a = y + R + 1, b = y - R;
    const double ea = a < H ? fi[(size_t)a * W + x] : 0.0;
    const double eb = b >= 0 ? fi[(size_t)b * W + x] : 0.0;
    s += ea;
    s -= eb;
  }
}

// Output stage of a row box pass: the plain box sum (mode 0), or the masked
// mean steps fused into it: mode 1 a = box(s m)/box(m) (Eq. 1), mode 2
// d = a - box(b m)/box(m) (Eq. 3), mode 3 the same d written as the final
// disparity (NaN where invalid) and mask.
__device__ __forceinline__ void box_store(const PostPair &P, int mode, int src, int out, size_t N,
                                          size_t k, double v) {
  if (mode == 0) {
    P.f[(size_t)out * N + k] = v;
    return;
  }
  const uint8_t mk = P.mb[src][k];
  const double mean = v / P.f[(size_t)F_CNT * N + k];
  if (mode == 1) {
    P.f[(size_t)F_A * N + k] = mk ? mean : 0.0;
  } else {
    const double d = mk ? P.f[(size_t)F_A * N + k] - mean : 0.0;
    if (mode == 2) {
      P.f[(size_t)F_D * N + k] = d;
    } else {
      P.disparity[k] = mk ? (float)d : __builtin_nanf("");
      if (P.valid_mask) P.valid_mask[k] = mk;
    }
  }
}

template <bool B>
__global__ void box_h_kernel(PostPair one, const PostPair *__restrict__ many, int R, int seg, int in, int out,
                             int mode, int src) {
  PAIR;
  const int y = blockIdx.x * blockDim.x + threadIdx.x;
  const int x0 = blockIdx.y * seg;
  const int H = P.H, W = P.W;
  if (y >= H || x0 >= W) return;
  const size_t N = (size_t)W * H;
  const double *row = P.f + in * N + (size_t)y * W;
  double s = 0.0;
  for (int u = x0 - R; u <= x0 + R; ++u)
    if (u >= 0 && u < W) s += row[u];
  const int x1 = min(x0 + seg, W);
  for (int x = x0; x < x1; ++x) {
    box_store(P, mode, src, out, N, (size_t)y * W + x, s);
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
__global__ __launch_bounds__(256) void box_h_lds_kernel(PostPair one, const PostPair *__restrict__ many, int R,
                                                        int in, int out, int mode, int src) {
  PAIR;
  __shared__ double row[BOXH_MAXW];
  __shared__ double part[256];
  const int y = blockIdx.x;
  const int H = P.H, W = P.W;
  if (y >= H) return;
  const size_t N = (size_t)W * H;
  const double *rin = P.f + in * N + (size_t)y * W;
  const int t = threadIdx.x;
  for (int x = t; x < W; x += 256) row[x] = rin[x];
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
    box_store(P, mode, src, out, N, (size_t)y * W + x, row[a] - (b >= 0 ? row[b] : 0.0));
  }
}

// ---- Eq. (4): re-search of the discrete disparities around d.  A block
// covers 128 pixels of a row and stages, as the sub-pixel kernel does, the
// L window rows and the R columns of every candidate of the block; each
// candidate's window sum is exact (v_dot4_u32_u8), z and the cost in FP64.
template <int ND>
__device__ __forceinline__ int sp_sum1(const uint8_t (*Ls)[SP_LROW], const uint8_t (*Rs)[SP_RROW],
                                       const int *misL, const int *misR, int win, int chess, int tx,
                                       int rs0) {
  const uint32_t lmask = (win & 3) ? (1u << (8 * (win & 3))) - 1u : 0xFFFFFFFFu;
  uint32_t acc = 0;
  for (int v = 0; v < win; ++v) {
    const uint32_t cm = chess_mask(chess, v);
    const int lb = tx + misL[v], rs = rs0 + misR[v];
    const uint32_t *lw = (const uint32_t *)&Ls[v][lb & ~3];
    const uint32_t *rw = (const uint32_t *)&Rs[v][rs & ~3];
    uint32_t lt[ND + 1], rt[ND + 1];
#pragma unroll
    for (int i = 0; i <= ND; ++i) {
      lt[i] = lw[i];
      rt[i] = rw[i];
    }
#pragma unroll
    for (int i = 0; i < ND; ++i) {
      uint32_t l = __builtin_amdgcn_alignbyte(lt[i + 1], lt[i], lb & 3) & cm;
      if (i == ND - 1) l &= lmask;
      acc = __builtin_amdgcn_udot4(l, __builtin_amdgcn_alignbyte(rt[i + 1], rt[i], rs & 3), acc, false);
    }
  }
  return (int)acc;
}

template <bool B>
__global__ __launch_bounds__(SP_TX) void research_kernel(PostPair one, const PostPair *__restrict__ many,
                                                         int osrc, int msrc, int odst, int dplane,
                                                         int range, double eta) {
  PAIR;
  __shared__ __align__(16) uint8_t Ls[SP_MAXWIN][SP_LROW];
  __shared__ __align__(16) uint8_t Rs[SP_MAXWIN][SP_RROW];
  __shared__ int s_cmin, s_cmax, misL[SP_MAXWIN], misR[SP_MAXWIN];
  const int tx = threadIdx.x;
  const int x0 = blockIdx.x * SP_TX, y = blockIdx.y;
  if (x0 >= P.W || y >= P.H) return;  // uniform per block
  const int W = P.W, H = P.H, win = P.win, h = win / 2;
  const int x = x0 + tx;
  const size_t N = (size_t)W * H, k = (size_t)y * W + x;
  // pixels whose own window is inside the image can have a defined candidate
  const bool inside = x < W && x >= h && x <= W - 1 - h && y >= h && y <= H - 1 - h;
  const uint8_t mk = x < W ? P.mb[msrc][k] : 0;
  const double d = mk ? P.f[(size_t)dplane * N + k] : 0.0;
  int lo = 0, hi = -1;
  if (mk && inside) {
    lo = max(max(P.dmin, (int)ceil(d - range)), x - (W - 1 - h));
    hi = min(min(P.dmax, (int)floor(d + range)), x - h);
  }
  if (tx == 0) {
    s_cmin = 1 << 30;
    s_cmax = -(1 << 30);
  }
  __syncthreads();
  if (lo <= hi) {
    atomicMin(&s_cmin, lo);
    atomicMax(&s_cmax, hi);
  }
  __syncthreads();
  const int cmin = s_cmin, cmax = s_cmax;
  if (cmin <= cmax) {
    // Ls[r][misL[r] + c] = L(y-h+r, x0-h+c), Rs[r][misR[r] + c] = R(y-h+r, x0-cmax-h+c)
    const int LW = SP_TX + 2 * h, RW = SP_TX + (cmax - cmin) + 2 * h;
    const int lx0 = x0 - h, rx0 = x0 - cmax - h;
    const GLOBAL uint8_t *Lg = gro(P.left), *Rg = gro(P.right);
    const long long span = (long long)(H - 1) * P.pitch + W;
#pragma unroll
    for (int r = 0; r < SP_MAXWIN; ++r) {
      if (r < win) {  // rows inside: the block has an inside pixel
        const long long row = (long long)(y - h + r) * P.pitch;
        stage_row(Ls[r], Lg, row + lx0, LW, span, tx);
        stage_row(Rs[r], Rg, row + rx0, RW, span, tx);
        if (tx == 0) {
          misL[r] = (int)(((uintptr_t)Lg + (uintptr_t)(row + lx0)) & 3);
          misR[r] = (int)(((uintptr_t)Rg + (uintptr_t)(row + rx0)) & 3);
        }
      }
    }
  }
  __syncthreads();
  if (x >= W) return;
  int onew = P.ob[osrc][k];
  if (lo <= hi) {
    const long long n = P.chess ? ((long long)win * win + 1) / 2 : (long long)win * win;
    const long long sl = P.SL[k];
    const long long varL = n * (long long)P.SSL[k] - sl * sl;
    if (varL > 0) {
      double best = __builtin_inf();
      const int nd = (win + 3) >> 2;
      for (int c = lo; c <= hi; ++c) {
        const size_t kr = (size_t)y * W + (x - c);
        const long long sr = P.SR[kr];
        const long long varR = n * (long long)P.SSR[kr] - sr * sr;
        if (varR <= 0) continue;
        const int rs0 = tx + cmax - c;  // window column 0 of candidate c in Rs
        int slr;
        switch (nd) {
          case 1: slr = sp_sum1<1>(Ls, Rs, misL, misR, win, P.chess, tx, rs0); break;
          case 2: slr = sp_sum1<2>(Ls, Rs, misL, misR, win, P.chess, tx, rs0); break;
          case 3: slr = sp_sum1<3>(Ls, Rs, misL, misR, win, P.chess, tx, rs0); break;
          default: slr = sp_sum1<4>(Ls, Rs, misL, misR, win, P.chess, tx, rs0); break;
        }
        const double z = (double)(n * (long long)slr - sl * sr) / sqrt((double)varL * (double)varR);
        const double e = (double)c - d;
        const double cost = 1.0 / (z > 1e-3 ? z : 1e-3) + eta * e * e;
        if (cost < best) {
          best = cost;
          onew = c;
        }
      }
    }
  }
  P.ob[odst][k] = (int16_t)onew;
}

// Output without smoothing (K = 0): s on valid pixels.
template <bool B>
__global__ void hc_copy_kernel(PostPair one, const PostPair *__restrict__ many, int src, int osrc,
                               int use_delta) {
  PAIR;
  const int W = P.W, H = P.H;
  (void)W;
  (void)H;
  for_pixels(P, [&](int x, int y, size_t k) {
    const uint8_t mk = P.mb[src][k];
    P.disparity[k] = mk ? (float)hc_s_at(P, k, mk, osrc, use_delta) : __builtin_nanf("");
    if (P.valid_mask) P.valid_mask[k] = mk;
  });
}


// b = a - alpha*s - (1-alpha)*d_prev on valid pixels, 0 elsewhere (Eq. 2);
// d_prev is s in the first iteration.
template <bool B>
__global__ void hc_b_kernel(PostPair one, const PostPair *__restrict__ many, int src, double alpha, int first) {
  PAIR;
  const int W = P.W, H = P.H;
  (void)W;
  (void)H;
  for_pixels(P, [&](int x, int y, size_t k) {
    const size_t N = (size_t)W * H;
    const double s = P.f[F_S * N + k];
    const double dp = first ? s : P.f[F_D * N + k];
    P.f[F_IN * N + k] = P.mb[src][k] ? P.f[F_A * N + k] - alpha * s - (1.0 - alpha) * dp : 0.0;
  });
}



// ---------------------------------------------------------------- host side
static inline dim3 pixgrid(const PostLaunch &L) { return dim3(ceil_div(L.maxW, PIX_SEG), L.maxH, L.npairs); }

#define LAUNCH(kern, grid, block, ...)                                                   \
  do {                                                                                   \
    if (L.many)                                                                          \
      hipLaunchKernelGGL(kern<true>, grid, block, 0, L.s, L.one, L.many, ##__VA_ARGS__); \
    else                                                                                 \
      hipLaunchKernelGGL(kern<false>, grid, block, 0, L.s, L.one, L.many, ##__VA_ARGS__); \
  } while (0)

hipError_t post_decode(const PostLaunch &L) {
  LAUNCH(decode_kernel, pixgrid(L), dim3(PIX_T));
  return hipGetLastError();
}
hipError_t post_subpixel(const PostLaunch &L) {
  LAUNCH(subpixel_kernel, dim3(ceil_div(L.maxW, SP_TX), L.maxH, L.npairs), dim3(SP_TX));
  return hipGetLastError();
}
hipError_t post_lr(const PostLaunch &L, int tol, int dst) {
  LAUNCH(lr_check_kernel, pixgrid(L), dim3(PIX_T), tol, dst);
  return hipGetLastError();
}
static dim3 rowgrid(const PostLaunch &L) { return dim3(ceil_div(L.maxW, 64), ceil_div(L.maxH, 4), L.npairs); }
static dim3 vscangrid(const PostLaunch &L) {
  const int n = (L.maxW + 2 * (L.maxW + L.maxH - 1)) * ceil_div(L.maxH, SEG);
  return dim3(ceil_div(n, 256), 1, L.npairs);
}

hipError_t post_outlier(const PostLaunch &L, int r, float thresh, int src, int dst) {
  LAUNCH(outlier_rows_kernel, rowgrid(L), dim3(256), r, thresh, src);
  LAUNCH(outlier_vscan_kernel, vscangrid(L), dim3(256), r, thresh, src);
  LAUNCH(outlier_combine_kernel, pixgrid(L), dim3(PIX_T), src, dst);
  return hipGetLastError();
}
// radial fill src -> tmp, disk fill tmp -> dst (dst may equal src)
hipError_t post_fill(const PostLaunch &L, int radial_r, int min_lines, int disk_r, float frac,
                     int src, int tmp, int dst) {
  LAUNCH(fill_rows_kernel, rowgrid(L), dim3(256), radial_r, src);
  LAUNCH(fill_vscan_kernel, vscangrid(L), dim3(256), radial_r, src);
  LAUNCH(fill_radial_kernel, dim3(L.maxH, 1, L.npairs), dim3(256), min_lines, src, tmp);
  LAUNCH(fill_disk_kernel, pixgrid(L), dim3(PIX_T), disk_r, frac, tmp, dst);
  return hipGetLastError();
}

// Box sum over the (2R+1)^2 window of plane `in`, stored by box_store's mode.
static void box2d(const PostLaunch &L, int R, int in, int out, int mode = 0, int src = 0) {
  const int seg = 32;
  LAUNCH(box_v_kernel, dim3(ceil_div(L.maxW, 64), ceil_div(L.maxH, seg), L.npairs), dim3(64), R,
         seg, in, F_TMP);
  if (L.maxW <= BOXH_MAXW)
    LAUNCH(box_h_lds_kernel, dim3(L.maxH, 1, L.npairs), dim3(256), R, F_TMP, out, mode, src);
  else
    LAUNCH(box_h_kernel, dim3(ceil_div(L.maxH, 64), ceil_div(L.maxW, seg), L.npairs), dim3(64), R,
           seg, F_TMP, out, mode, src);
}

// Improved Laplacian smoothing of (ob[src], delta, mb[src]) or s_in; writes
// disparity (NaN where invalid) and valid_mask.
hipError_t post_research(const PostLaunch &L, int osrc, int msrc, int odst, int dplane, int range,
                         float eta) {
  LAUNCH(research_kernel, dim3(ceil_div(L.maxW, SP_TX), L.maxH, L.npairs), dim3(SP_TX), osrc, msrc,
         odst, dplane, range, (double)eta);
  return hipGetLastError();
}

hipError_t post_hc(const PostLaunch &L, int src, int R, int K, float alpha, int use_delta,
                   int research, int range, float eta) {
  if (K == 0) {
    LAUNCH(hc_copy_kernel, pixgrid(L), dim3(PIX_T), src, src, use_delta);
    return hipGetLastError();
  }
  // research: Eqs. (1)-(4), the discrete o (no sub-pixel offset) is smoothed
  // and re-searched after every iteration but the last; o ping-pongs between
  // the two fill planes while the mask stays in plane src
  int ocur = src, oalt = src == 1 ? 2 : 1;
  if (research) use_delta = 0;
  LAUNCH(hc_init_kernel, pixgrid(L), dim3(PIX_T), src, ocur, use_delta, 1);
  box2d(L, R, F_D, F_CNT);  // counts of valid pixels
  for (int it = 0; it < K; ++it) {
    if (it == 0 || research) {
      if (it > 0) LAUNCH(hc_init_kernel, pixgrid(L), dim3(PIX_T), src, ocur, use_delta, 0);
      box2d(L, R, F_IN, F_IN, 1, src);  // a = box(o m) / box(m) or box(s m) / box(m)
    }
    LAUNCH(hc_b_kernel, pixgrid(L), dim3(PIX_T), src, (double)alpha, it == 0 ? 1 : 0);
    box2d(L, R, F_IN, F_IN, it == K - 1 ? 3 : 2, src);  // d = a - box(b m) / box(m)
    if (research && it < K - 1) {
      LAUNCH(research_kernel, dim3(ceil_div(L.maxW, SP_TX), L.maxH, L.npairs), dim3(SP_TX), ocur,
             src, oalt, (int)F_D, range, (double)eta);
      std::swap(ocur, oalt);
    }
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- reprojection
// [X Y Z W] = Q [x y d 1], point (X/W, Y/W, Z/W); NaN for a NaN disparity or
// W == 0.
__global__ void reproject_kernel(const float *__restrict__ disp, int H, int W, Mat4 Q,
                                 float *__restrict__ xyz) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= W || y >= H) return;
  const size_t k = (size_t)y * W + x;
  const float df = disp[k];
  float px = __builtin_nanf(""), py = px, pz = px;
  if (!__builtin_isnan(df)) {
    const double v[4] = {(double)x, (double)y, (double)df, 1.0};
    double r[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
      r[i] = Q.q[4 * i] * v[0] + Q.q[4 * i + 1] * v[1] + Q.q[4 * i + 2] * v[2] + Q.q[4 * i + 3] * v[3];
    if (r[3] != 0.0) {
      px = (float)(r[0] / r[3]);
      py = (float)(r[1] / r[3]);
      pz = (float)(r[2] / r[3]);
    }
  }
  xyz[3 * k] = px;
  xyz[3 * k + 1] = py;
  xyz[3 * k + 2] = pz;
}

hipError_t launch_reproject(const float *disp, int H, int W, const Mat4 &Q, float *xyz, hipStream_t s) {
  hipLaunchKernelGGL(reproject_kernel, dim3(ceil_div(W, 256), H), dim3(256), 0, s, disp, H, W, Q, xyz);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, int N, uint32_t v, hipStream_t s) {
  hipLaunchKernelGGL(fill_u32_kernel, dim3(ceil_div(N, 256)), dim3(256), 0, s, p, N, v);
  return hipGetLastError();
}

}  // namespace st
