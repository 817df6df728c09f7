// Post-processing of the WTA disparities (Section II-B and II-C of the paper)
// and the exact sub-pixel step.  Every kernel is a Jacobi step: it reads
// whole input maps and writes new ones, one thread per pixel, so results do
// not depend on scheduling.  Integer results are exact; smoothing runs in
// FP64.  Each kernel serves one pair (descriptor by value) or a batch (table
// in device memory; see block_pos for the block-to-pair mapping).
#include <algorithm>

#include "common.h"

namespace st {

#define PAIR                          \
  const BlockPos bp = block_pos();    \
  const PostPair &P = B ? many[bp.pair] : one
// Per-pixel kernels: a block of PIX_T threads covers PIX_SEG columns of one
// row, PIX_SEG / PIX_T pixels per thread at stride PIX_T (coalesced).  Few,
// fat blocks: with one short-lived block per 128 pixels these kernels were
// limited by the rate at which waves are launched, not by work.
constexpr int PIX_T = 256, PIX_SEG = 1024;
template <class F>
__device__ __forceinline__ void for_pixels(const PostPair &P, const BlockPos &bp, F f) {
  const int y = bp.y;
  if (y >= P.H) return;
  const int x1 = min(P.W, (bp.x + 1) * PIX_SEG);
  for (int x = bp.x * PIX_SEG + threadIdx.x; x < x1; x += PIX_T) f(x, y, (size_t)y * P.W + x);
}

// Four consecutive pixels per thread (PIX_SEG = 4 PIX_T columns per block),
// for the kernels whose per-pixel work is a few loads and stores: when the
// width is a multiple of 4 every quad starts 4-aligned in the flat planes and
// lies inside its row, and, if the caller's planes are aligned for it
// (`aligned`: a stage entry point may hand in any pointer), `quad` moves it
// with one wide load or store per plane (a quarter of the address work of a
// pixel per lane, which bounded these kernels); otherwise `one` takes the
// pixels one by one.
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
template <class Q, class S>
__device__ __forceinline__ void for_quads(const PostPair &P, const BlockPos &bp, bool aligned, Q quad,
                                          S one) {
  const int y = bp.y, W = P.W;
  if (y >= P.H) return;
  const int x = bp.x * PIX_SEG + 4 * (int)threadIdx.x;
  if (x >= W) return;
  const size_t k = (size_t)y * W + x;
  if ((W & 3) == 0 && aligned) {
    quad(k);
  } else {
    for (int i = 0; i < 4 && x + i < W; ++i) one(k + i);
  }
}
template <class T>
__device__ __forceinline__ T ldq(const void *p, size_t byte_off) {
  return *(const GLOBAL T *)((const GLOBAL char *)p + byte_off);
}
template <class T>
__device__ __forceinline__ void stq(void *p, size_t byte_off, T v) {
  *(GLOBAL T *)((GLOBAL char *)p + byte_off) = v;
}

// floor(a / b) for b > 0.  With |a|, b < 2^52 (every case of the default
// radii) a double estimate, off by at most one, is corrected with the exact
// integer remainder, which avoids the long 64-bit integer division.
__device__ __forceinline__ long long floordiv_ll(long long a, long long b) {
  constexpr long long LIM = 1LL << 52;
  if (a > -LIM && a < LIM && b < LIM) {
    long long q = (long long)floor((double)a / (double)b);
    const long long r = a - q * b;
    if (r < 0) --q;
    else if (r >= b) ++q;
    return q;
  }
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
  // bit 31 marks a key with a valid candidate
  auto dis = [&](uint32_t key) -> uint32_t {
    return (int)key < 0 ? (uint32_t)(uint16_t)(int16_t)(P.dmin + 255 - (int)(key & 255u)) : 0x8000u;
  };
  // quads: keys 16-byte, disparity maps 8-byte, masks 4-byte aligned
  const bool al = (((uintptr_t)P.keyL | (uintptr_t)P.keyR) & 15) == 0 &&
                  (((uintptr_t)P.ob[0] | (uintptr_t)P.oR) & 7) == 0 &&
                  (((uintptr_t)P.mb[0] | (uintptr_t)P.mR) & 3) == 0;
  for_quads(
      P, bp, al,
      [&](size_t k) {
        const u32x4 a = ldq<u32x4>(P.keyL, 4 * k), b = ldq<u32x4>(P.keyR, 4 * k);
        const u32x2 oa = {dis(a.x) | dis(a.y) << 16, dis(a.z) | dis(a.w) << 16};
        const u32x2 ob = {dis(b.x) | dis(b.y) << 16, dis(b.z) | dis(b.w) << 16};
        const uint32_t ma = (a.x >> 31) | (a.y >> 31) << 8 | (a.z >> 31) << 16 | (a.w >> 31) << 24;
        const uint32_t mb = (b.x >> 31) | (b.y >> 31) << 8 | (b.z >> 31) << 16 | (b.w >> 31) << 24;
        stq(P.ob[0], 2 * k, oa);
        stq(P.mb[0], k, ma);
        stq(P.oR, 2 * k, ob);
        stq(P.mR, k, mb);
        stq(P.keyL, 4 * k, u32x4{0u, 0u, 0u, 0u});
        stq(P.keyR, 4 * k, u32x4{0u, 0u, 0u, 0u});
      },
      [&](size_t k) {
        const uint32_t a = P.keyL[k], b = P.keyR[k];
        P.ob[0][k] = (int16_t)dis(a);
        P.mb[0][k] = (uint8_t)(a >> 31);
        P.oR[k] = (int16_t)dis(b);
        P.mR[k] = (uint8_t)(b >> 31);
        P.keyL[k] = 0;
        P.keyR[k] = 0;
      });
}

__global__ void fill_u32_kernel(uint32_t *p, int N, uint32_t v) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < N) p[k] = v;
}

__global__ void mark_invalid_kernel(const int16_t *__restrict__ o, const uint8_t *__restrict__ m,
                                    int16_t *__restrict__ out, size_t N) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < N) out[k] = m[k] ? o[k] : O_NONE;
}

// ---------------------------------------------------------------- sub-pixel
// Exact ZNCC at o-1, o, o+1 (int32 window sums of L*R, int64 numerator
// n*S_LR - S_L*S_R, FP64 normalisation), then the parabola offset
// delta = (zm - zp) / (2 (zm - 2 z0 + zp)) clamped to [-1/2, 1/2]; 0 at the
// ends of the range, when a neighbour is missing or the curvature is >= 0.
//
// A block of 256 threads covers 128 columns x 8 rows; each thread takes
// four pixels of its column (rows ty, ty + 2, ty + 4, ty + 6 of the band).
// The block stages the image rows its windows meet in LDS, column-packed:
// dword (p, c) holds the bytes of stage rows p .. p + 3 of stage column c,
// byte 0 from row p.  A window is then NG = ceil(win / 4) packed rows of win
// dwords, and sum_u L(u) R(u + e) over four window rows is one v_dot4_u32_u8
// of aligned dwords, for any column and any shift e: no byte realignment per
// lane.  Stage columns 0 .. 4 QL - 1 are L(., x0 - h + c); the next 4 QR
// are R(., x0 - omax - 1 - h + c), omax the largest disparity of the block.
constexpr int SP_TX = 128, SP_MAXWIN = 15;
constexpr int SPB_T = 256, SPB_TY = 8;

__host__ __device__ inline int sp_groups(int win) { return (win + 3) / 4; }
__host__ __device__ inline int sp_quads_l(int win) { return (SP_TX + win - 1 + 3) / 4; }
__host__ __device__ inline int sp_quads_r(int win, int range) { return (SP_TX + range + 2 + win - 1 + 3) / 4; }
// LDS bytes of the packed stage for windows up to maxWin and maxD
// disparities, bands of ty rows
static size_t sp_lds_bytes(int maxWin, int maxD, int ty = SPB_TY) {
  const size_t S = 4 * (size_t)(sp_quads_l(maxWin) + sp_quads_r(maxWin, maxD - 1));
  return (size_t)(ty + 4 * (sp_groups(maxWin) - 1)) * S * 4;
}

// The dword-aligned dword at byte offset a of base[0, span) (base + a is
// 4-aligned), its bytes outside the buffer 0.  A dword that straddles an end
// of the buffer lies in the page of a byte inside and is read whole; one
// wholly outside is not read (the aligned dword holding base[0] is read in
// its place and dropped).
__device__ __forceinline__ uint32_t sp_dword(const GLOBAL uint8_t *base, long long a, long long span) {
  const bool ok = a > -4 && a < span;
  const uint32_t x = *(const GLOBAL uint32_t *)(base + (ok ? a : -(long long)((uintptr_t)base & 3)));
  const int lo = a < 0 ? (int)(-a) : 0, hi = a + 4 > span ? (int)(a + 4 - span) : 0;
  return ok ? x & ((0xFFFFFFFFu << (8 * (lo & 3))) & (0xFFFFFFFFu >> (8 * (hi & 3)))) : 0u;
}

// Build packed rows 0 .. PR - 1 of the stage (row stride S dwords).  Work
// item (chunk k, quad q): packed rows 4k .. 4k + 3 of stage columns
// 4q .. 4q + 3, from image rows yr0 + 4k .. yr0 + 4k + 6 (one 4-byte load
// each, realigned from two aligned dwords), shifting each row's bytes in at
// the top of the four column dwords.  Bytes outside the buffer are 0; bytes
// of columns outside the image only reach sums whose z is discarded.  When
// every byte the block reads lies inside the buffer (all bands but the
// image's first and last ones), the loads take no bounds checks.
// One side of the stage: nq quads from image column col0, stage columns
// from cbase.  g is the same for every lane, so a load takes the plane's
// base in scalar registers and a 32-bit lane offset (the fast path, taken
// when every offset of the block is below 2^31).
__device__ __forceinline__ void sp_pack_side(uint32_t *Pk, int S, int PR, const GLOBAL uint8_t *g,
                                             int pitch, long long span, int yr0, int col0, int nq,
                                             int cbase, bool inside, int tid) {
  const int items = nq * ((PR + 3) >> 2), pm = pitch & 3;
  for (int it = tid; it < items; it += SPB_T) {
    const int k = it / nq, q = it - k * nq;
    const long long off0 = (long long)(yr0 + 4 * k) * pitch + col0 + 4 * q;
    uint32_t raw[7];
    if (inside) {
      const uint32_t o0 = (uint32_t)off0;
      const int m0 = (int)(((uintptr_t)g + o0) & 3);
#pragma unroll
      for (int t = 0; t < 7; ++t) {
        const int mis = (m0 + t * pm) & 3;
        const uint32_t a = o0 + (uint32_t)(t * pitch) - (uint32_t)mis;
        const GLOBAL uint32_t *w = (const GLOBAL uint32_t *)(g + a);
        raw[t] = __builtin_amdgcn_alignbyte(w[1], w[0], mis);
      }
    } else {
#pragma unroll
      for (int t = 0; t < 7; ++t) {
        const long long off = off0 + (long long)t * pitch;
        const int mis = (int)(((uintptr_t)g + (uintptr_t)off) & 3);
        const long long a = off - mis;
        raw[t] = __builtin_amdgcn_alignbyte(sp_dword(g, a + 4, span), sp_dword(g, a, span), mis);
      }
    }
    uint32_t c0 = 0, c1 = 0, c2 = 0, c3 = 0;
    uint32_t *dst = Pk + (cbase + 4 * q);
#pragma unroll
    for (int t = 0; t < 7; ++t) {
      const uint32_t v = raw[t];
      c0 = (c0 >> 8) | (v << 24);
      c1 = (c1 >> 8) | ((v >> 8) << 24);
      c2 = (c2 >> 8) | ((v >> 16) << 24);
      c3 = (c3 >> 8) | ((v >> 24) << 24);
      const int p = 4 * k + t - 3;
      if (t >= 3 && p < PR) *(uint4 *)(dst + p * S) = make_uint4(c0, c1, c2, c3);
    }
  }
}

// Build packed rows 0 .. PR - 1 of the stage (row stride S dwords).  Work
// item (chunk k, quad q): packed rows 4k .. 4k + 3 of stage columns
// 4q .. 4q + 3, from image rows yr0 + 4k .. yr0 + 4k + 6 (one 4-byte load
// each, realigned from two aligned dwords), shifting each row's bytes in at
// the top of the four column dwords.  Bytes outside the buffer are 0; bytes
// of columns outside the image only reach sums whose z is discarded.  When
// every byte the block reads lies inside the buffer (all bands but the
// image's first and last ones), the loads take no bounds checks.
__device__ __forceinline__ void sp_pack(uint32_t *Pk, int S, int PR, const GLOBAL uint8_t *Lg,
                                        const GLOBAL uint8_t *Rg, int pitch, long long span, int yr0,
                                        int lx0, int QL, int rx0, int QR, int tid) {
  const int nk = (PR + 3) >> 2;
  // bytes read: rows yr0 .. yr0 + 4 nk + 2, columns from 3 before the first
  // staged one to 7 past the last one's start (two dwords per load)
  const long long first = (long long)yr0 * pitch + min(lx0, rx0) - 3;
  const long long last = (long long)(yr0 + 4 * nk + 2) * pitch + max(lx0 + 4 * QL, rx0 + 4 * QR) + 8;
  // (and the offsets fit 31 bits: the pitch is the caller's, not bounded)
  const bool inside = first >= 0 && last <= span && last < (1LL << 31);
  sp_pack_side(Pk, S, PR, Lg, pitch, span, yr0, lx0, QL, 0, inside, tid);
  sp_pack_side(Pk, S, PR, Rg, pitch, span, yr0, rx0, QR, 4 * QL, inside, tid);
}

// Window sums at the disparities o + 1, o, o - 1 (sp, s0, sm) of a pixel
// whose window starts at packed row r0, stage column tx of L and column rs
// of the R part: sum over the packed rows and columns u of
// L(u) . R(rs + u + e), e = 0, 1, 2.  The last packed row keeps the
// win - 4 (NG - 1) rows inside the window; the chessboard window keeps the
// bytes whose row and column have the parity of the window's corner.
template <int WIN, bool CH>
__device__ __forceinline__ void sp_sums(const uint32_t *Pk, int S, int QL, int r0, int tx, int rs,
                                        int &sp, int &s0, int &sm) {
  constexpr int NG = (WIN + 3) / 4, LAST = WIN - 4 * (NG - 1);
  constexpr uint32_t lastmask = LAST == 4 ? 0xFFFFFFFFu : (1u << (8 * LAST)) - 1u;
  uint32_t a0 = 0, a1 = 0, a2 = 0;
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    const uint32_t *lrow = Pk + (r0 + 4 * g) * S + tx;
    const uint32_t *rrow = Pk + (r0 + 4 * g) * S + 4 * QL + rs;
    uint32_t rv[WIN + 2];
#pragma unroll
    for (int u = 0; u < WIN + 2; ++u) rv[u] = rrow[u];
#pragma unroll
    for (int u = 0; u < WIN; ++u) {
      uint32_t m = g == NG - 1 ? lastmask : 0xFFFFFFFFu;
      if (CH) m &= (u & 1) ? 0xFF00FF00u : 0x00FF00FFu;
      const uint32_t l = m == 0xFFFFFFFFu ? lrow[u] : lrow[u] & m;
      a0 = __builtin_amdgcn_udot4(l, rv[u], a0, false);
      a1 = __builtin_amdgcn_udot4(l, rv[u + 1], a1, false);
      a2 = __builtin_amdgcn_udot4(l, rv[u + 2], a2, false);
    }
    // one packed row at a time (2 win + 2 registers live): the products
    // are formed here rather than sunk to the end of the window
    asm volatile("" : "+v"(a0), "+v"(a1), "+v"(a2));
  }
  sp = (int)a0;
  s0 = (int)a1;
  sm = (int)a2;
}

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// The int32 at byte offset off of a plane (offsets of planes under 4 GiB):
// the base stays scalar, the lane keeps a 32-bit offset.
__device__ __forceinline__ int ld32(const int32_t *p, uint32_t off) {
  return *(const GLOBAL int32_t *)((const GLOBAL char *)p + off);
}

// Per-pixel state of the sub-pixel block (bands of TY rows, NPT pixels a
// thread): the WTA disparity and whether it is a valid candidate.
template <int TY>
struct SpPix {
  static constexpr int NPT = TY * SP_TX / SPB_T;
  int o[NPT];
  bool valid[NPT];
};

template <int WIN, bool CH, int TY>
__device__ __forceinline__ void sp_finish(const PostPair &P, const uint32_t *Pk, int S, int QL,
                                          const SpPix<TY> &X, int tx, int ty, int x, int y0, int omax) {
  const long long n = CH ? ((long long)WIN * WIN + 1) / 2 : (long long)WIN * WIN;
  const double qn = __builtin_nan("");
  const int W = P.W, H = P.H;
#pragma unroll
  for (int j = 0; j < SpPix<TY>::NPT; ++j) {
    const int r0 = ty + 2 * j, y = y0 + r0;
    if (x >= W || y >= H) continue;
    const size_t k = (size_t)y * W + x;
    if (!X.valid[j]) {
      if (P.zbest) P.zbest[k] = qn;
      if (P.zm) P.zm[k] = qn;
      if (P.zp) P.zp[k] = qn;
      P.delta[k] = 0.0f;
      continue;
    }
    // window statistics: left at (x, y), right at x - d for d = o - 1, o,
    // o + 1 (bit q of rok: d = o - 1 + q is a candidate whose right window
    // is inside the image); issued before the sums, which hide their latency
    const int o = X.o[j];
    // statistics planes hold under 2^28 int32 values: 32-bit byte offsets
    const uint32_t k4 = 4u * (uint32_t)k;
    const int sli = ld32(P.SL, k4), ssli = ld32(P.SSL, k4);
    int sri[3], ssri[3], rok = 0;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int d = o + q - 1, xr = x - d;
      const bool ok = d >= P.dmin && d <= P.dmax && xr >= WIN / 2 && xr <= W - 1 - WIN / 2;
      const uint32_t kr4 = ok ? k4 + 4u * (uint32_t)(xr - x) : k4;
      sri[q] = ld32(P.SR, kr4);
      ssri[q] = ld32(P.SSR, kr4);
      rok |= ok ? 1 << q : 0;
    }
    // window column u at d = o + 1 - e is R stage column rs + e + u
    int sm = 0, s0 = 0, sp = 0;  // sums at d = o - 1, o, o + 1
    sp_sums<WIN, CH>(Pk, S, QL, r0, tx, tx + omax - o, sp, s0, sm);
    // the sums are formed here, interleaved, not sunk into the branches
    // below that use them (which would keep every LDS value live)
    asm volatile("" ::"v"(sp), "v"(s0), "v"(sm));
    // varN = n S2 - S1^2 and num = n S_LR - S_L S_R in FP64: every product
    // and difference is an integer below 2^40, so exact.  z = num /
    // sqrt(varN_L varN_R) as num * rsqrt(varN_L varN_R): within a few ulp of
    // the quotient, without the FP64 division.
    const double nd = (double)n, sl = (double)sli;
    const double varL = fma(nd, (double)ssli, -(sl * sl));
    const int slr[3] = {sm, s0, sp};
    double z[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      z[q] = qn;
      if (!((rok >> q) & 1)) continue;
      const double sr = (double)sri[q];
      const double varR = fma(nd, (double)ssri[q], -(sr * sr));
      if (varR <= 0.0) continue;
      const double num = fma(nd, (double)slr[q], -(sl * sr));
      z[q] = num * rsqrt(varL * varR);
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
    // one pixel's LDS reads at a time: hoisting the next pixel's reads
    // above this one's sums would hold them all in registers
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Pk: the packed stage in dynamic LDS, sp_lds_bytes(win, dmax - dmin + 1,
// TY) bytes at least.  TY: rows per band (SPB_TY, or 4 in launches with few
// blocks).
template <int TY>
__device__ __forceinline__ void subpixel_block(const PostPair &P, const BlockPos &bp, uint32_t *Pk) {
  constexpr int NPT = SpPix<TY>::NPT;
  __shared__ int s_omin, s_omax;
  const int tid = threadIdx.x, tx = tid & (SP_TX - 1), ty = tid / SP_TX;
  const int x0 = bp.x * SP_TX, y0 = bp.y * TY;
  if (x0 >= P.W || y0 >= P.H) return;  // uniform per block
  const int W = P.W, H = P.H, win = P.win, h = win / 2;
  const int x = x0 + tx;
  SpPix<TY> X;
  int lo = 1 << 30, hi = -(1 << 30);
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    const int y = y0 + ty + 2 * j;
    const bool in = x < W && y < H;
    const size_t k = (size_t)y * W + x;
    X.o[j] = in ? (int)P.ob[0][k] : 0;
    const bool mk = in && P.mb[0][k];
    // a disparity outside [dmin, dmax] counts as unmatched: the staged R
    // columns cover the range only
    X.valid[j] = mk && X.o[j] >= P.dmin && X.o[j] <= P.dmax;
    if (!X.valid[j]) X.o[j] = 0;
    if (X.valid[j]) {
      lo = min(lo, X.o[j]);
      hi = max(hi, X.o[j]);
    }
  }
  if (tid == 0) {
    s_omin = 1 << 30;
    s_omax = -(1 << 30);
  }
  __syncthreads();
  lo = wave_min(lo);
  hi = wave_max(hi);
  if ((tid & (WV - 1)) == 0 && lo <= hi) {
    atomicMin(&s_omin, lo);
    atomicMax(&s_omax, hi);
  }
  __syncthreads();
  const int omin = s_omin, omax = s_omax;
  const int QL = sp_quads_l(win), QR = omin <= omax ? sp_quads_r(win, omax - omin) : 0;
  const int S = 4 * (QL + QR);
  if (omin <= omax) {
    // a valid pixel's window rows lie inside the band's rows plus the halo
    const int PR = min(TY, H - y0) + 4 * (sp_groups(win) - 1);
    sp_pack(Pk, S, PR, gro(P.left), gro(P.right), P.pitch, (long long)(H - 1) * P.pitch + W, y0 - h,
            x0 - h, QL, x0 - omax - 1 - h, QR, tid);
  }
  __syncthreads();
#define SPF(w)                                                               \
  case w:                                                                    \
    if (P.chess) sp_finish<w, true, TY>(P, Pk, S, QL, X, tx, ty, x, y0, omax);   \
    else sp_finish<w, false, TY>(P, Pk, S, QL, X, tx, ty, x, y0, omax);          \
    break
  switch (win) {
    SPF(3);
    SPF(5);
    SPF(7);
    SPF(9);
    SPF(11);
    SPF(13);
    default:
      if (P.chess) sp_finish<15, true, TY>(P, Pk, S, QL, X, tx, ty, x, y0, omax);
      else sp_finish<15, false, TY>(P, Pk, S, QL, X, tx, ty, x, y0, omax);
      break;
  }
#undef SPF
}

extern __shared__ __align__(16) uint32_t sp_dyn[];

template <bool B>
__global__ __launch_bounds__(SPB_T) void subpixel_kernel(PostPair one, const PostPair *__restrict__ many) {
  PAIR;
  subpixel_block<SPB_TY>(P, bp, sp_dyn);
}

// ---------------------------------------------------------------- LR check
// (ob[0], mb[0]) and (oR, mR) -> (ob[dst], mb[dst]): kept when the right
// pixel x - oL points back within tol.
__device__ __forceinline__ void lr_check_block(const PostPair &P, const BlockPos &bp, int tol, int dst) {
  // four consecutive pixels per thread (PIX_SEG = 4 PIX_T columns per
  // block): the left maps of all four are read together, then the four right
  // pixels they point at, so a thread waits for two round trips
  const int W = P.W, y = bp.y;
  if (y >= P.H) return;
  const int xb = bp.x * PIX_SEG + 4 * (int)threadIdx.x;
  const size_t row = (size_t)y * W;
  int o[4], m[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int x = xb + i;
    o[i] = x < W ? (int)P.ob[0][row + x] : 0;
    m[i] = x < W ? (int)P.mb[0][row + x] : 0;
  }
  int orr[4], mrr[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int xr = xb + i - o[i];
    const bool in = m[i] && xr >= 0 && xr < W;
    const size_t kr = row + (in ? xr : 0);
    orr[i] = in ? (int)P.oR[kr] : 0;
    mrr[i] = in ? (int)P.mR[kr] : 0;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int x = xb + i;
    if (x >= W) break;
    const int diff = o[i] - orr[i];
    const bool keep = m[i] && mrr[i] && (diff < 0 ? -diff : diff) <= tol;
    P.ob[dst][row + x] = keep ? (int16_t)o[i] : O_NONE;
    P.mb[dst][row + x] = keep ? 1 : 0;
  }
}
template <bool B>
__global__ void lr_check_kernel(PostPair one, const PostPair *__restrict__ many, int tol, int dst) {
  PAIR;
  lr_check_block(P, bp, tol, dst);
}

// Sub-pixel fit and left-right check in one launch (independent work on the
// same maps): the first nsp blocks of a pair run the sub-pixel blocks (nspx
// of them per row band), the rest the check (nlrx per row).
template <bool B, int TY>
__global__ __launch_bounds__(SPB_T) void subpixel_lr_kernel(PostPair one, const PostPair *__restrict__ many,
                                                           int nspx, int nsp, int nlrx, int tol, int dst) {
  PAIR;
  BlockPos q = bp;
  if (bp.x < nsp) {
    q.x = bp.x % nspx;
    q.y = bp.x / nspx;
    subpixel_block<TY>(P, q, sp_dyn);
  } else {
    const int i = bp.x - nsp;
    q.x = i % nlrx;
    q.y = i / nlrx;
    lr_check_block(P, q, tol, dst);
  }
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
// Rows: one wave per row sweeps its 64-column blocks left to right and then
// right to left, lanes are columns, ballot masks give the breaks or valid
// pixels of a block, and the position of the nearest one so far is carried
// from block to block; each pixel is read once per sweep.  Columns and
// diagonals: a thread scans SEG rows of one line (SEG / 2 in launches of
// few blocks; plus the look-ahead) and
// the lanes of a wave are neighbouring lines, so each step reads
// consecutive columns of one row.
constexpr int SEG = 32;

__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }
__device__ __forceinline__ int ctz64(uint64_t v) { return __builtin_ctzll(v); }
__device__ __forceinline__ int top64(uint64_t v) { return 63 - __builtin_clzll(v); }
// lanes strictly below / at or below / strictly above `lane`
__device__ __forceinline__ uint64_t lanes_below(int lane) { return (1ull << lane) - 1; }
__device__ __forceinline__ uint64_t lanes_upto(int lane) { return lane == 63 ? ~0ull : (2ull << lane) - 1; }
__device__ __forceinline__ uint64_t lanes_above(int lane) { return lane == 63 ? 0ull : ~0ull << (lane + 1); }

// A step between neighbouring pixels holds when the far one is valid and
// within thresh in disparity.
__device__ __forceinline__ bool step_holds(int o_near, int o_far, bool m_far, float thresh) {
  const int dv = o_far - o_near;
  return m_far && (float)(dv < 0 ? -dv : dv) < thresh;
}

// The same test against an integer bound: for an integer dv, |dv| < thresh
// exactly when |dv| <= ceil(thresh) - 1; a bound below 0 lets no step hold.
__device__ __forceinline__ int step_bound(float thresh) {
  return thresh >= 1048576.0f ? 1048576 : thresh > 0.0f ? (int)ceilf(thresh) - 1 : -1;
}
__device__ __forceinline__ bool step_ok(int o_near, int o_far, bool m_far, int ti) {
  return m_far && ti >= 0 && (unsigned)(o_far - o_near + ti) <= (unsigned)(2 * ti);
}

// The 64-column blocks b0 .. b0 + RCH - 1 of a row, one int16 disparity per
// lane and block (O_NONE outside the row): the loads of a whole chunk issue
// together, so a sweep over a row of up to 64 RCH columns waits for one
// memory round trip rather than one per block.
constexpr int RCH = 16;
__device__ __forceinline__ void row_chunk(const GLOBAL int16_t *o, int W, int b0, int lane, int (&ov)[RCH]) {
#pragma unroll
  for (int i = 0; i < RCH; ++i) {
    const int x = 64 * (b0 + i) + lane;
    ov[i] = x < W ? (int)o[x] : (int)O_NONE;
  }
}

// Outlier test along rows: db = distance from x back to the last break at or
// before x (the step x -> x-1 fails, or x = 0), df = distance to the first
// break at or after x (the step x -> x+1 fails, or x = W-1); bit 0 of pass
// is df >= r, bit 1 db >= r.  The backward bits of the first sweep wait in a
// register mask, one bit per block, when W <= 64 * 64; wider rows keep them
// in pass itself.  Chunks of RCH blocks are swept from registers; a row of
// one chunk is loaded once for both sweeps.
__device__ __forceinline__ void outlier_rows(const PostPair &P, int bx, int r, float thresh, int src) {
  const int H = P.H, W = P.W;
  const int lane = threadIdx.x & 63, y = bx * 4 + (threadIdx.x >> 6);
  if (y >= H) return;  // whole wave
  const GLOBAL int16_t *o = gro(P.ob[src]) + (size_t)y * W;  // O_NONE where invalid
  GLOBAL uint8_t *pass = grw(P.pass) + (size_t)y * W;
  const int nb = ceil_div(W, 64), last = (nb - 1) / RCH * RCH;
  const bool inreg = nb <= 64;
  uint64_t dbits = 0;
  int ov[RCH];
  int lastb = -(1 << 30), co = 0, cm = 0;  // carried: last break, o and m of column 64 b - 1
  for (int c0 = 0; c0 < nb; c0 += RCH) {
    row_chunk(o, W, c0, lane, ov);
#pragma unroll
    for (int i = 0; i < RCH; ++i) {
      const int b = c0 + i;
      if (b >= nb) break;  // uniform
      const int x = 64 * b + lane;
      const bool in = x < W;
      const int mv = ov[i] != O_NONE ? 1 : 0;
      int on = __shfl_up(ov[i], 1, 64), mn = __shfl_up(mv, 1, 64);
      if (lane == 0) {
        on = co;
        mn = cm;
      }
      const uint64_t bm = ballot64(in && (x == 0 || !step_holds(ov[i], on, mn, thresh)));
      const uint64_t low = bm & lanes_upto(lane);
      const int lb = low ? 64 * b + top64(low) : lastb;
      if (inreg) {
        if (x - lb >= r) dbits |= 1ull << b;
      } else if (in && mv) {
        pass[x] = x - lb >= r ? 2 : 0;
      }
      if (bm) lastb = 64 * b + top64(bm);
      co = __shfl(ov[i], 63, 64);
      cm = __shfl(mv, 63, 64);
    }
  }
  int nextb = 1 << 30;
  co = 0;
  cm = 0;  // o and m of column 64 (b + 1)
  for (int c0 = last; c0 >= 0; c0 -= RCH) {
    if (nb > RCH) row_chunk(o, W, c0, lane, ov);
#pragma unroll
    for (int i = RCH - 1; i >= 0; --i) {
      const int b = c0 + i;
      if (b >= nb) continue;  // uniform
      const int x = 64 * b + lane;
      const bool in = x < W;
      const int mv = ov[i] != O_NONE ? 1 : 0;
      int on = __shfl_down(ov[i], 1, 64), mn = __shfl_down(mv, 1, 64);
      if (lane == 63) {
        on = co;
        mn = cm;
      }
      const uint64_t bm = ballot64(in && (x + 1 >= W || !step_holds(ov[i], on, mn, thresh)));
      const uint64_t rest = bm & ~lanes_below(lane);
      const int fb = rest ? 64 * b + ctz64(rest) : nextb;
      if (in && mv) {
        const int bbit = inreg ? (((dbits >> b) & 1) ? 2 : 0) : pass[x];
        pass[x] = (fb - x >= r ? 1 : 0) | bbit;
      }
      if (bm) nextb = 64 * b + ctz64(bm);
      co = __shfl(ov[i], 0, 64);
      cm = __shfl(mv, 0, 64);
    }
  }
}

// Outlier rows for r <= 63, bit-parallel: per 64-column block, ballots give
// the masks of forward breaks (the step x -> x+1 fails, or x = W-1) and of
// backward breaks (x -> x-1 fails, or x = 0).  Bit 0 of pass (df >= r) is
// that bits x .. x + r - 1 of the forward mask are clear, bit 1 (db >= r)
// that bits x - r + 1 .. x of the backward mask are; each window is one
// 64-bit funnel shift of the masks of two neighbouring blocks.  A chunk of
// RCB blocks is loaded with one block more on either side; the outermost
// lanes of those two, whose masks would need a third block, are never read
// (r <= 63).
constexpr int RCB = 8;  // blocks per chunk of the bit-parallel rows (register budget)
__device__ __forceinline__ void outlier_rows_bits(const PostPair &P, int bx, int r, int ti, int src) {
  const int H = P.H, W = P.W;
  const int lane = threadIdx.x & 63, y = bx * 4 + (threadIdx.x >> 6);
  if (y >= H) return;  // whole wave
  const GLOBAL int16_t *o = gro(P.ob[src]) + (size_t)y * W;  // O_NONE where invalid
  GLOBAL uint8_t *pass = grw(P.pass) + (size_t)y * W;
  const int nb = ceil_div(W, 64);
  const uint64_t rmask = (1ull << r) - 1;
  for (int c0 = 0; c0 < nb; c0 += RCB) {
    int ov[RCB + 2];  // blocks c0 - 1 .. c0 + RCB
#pragma unroll
    for (int i = 0; i < RCB + 2; ++i) {
      const int x = 64 * (c0 - 1 + i) + lane;
      ov[i] = x >= 0 && x < W ? (int)o[x] : (int)O_NONE;
    }
    auto masks = [&](int i, uint64_t &fm, uint64_t &bm) {
      const int x = 64 * (c0 - 1 + i) + lane;
      const bool in = x >= 0 && x < W;
      // every shuffle with all lanes active: a lane reading an inactive one
      // gets 0
      int nx = __shfl_down(ov[i], 1, 64), pv = __shfl_up(ov[i], 1, 64);
      const int n0 = i + 1 < RCB + 2 ? __shfl(ov[i + 1], 0, 64) : (int)O_NONE;
      const int p63 = i > 0 ? __shfl(ov[i - 1], 63, 64) : (int)O_NONE;
      if (lane == 63) nx = n0;
      if (lane == 0) pv = p63;
      fm = ballot64(in && (x == W - 1 || !step_ok(ov[i], nx, nx != O_NONE, ti)));
      bm = ballot64(in && (x == 0 || !step_ok(ov[i], pv, pv != O_NONE, ti)));
    };
    uint64_t fA, bA, fB, bB, fC, bC;  // masks of blocks i - 1, i, i + 1
    masks(0, fA, bA);
    masks(1, fB, bB);
#pragma unroll
    for (int i = 1; i <= RCB; ++i) {
      masks(i + 1, fC, bC);
      const int x = 64 * (c0 - 1 + i) + lane;
      if (x < W && ov[i] != O_NONE) {
        const uint64_t wf = lane ? (fB >> lane) | (fC << (64 - lane)) : fB;
        const uint64_t wb = lane < 63 ? (bB << (63 - lane)) | (bA >> (lane + 1)) : bB;
        pass[x] = ((wf & rmask) == 0 ? 1 : 0) | ((wb >> (64 - r)) == 0 ? 2 : 0);
      }
      fA = fB;
      bA = bB;
      fB = fC;
      bB = bC;
    }
  }
}

// Nearest valid pixel along rows for the holes: hits[0] to the right
// (forward), hits[1] to the left, within R.  Swept from registers in chunks
// of RCH blocks, as the outlier rows are.
__device__ __forceinline__ void fill_rows(const PostPair &P, int bx, int R, int src) {
  const int H = P.H, W = P.W;
  const int lane = threadIdx.x & 63, y = bx * 4 + (threadIdx.x >> 6);
  if (y >= H) return;  // whole wave
  const GLOBAL int16_t *o = gro(P.ob[src]) + (size_t)y * W;  // O_NONE where invalid
  const size_t N = (size_t)W * H;
  GLOBAL uint32_t *hf = grw(P.hits) + (size_t)y * W;
  GLOBAL uint32_t *hb = grw(P.hits) + N + (size_t)y * W;
  const int nb = ceil_div(W, 64), last = (nb - 1) / RCH * RCH;
  auto hit = [&](int q, int oq, int x) -> uint32_t {
    const int dq = q > x ? q - x : x - q;
    return (q >= 0 && dq <= R) ? ((uint32_t)dq << 16) | (uint16_t)oq : 0u;
  };
  int ov[RCH];
  int lastv = -1, lasto = 0;  // carried: last valid column left of the block
  for (int c0 = 0; c0 < nb; c0 += RCH) {
    row_chunk(o, W, c0, lane, ov);
#pragma unroll
    for (int i = 0; i < RCH; ++i) {
      const int b = c0 + i;
      if (b >= nb) break;  // uniform
      const int x = 64 * b + lane;
      const bool in = x < W;
      const bool mv = ov[i] != O_NONE;
      const uint64_t vm = ballot64(mv);
      const uint64_t low = vm & lanes_below(lane);
      const int oq = __shfl(ov[i], low ? top64(low) : 0, 64);
      if (in && !mv) hb[x] = low ? hit(64 * b + top64(low), oq, x) : hit(lastv, lasto, x);
      if (vm) {
        lastv = 64 * b + top64(vm);
        lasto = __shfl(ov[i], top64(vm), 64);
      }
    }
  }
  int nextv = -1, nexto = 0;  // carried: first valid column right of the block
  for (int c0 = last; c0 >= 0; c0 -= RCH) {
    if (nb > RCH) row_chunk(o, W, c0, lane, ov);
#pragma unroll
    for (int i = RCH - 1; i >= 0; --i) {
      const int b = c0 + i;
      if (b >= nb) continue;  // uniform
      const int x = 64 * b + lane;
      const bool in = x < W;
      const bool mv = ov[i] != O_NONE;
      const uint64_t vm = ballot64(mv);
      const uint64_t rest = vm & lanes_above(lane);
      const int oq = __shfl(ov[i], rest ? ctz64(rest) : 0, 64);
      if (in && !mv) hf[x] = rest ? hit(64 * b + ctz64(rest), oq, x) : hit(nextv, nexto, x);
      if (vm) {
        nextv = 64 * b + ctz64(vm);
        nexto = __shfl(ov[i], ctz64(vm), 64);
      }
    }
  }
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
// Thread index -> (line type 1..3, line, row segment); false for an idle
// thread.  The rows [a0, a1) of a segment meet W columns and W + (a1 - a0) -
// 1 lines of either diagonal direction: a line type gives each segment
// W + SEG - 1 threads (W for columns), and its range of thread indices is
// rounded up to whole waves, so that the lanes of a wave share one line type
// and with it the step between a line's pixels in the plane.
// SG: rows per segment (SEG, or SEG / 2 for launches with few blocks).
template <int SG>
__host__ __device__ inline int vscan_slots(int t, int W) { return t == 1 ? W : W + SG - 1; }
template <int SG>
__host__ __device__ inline int vscan_span(int t, int H, int W) {
  return (ceil_div(H, SG) * vscan_slots<SG>(t, W) + WV - 1) / WV * WV;
}
template <int SG>
__device__ __forceinline__ bool vscan_task(int idx, int H, int W, int &t, int &l, int &sg) {
  const int ns = ceil_div(H, SG);
  for (t = 1; t < 4; ++t) {
    const int span = vscan_span<SG>(t, H, W);
    if (idx < span) {
      const int nper = vscan_slots<SG>(t, W);
      sg = idx / nper;
      if (sg >= ns) return false;  // rounding to whole waves
      const int i = idx - sg * nper;
      if (t == 1) {
        l = i;
        return true;
      }
      const int a0 = sg * SG, a1 = min(H, a0 + SG);
      if (i >= W + (a1 - a0) - 1) return false;  // a short last segment
      // the first line through the segment: through (0, a1 - 1) for the
      // diagonals, through (0, a0) for the anti-diagonals
      l = (t == 2 ? H - a1 : a0) + i;
      return true;
    }
    idx -= span;
  }
  return false;
}

// Element k (>= 0) of a 16-bit plane: planes hold at most 2^28 pixels, so
// the byte offset fits 32 bits and the load takes the plane's base in
// scalar registers plus one 32-bit lane offset (no 64-bit address per
// step).
__device__ __forceinline__ int16_t ld16(const GLOBAL int16_t *p, int k) {
  return *(const GLOBAL int16_t *)((const GLOBAL char *)p + 2u * (uint32_t)k);
}

// Visit the n pixels k0, k0 + ks, ... of a line in order (ks the same for
// every lane of the wave).  Whole groups of LW pixels are loaded before any
// of them is visited, so that a visit's conditional store never stands
// between a load and the next one: each group waits for one memory round
// trip; the last n % LW pixels go one by one.  Load i of a group takes the
// scalar base o + i ks (below o for a negative step: the sum with the lane's
// offset, the byte offset of the group's first pixel, is a pixel of the
// line) and the one lane offset of the group.
constexpr int LW = 8;
template <class F>
__device__ __forceinline__ void line_walk(const GLOBAL int16_t *o, int k0, int ks, int n, F f) {
  const int ksu = __builtin_amdgcn_readfirstlane(ks);
  const GLOBAL char *bs[LW];
#pragma unroll
  for (int i = 0; i < LW; ++i)
    bs[i] = (const GLOBAL char *)((uintptr_t)o + (uintptr_t)(2 * (intptr_t)i * ksu));
  int j = 0, k = k0;
  for (; j + LW <= n; j += LW, k += LW * ksu) {
    const uint32_t kb = 2u * (uint32_t)k;
    int16_t v[LW];
#pragma unroll
    for (int i = 0; i < LW; ++i) v[i] = *(const GLOBAL int16_t *)(bs[i] + kb);
#pragma unroll
    for (int i = 0; i < LW; ++i) f(j + i, k + i * ksu, v[i]);
  }
  for (; j < n; ++j, k += ksu) f(j, k, ld16(o, k));
}

// Each scan first runs through the look-ahead rows (state only), then through
// its own rows, writing results only where a later kernel reads them: pass
// for valid pixels, hits for holes.
template <int SG>
__device__ __forceinline__ void outlier_vscan(const PostPair &P, int bx, int r, float thresh, int src) {
  static_assert(SG <= 32, "the forward results of a segment wait in a 32-bit mask");
  const int H = P.H, W = P.W;
  int t, l, sg;
  if (!vscan_task<SG>(bx * blockDim.x + threadIdx.x, H, W, t, l, sg)) return;
  const VLine L = vline(t, l, H, W);
  const int a = max(L.ylo, sg * SG), b = min(L.yhi, sg * SG + SG);
  if (a >= b) return;
  const GLOBAL int16_t *__restrict__ o = gro(P.ob[src]);  // O_NONE where invalid
  // pass byte of flat index k of this line type: the four planes hold at
  // most 2^30 bytes, so the offset is 32-bit from the scalar base
  GLOBAL uint8_t *const pbase = grw(P.pass);
  const uint32_t poff = (uint32_t)t * (uint32_t)W * (uint32_t)H;
  auto pass_at = [&](int k) -> GLOBAL uint8_t & { return pbase[poff + (uint32_t)k]; };
  // run = consecutive good steps from y along the scan direction (not
  // capped: only run >= r is asked)
  const int ti = step_bound(thresh);
  // forward results of the own rows wait in a bit mask (bit y - a) and are
  // stored with the backward ones
  uint32_t fbits = 0;
  {  // forward (+y), walked from the end of the look-ahead back to a; the
     // line's last pixel has no forward step (bit stays 0)
    const int e = min(L.yhi - 1, b - 1 + r);
    int on = ld16(o, e * L.st + L.c0), run = 0;
    bool vn = on != O_NONE;
    auto step = [&](int op) {
      const bool v = op != O_NONE;
      run = step_ok(op, on, vn, ti) ? run + 1 : 0;
      on = op;
      vn = v;
      return v;
    };
    // look-ahead rows e-1 .. b, then own rows min(e-1, b-1) .. a
    line_walk(o, (e - 1) * L.st + L.c0, -L.st, e - b, [&](int, int, int16_t op) { step(op); });
    const int y0 = min(e - 1, b - 1);
    line_walk(o, y0 * L.st + L.c0, -L.st, y0 - a + 1, [&](int i, int, int16_t op) {
      const bool v = step(op);
      fbits |= (v && run >= r ? 1u : 0u) << (y0 - i - a);
    });
  }
  {  // backward (-y); when e == a the first row has no step (run 0 < r)
    const int e = max(L.ylo, a - r);
    const int ke = e * L.st + L.c0;
    int on = ld16(o, ke), run = 0;
    bool vn = on != O_NONE;
    if (e == a && vn) pass_at(ke) = (uint8_t)(fbits & 1u);
    auto step = [&](int op) {
      const bool v = op != O_NONE;
      run = step_ok(op, on, vn, ti) ? run + 1 : 0;
      on = op;
      vn = v;
      return v;
    };
    // look-ahead rows e+1 .. a-1, then own rows max(e+1, a) .. b-1
    line_walk(o, (e + 1) * L.st + L.c0, L.st, a - 1 - e, [&](int, int, int16_t op) { step(op); });
    const int y0 = max(e + 1, a);
    line_walk(o, y0 * L.st + L.c0, L.st, b - y0, [&](int i, int k, int16_t op) {
      if (step(op)) pass_at(k) = (uint8_t)(((fbits >> (y0 + i - a)) & 1u) | (run >= r ? 2u : 0u));
    });
  }
}

// The first valid pixel of a line walking from k0 in steps of ks, at most n
// pixels (its index along the walk in i, its disparity in vq; i = -1 when
// there is none).  Groups of LW loads, stopping after the first group that
// holds a valid pixel: where most pixels are valid that is the first.
__device__ __forceinline__ int first_valid(const GLOBAL int16_t *o, int k0, int ks, int n,
                                           uint32_t &vq) {
  for (int j = 0; j < n; j += LW) {
    int16_t v[LW];
#pragma unroll
    for (int i = 0; i < LW; ++i) v[i] = ld16(o, k0 + min(j + i, n - 1) * ks);
    int f = -1;
#pragma unroll
    for (int i = LW - 1; i >= 0; --i)
      if (j + i < n && v[i] != O_NONE) {
        f = j + i;
        vq = (uint32_t)(uint16_t)v[i];
      }
    if (f >= 0) return f;
  }
  return -1;
}

template <int SG>
__device__ __forceinline__ void fill_vscan(const PostPair &P, int bx, int R, int src) {
  const int H = P.H, W = P.W;
  int t, l, sg;
  if (!vscan_task<SG>(bx * blockDim.x + threadIdx.x, H, W, t, l, sg)) return;
  const VLine L = vline(t, l, H, W);
  const int a = max(L.ylo, sg * SG), b = min(L.yhi, sg * SG + SG);
  if (a >= b) return;
  const GLOBAL int16_t *__restrict__ o = gro(P.ob[src]);  // O_NONE where invalid
  const size_t N = (size_t)W * H;
  GLOBAL uint32_t *__restrict__ hf = grw(P.hits) + (size_t)(2 * t) * N;
  GLOBAL uint32_t *__restrict__ hb = grw(P.hits) + (size_t)(2 * t + 1) * N;
  {  // nearest valid pixel in +y: the first one at or after b (at most up to
     // b - 1 + R), then own rows b-1 .. a
    const int e = min(L.yhi - 1, b - 1 + R);
    uint32_t vq = 0;
    const int f = first_valid(o, b * L.st + L.c0, L.st, e - b + 1, vq);
    int q = f >= 0 ? b + f : -1;
    line_walk(o, (b - 1) * L.st + L.c0, -L.st, b - a, [&](int i, int k, int16_t oo) {
      const int y = b - 1 - i;
      const bool v = oo != O_NONE;
      if (!v) hf[k] = (q >= 0 && q - y <= R) ? ((uint32_t)(q - y) << 16) | vq : 0u;
      q = v ? y : q;
      vq = v ? (uint32_t)(uint16_t)oo : vq;
    });
  }
  {  // nearest valid pixel in -y: the first one at or before a - 1 (at most
     // down to a - R), then own rows a .. b-1
    const int e = max(L.ylo, a - R);
    uint32_t vq = 0;
    const int f = first_valid(o, (a - 1) * L.st + L.c0, -L.st, a - e, vq);
    int q = f >= 0 ? a - 1 - f : -1;
    line_walk(o, a * L.st + L.c0, L.st, b - a, [&](int i, int k, int16_t oo) {
      const int y = a + i;
      const bool v = oo != O_NONE;
      if (!v) hb[k] = (q >= 0 && y - q <= R) ? ((uint32_t)(y - q) << 16) | vq : 0u;
      q = v ? y : q;
      vq = v ? (uint32_t)(uint16_t)oo : vq;
    });
  }
}

// The four line types of a scan in one launch: the first nrow blocks of a
// pair take rows (a wave per row), the others columns and diagonals; the
// two kinds of work are independent and overlap on the GPU.
template <bool B, int SG>
__global__ __launch_bounds__(256) void outlier_scan_kernel(PostPair one, const PostPair *__restrict__ many,
                                                          int r, float thresh, int src, int nrow) {
  PAIR;
  if (bp.x < nrow) {
    if (r <= 63) outlier_rows_bits(P, bp.x, r, step_bound(thresh), src);
    else outlier_rows(P, bp.x, r, thresh, src);
  } else {
    outlier_vscan<SG>(P, bp.x - nrow, r, thresh, src);
  }
}
template <bool B, int SG>
__global__ __launch_bounds__(256) void fill_scan_kernel(PostPair one, const PostPair *__restrict__ many,
                                                       int R, int src, int nrow) {
  PAIR;
  if (bp.x < nrow) fill_rows(P, bp.x, R, src);
  else fill_vscan<SG>(P, bp.x - nrow, R, src);
}

// A valid pixel stays when some direction passes (Section II-B).
template <bool B>
__global__ void outlier_combine_kernel(PostPair one, const PostPair *__restrict__ many, int src, int dst) {
  PAIR;
  const int W = P.W, H = P.H;
  (void)W;
  (void)H;
  const size_t N = (size_t)W * H;
  const bool al = (((uintptr_t)P.mb[src] | (uintptr_t)P.mb[dst] | (uintptr_t)P.pass) & 3) == 0 &&
                  (((uintptr_t)P.ob[src] | (uintptr_t)P.ob[dst]) & 7) == 0;
  for_quads(
      P, bp, al,
      [&](size_t k) {
        const uint32_t mk = ldq<uint32_t>(P.mb[src], k);
        const uint32_t any = ldq<uint32_t>(P.pass, k) | ldq<uint32_t>(P.pass, N + k) |
                             ldq<uint32_t>(P.pass, 2 * N + k) | ldq<uint32_t>(P.pass, 3 * N + k);
        const u32x2 o = ldq<u32x2>(P.ob[src], 2 * k);
        // per byte i: the mask code if the pixel stays (valid, some
        // direction passes), else 0; its disparity, or O_NONE
        uint32_t mo = 0, oo[2] = {0u, 0u};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const uint32_t m = (mk >> (8 * i)) & 255u;
          const bool keep = m != 0 && ((any >> (8 * i)) & 255u) != 0;
          mo |= (keep ? m : 0u) << (8 * i);
          const uint32_t oi = ((i < 2 ? o.x : o.y) >> (16 * (i & 1))) & 0xFFFFu;
          oo[i >> 1] |= (keep ? oi : 0x8000u) << (16 * (i & 1));
        }
        stq(P.ob[dst], 2 * k, u32x2{oo[0], oo[1]});
        stq(P.mb[dst], k, mo);
      },
      [&](size_t k) {
        const uint8_t mk = P.mb[src][k];
        const bool any = (P.pass[k] | P.pass[N + k] | P.pass[2 * N + k] | P.pass[3 * N + k]) != 0;
        const bool keep = mk && any;
        const int16_t o = P.ob[src][k];
        P.ob[dst][k] = keep ? o : O_NONE;
        P.mb[dst][k] = keep ? mk : 0;
      });
}

// (i) radial fill from the scanned hits: complete lines (both opposite
// directions hit) give (va*sb + vb*sa)/(sa+sb); with >= min_lines complete
// lines the hole takes their mean, an exact rational rounded half to even;
// code 2.  Fused with the row prefix sums of the result that the disk fill
// reads: pc[y][x+1] = number of valid pixels x' <= x in row y, ps[y][x+1]
// the sum of their disparities.  One block per row; a thread takes the
// columns t, t + 256, t + 512, t + 768 of each 1024-column piece, so that
// the maps of all four, then the hits of all their holes, are loaded
// together (two round trips per piece), and the piece's prefix sums take
// one block barrier (wave scans, then the wave totals of the four chunks
// in LDS).
// packed (the disk fill's radius up to DISK_RPK and rows narrower than 4096):
// one 32-bit word per prefix, count | sum << 12 (the sum modulo 2^20; see
// fill_disk_kernel), in plane pc alone.
constexpr int RF_CPT = 4;
template <bool B>
__global__ __launch_bounds__(256) void fill_radial_kernel(PostPair one, const PostPair *__restrict__ many,
                                                          int min_lines, int src, int dst, int packed) {
  PAIR;
  __shared__ int wc[RF_CPT][4], wsum[RF_CPT][4];
  const int y = bp.x;
  if (y >= P.H) return;  // uniform per block
  const int W = P.W, H = P.H, t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const size_t N = (size_t)W * H;
  const GLOBAL int16_t *o = gro(P.ob[src]);
  const GLOBAL uint8_t *m = gro(P.mb[src]);
  GLOBAL int32_t *pcr = grw(P.pc) + (size_t)y * (W + 1);
  GLOBAL int32_t *psr = grw(P.ps) + (size_t)y * (W + 1);
  if (t == 0) {
    pcr[0] = 0;
    if (!packed) psr[0] = 0;
  }
  const uint32_t row = (uint32_t)y * (uint32_t)W;  // flat index of (0, y): below 2^28
  int carry_c = 0, carry_s = 0;
  for (int x0 = 0; x0 < W; x0 += 256 * RF_CPT) {
    int ov[RF_CPT], mv[RF_CPT];
#pragma unroll
    for (int j = 0; j < RF_CPT; ++j) {
      const int x = x0 + 256 * j + t;
      const bool in = x < W;
      ov[j] = in ? (int)ld16(o, (int)(row + x)) : 0;
      mv[j] = in ? (int)m[row + x] : 0;
    }
    // the eight hits of every hole of the thread, all in flight together
    // (plane i from its own base, 32-bit lane offsets)
    uint32_t hv[RF_CPT][8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const GLOBAL char *hp = (const GLOBAL char *)(gro(P.hits) + (size_t)i * N);
#pragma unroll
      for (int j = 0; j < RF_CPT; ++j) {
        const int x = x0 + 256 * j + t;
        const bool hole = x < W && mv[j] == 0;
        hv[j][i] = hole ? *(const GLOBAL uint32_t *)(hp + 4u * (row + (uint32_t)x)) : 0u;
      }
    }
#pragma unroll
    for (int j = 0; j < RF_CPT; ++j) {
      const int x = x0 + 256 * j + t;
      if (x >= W) continue;
      if (mv[j] == 0) {
        long long num = 0, den = 1;
        int lines = 0;
#pragma unroll
        for (int ln = 0; ln < 4; ++ln) {
          const uint32_t ha = hv[j][2 * ln], hb = hv[j][2 * ln + 1];
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
          ov[j] = (int)round_half_even(num, den * lines);
          mv[j] = 2;
        }
      }
      grw(P.ob[dst])[row + x] = (int16_t)ov[j];
      grw(P.mb[dst])[row + x] = (uint8_t)mv[j];
    }
    int c[RF_CPT], sv[RF_CPT];
#pragma unroll
    for (int j = 0; j < RF_CPT; ++j) {
      c[j] = wave_scan_incl(mv[j] ? 1 : 0);
      sv[j] = wave_scan_incl(mv[j] ? ov[j] : 0);
    }
    if (lane == 63) {
#pragma unroll
      for (int j = 0; j < RF_CPT; ++j) {
        wc[j][wave] = c[j];
        wsum[j][wave] = sv[j];
      }
    }
    __syncthreads();
    // chunk j, wave w starts after the whole chunks before j and the waves
    // of chunk j before w
#pragma unroll
    for (int j = 0; j < RF_CPT; ++j) {
      int bc = carry_c, bs = carry_s;
      for (int w = 0; w < wave; ++w) {
        bc += wc[j][w];
        bs += wsum[j][w];
      }
      const int x = x0 + 256 * j + t;
      if (x < W) {
        if (packed) {
          pcr[x + 1] = (int32_t)((uint32_t)(bc + c[j]) | ((uint32_t)(bs + sv[j]) << 12));
        } else {
          pcr[x + 1] = bc + c[j];
          psr[x + 1] = bs + sv[j];
        }
      }
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        carry_c += wc[j][w];
        carry_s += wsum[j][w];
      }
    }
    __syncthreads();  // wc / wsum are rewritten by the next piece
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
constexpr int DISK_TAB = 512, DISK_R32 = 256, DISK_RPK = 63;

template <bool B>
__global__ __launch_bounds__(PIX_T) void fill_disk_kernel(PostPair one, const PostPair *__restrict__ many, int R,
                                                        float frac, int src, int dst, int packed) {
  PAIR;
  __shared__ int hw[2 * DISK_TAB + 1];
  __shared__ int holes[PIX_SEG];
  __shared__ int nholes;
  const int RT = min(R, DISK_TAB);
  for (int i = threadIdx.x; i <= 2 * RT; i += blockDim.x) {
    const int dy = i - RT;
    hw[i] = isqrt_floor(R * R - dy * dy);
  }
  if (threadIdx.x == 0) nholes = 0;
  __syncthreads();
  const int W = P.W, H = P.H, y = bp.y;
  const GLOBAL int16_t *o = gro(P.ob[src]);
  const GLOBAL uint8_t *m = gro(P.mb[src]);
  // copy the segment, and list its holes in LDS (one slot reservation per
  // wave and pass: ballot, then each hole lane at its rank)
  const int lane = threadIdx.x & (WV - 1);
  if (y < H) {
    // the segment's maps are loaded together, then copied and listed
    constexpr int NP = PIX_SEG / PIX_T;
    const int x1 = min(W, (bp.x + 1) * PIX_SEG), xb = bp.x * PIX_SEG + (int)threadIdx.x;
    int16_t ov[NP];
    uint8_t mv[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const int x = xb + i * PIX_T;
      ov[i] = x < x1 ? o[(size_t)y * W + x] : (int16_t)0;
      mv[i] = x < x1 ? m[(size_t)y * W + x] : (uint8_t)1;
    }
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const int x = xb + i * PIX_T;
      if (x < x1) {
        const size_t k = (size_t)y * W + x;
        grw(P.ob[dst])[k] = ov[i];
        grw(P.mb[dst])[k] = mv[i];
      }
      const bool hole = x < x1 && mv[i] == 0;
      const uint64_t hm = ballot64(hole);
      int base = 0;
      if (lane == 0 && hm) base = atomicAdd(&nholes, __builtin_popcountll(hm));
      base = __shfl(base, 0, WV);
      if (hole) holes[base + __builtin_popcountll(hm & lanes_below(lane))] = x;
    }
  }
  __syncthreads();
  if (y >= H) return;  // uniform per block
  // the disk sums, one hole per thread
  const int nh = nholes;
  const GLOBAL int32_t *__restrict__ pc = gro(P.pc);
  const GLOBAL int32_t *__restrict__ ps = gro(P.ps);
  if (packed) {
    // one load at either end of a disk row (the address unit, not the bytes,
    // bounds this loop): the difference of two packed prefixes is cnt +
    // sum * 4096 exactly as an int32, since a row segment holds at most
    // 2 DISK_RPK + 1 = 127 cells (cnt in [0, 127]) of |o| <= 4096 (|sum| <
    // 2^19), and the counts below 4096 never wrap
    for (int i = threadIdx.x; i < nh; i += PIX_T) {
      const int x = holes[i];
      const size_t k = (size_t)y * W + x;
      int cells = 0, cnt = 0, sum = 0;
      const int ya = max(-R, -y), yb = min(R, H - 1 - y);
      const GLOBAL char *pcb = (const GLOBAL char *)pc;
      uint32_t ro = 4u * (uint32_t)(y + ya) * (uint32_t)(W + 1);
#pragma unroll 8
      for (int dy = ya; dy <= yb; ++dy, ro += 4u * (uint32_t)(W + 1)) {
        const int w = hw[dy + RT];
        const int xl = max(0, x - w), xh = min(W - 1, x + w);
        cells += xh - xl + 1;
        const int d = (int)(*(const GLOBAL uint32_t *)(pcb + ro + 4u * (uint32_t)(xh + 1)) -
                            *(const GLOBAL uint32_t *)(pcb + ro + 4u * (uint32_t)xl));
        cnt += d & 0xFFF;
        sum += d >> 12;
      }
      const double need = ceil((double)frac * (double)cells);
      if (cnt > 0 && (double)cnt >= need) {
        grw(P.ob[dst])[k] = (int16_t)round_half_even(sum, cnt);
        grw(P.mb[dst])[k] = 2;
      }
    }
    return;
  }
  if (R <= DISK_R32) {
    // every sum fits 32 bits: (2R+1)^2 cells of |o| <= 4096 stay below 2^31
    for (int i = threadIdx.x; i < nh; i += PIX_T) {
      const int x = holes[i];
      const size_t k = (size_t)y * W + x;
      int cells = 0, cnt = 0, sum = 0;
      const int ya = max(-R, -y), yb = min(R, H - 1 - y);
      // byte offsets into the prefix planes (under 4 GiB): the row part is
      // the same for every lane, the column part a 32-bit lane offset
      const GLOBAL char *pcb = (const GLOBAL char *)pc, *psb = (const GLOBAL char *)ps;
      uint32_t ro = 4u * (uint32_t)(y + ya) * (uint32_t)(W + 1);
#pragma unroll 8
      for (int dy = ya; dy <= yb; ++dy, ro += 4u * (uint32_t)(W + 1)) {
        const int w = hw[dy + RT];
        const int xl = max(0, x - w), xh = min(W - 1, x + w);
        cells += xh - xl + 1;
        const uint32_t oh = ro + 4u * (uint32_t)(xh + 1), ol = ro + 4u * (uint32_t)xl;
        cnt += *(const GLOBAL int32_t *)(pcb + oh) - *(const GLOBAL int32_t *)(pcb + ol);
        sum += *(const GLOBAL int32_t *)(psb + oh) - *(const GLOBAL int32_t *)(psb + ol);
      }
      const double need = ceil((double)frac * (double)cells);
      if (cnt > 0 && (double)cnt >= need) {
        grw(P.ob[dst])[k] = (int16_t)round_half_even(sum, cnt);
        grw(P.mb[dst])[k] = 2;
      }
    }
    return;
  }
  for (int i = threadIdx.x; i < nh; i += PIX_T) {
    const int x = holes[i];
    const size_t k = (size_t)y * W + x;
    long long cells = 0, cnt = 0, sum = 0;
    const int ya = max(-R, -y), yb = min(R, H - 1 - y);
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
  }
}

// ---------------------------------------------------------------- smoothing (FP64)
// Planes of P.f: 0 b_1 = a - s, 1 b, 2 box(m) (as float), 3 column pass,
// 4 a = A(s), 5 d / b.
enum { F_S = 0, F_IN = 1, F_CNT = 2, F_TMP = 3, F_A = 4, F_D = 5 };

// s = o + delta for matched pixels (code 1), o for filled ones (code 2), or
// the given s_in.
__device__ __forceinline__ double hc_s_at(const PostPair &P, size_t k, uint8_t mk, int osrc,
                                          int use_delta) {
  if (P.s_in) return (double)gro(P.s_in)[k];
  const double o = (double)gro(P.ob[osrc])[k];
  return (mk == 1 && use_delta) ? o + (double)gro(P.delta)[k] : o;
}

// One box pass: its input, output stage and the smoothing's inputs.
//   in >= 0: plane in of P.f; BOX_IN_MASK: the mask (1 on valid pixels);
//   BOX_IN_S: s on valid pixels, 0 elsewhere (formed on the fly).
//   mode / out / alpha: see box_store; src: plane of the mask; osrc and
//   use_delta: where s comes from (hc_s_at).
enum { BOX_IN_MASK = -1, BOX_IN_S = -2 };
struct BoxArgs {
  int R, in, out, mode, src, osrc, use_delta;
  int sy;      // rows per block of the fused pass
  int counts;  // 1: the pass also boxes the mask (mode 4, input BOX_IN_S) and
               // stores the counts, instead of reading them
  double alpha;
};

__device__ __forceinline__ double box_in(const PostPair &P, const BoxArgs &A, size_t N, size_t k) {
  if (A.in >= 0) return gro(P.f)[(size_t)A.in * N + k];
  const uint8_t mk = gro(P.mb[A.src])[k];
  if (A.in == BOX_IN_MASK) return mk ? 1.0 : 0.0;
  return mk ? hc_s_at(P, k, mk, A.osrc, A.use_delta) : 0.0;
}

// Box sums over a (2R+1) window along columns into plane F_TMP: a thread
// owns one column and a segment of seg rows, seeds the window sum, then
// slides it.
template <bool B>
__global__ void box_v_kernel(PostPair one, const PostPair *__restrict__ many, BoxArgs A, int seg) {
  PAIR;
  const int x = bp.x * blockDim.x + threadIdx.x;
  const int y0 = bp.y * seg;
  const int H = P.H, W = P.W, R = A.R;
  if (x >= W || y0 >= H) return;
  const size_t N = (size_t)W * H;
  GLOBAL double *__restrict__ fo = grw(P.f) + F_TMP * N;
  double s = 0.0;
  const int va = max(0, y0 - R), vb = min(H - 1, y0 + R);
#pragma unroll 8
  for (int v = va; v <= vb; ++v) s += box_in(P, A, N, (size_t)v * W + x);
  const int y1 = min(y0 + seg, H);
#pragma unroll 4
  for (int y = y0; y < y1; ++y) {
    fo[(size_t)y * W + x] = s;
    const int a = y + R + 1, b = y - R;
    const double ea = a < H ? box_in(P, A, N, (size_t)a * W + x) : 0.0;
    const double eb = b >= 0 ? box_in(P, A, N, (size_t)b * W + x) : 0.0;
    s += ea;
    s -= eb;
  }
}

// Output stage of a box pass with window sum v at pixel k: the counts of
// valid pixels (mode 0: the box sum of the mask, stored as float - an exact
// small integer - in plane F_CNT), or the masked mean steps fused into it:
//   mode 2: d = a - box(b m)/box(m) (Eq. 3) -> F_D
//   mode 3: the same d written as the final disparity (NaN where invalid)
//           and mask
//   mode 4: a = box(s m)/box(m) (Eq. 1) -> F_A, and b_1 = a - alpha s -
//           (1 - alpha) s (Eq. 2 of the first iteration, d_prev = s) ->
//           plane out
//   mode 5: the next iteration's b = a - alpha s - (1 - alpha) d (Eq. 2)
//           with d = a - box(b m)/box(m) (Eq. 3), formed as
//           c + (1 - alpha) box(b m)/box(m) with c = alpha (a - s) =
//           alpha b_1 (plane F_S) -> plane out
//   mode 6: (re-search, where s changes between iterations) a -> F_A as in
//           mode 4, and b = a - alpha s - (1 - alpha) d_prev (Eq. 2) with
//           d_prev the previous iteration's d (plane F_D) and s from plane
//           F_S, the re-search's output -> plane out
// (b and a are 0 on invalid pixels, as the masked sums need.)  The inputs
// the stage reads are gathered first (box_store_in), so that a caller can
// load them ahead of time.
struct BoxStoreIn {
  uint8_t mk;
  float cnt;
  double a, s;  // a (d_prev in mode 6); s (modes 4, 6) or b_1 (mode 5)
};
__device__ __forceinline__ BoxStoreIn box_store_in(const PostPair &P, const BoxArgs &A, size_t N,
                                                   size_t k) {
  BoxStoreIn q;
  q.mk = 0;
  q.cnt = 1.0f;
  q.a = 0.0;
  q.s = 0.0;
  if (A.mode == 0) return q;
  q.mk = gro(P.mb[A.src])[k];
  if (!A.counts) q.cnt = ((const GLOBAL float *)(gro(P.f) + (size_t)F_CNT * N))[k];
  if (A.mode == 2 || A.mode == 3) q.a = gro(P.f)[(size_t)F_A * N + k];
  if (A.mode == 5) q.s = gro(P.f)[(size_t)F_S * N + k];
  if (A.mode == 6) {
    q.a = gro(P.f)[(size_t)F_D * N + k];
    q.s = gro(P.f)[(size_t)F_S * N + k];
  }
  if (A.mode == 4) {
    // s without a branch on the mask: both loads issue at once
    if (P.s_in) {
      q.s = (double)gro(P.s_in)[k];
    } else {
      const double o = (double)gro(P.ob[A.osrc])[k];
      const double dl = A.use_delta ? (double)gro(P.delta)[k] : 0.0;
      q.s = q.mk == 1 ? o + dl : o;
    }
  }
  return q;
}
__device__ __forceinline__ void box_store(const PostPair &P, const BoxArgs &A, size_t N, size_t k,
                                          double v, const BoxStoreIn &q) {
  if (A.mode == 0) {
    ((GLOBAL float *)(grw(P.f) + (size_t)F_CNT * N))[k] = (float)v;
    return;
  }
  const uint8_t mk = q.mk;
  const double mean = v / (double)q.cnt;
  if (A.mode == 4 || A.mode == 6) {
    P.f[(size_t)F_A * N + k] = mk ? mean : 0.0;
    // b_1 = a - alpha s - (1 - alpha) d_0 with d_0 = s (the later passes of
    // the plain path take c = alpha (a - s) = alpha b_1 from this plane), or
    // b = a - alpha s - (1 - alpha) d_prev
    const double s = mk ? q.s : 0.0;
    const double dp = A.mode == 4 ? s : q.a;
    P.f[(size_t)A.out * N + k] = mk ? mean - A.alpha * s - (1.0 - A.alpha) * dp : 0.0;
    return;
  }
  if (A.mode == 5) {
    // b_{k+1} = c + (1 - alpha) box(b_k m) / box(m), c = alpha b_1 (q.s)
    P.f[(size_t)A.out * N + k] = mk ? A.alpha * q.s + (1.0 - A.alpha) * mean : 0.0;
    return;
  }
  const double d = mk ? q.a - mean : 0.0;
  if (A.mode == 2) {
    P.f[(size_t)F_D * N + k] = d;
  } else {
    P.disparity[k] = mk ? (float)d : __builtin_nanf("");
    if (P.valid_mask) P.valid_mask[k] = mk;
  }
}
__device__ __forceinline__ void box_store(const PostPair &P, const BoxArgs &A, size_t N, size_t k,
                                          double v) {
  box_store(P, A, N, k, v, box_store_in(P, A, N, k));
}

// 2-D box sum over the (2R+1)^2 window of the pass's input (clipped at the
// image border) in one pass, written through box_store.  A block of BX_T
// threads owns BX_T columns, of which the middle BX_T - 2R are output, and a
// segment of A.sy rows: each thread keeps the vertical window sum of its
// column in a register and slides it down the segment.  Per row the
// horizontal sums are differences of the block's prefix sum, with one block
// barrier: every wave stores its own inclusive scan and its total in LDS,
// and a thread forms the prefix at the two window ends from the scan value
// there plus the totals of the waves before it.  The input plane must
// differ from every plane the output stage writes.  CNT: the same pass
// boxes the mask as well (an integer sum beside the FP64 one) and stores the
// counts, so that the first smoothing pass needs no counts pass before it.
constexpr int BX_T = 256, BX_RMAX = 96;
constexpr int BX_SY = 32;  // rows per segment (64 measured slower: half the blocks)
constexpr int BX_SYMIN = 4;  // one 960x540 pair: 4 rows (2 measured slower)
template <bool B, bool CNT>
__global__ __launch_bounds__(BX_T) void box2d_kernel(PostPair one, const PostPair *__restrict__ many,
                                                     BoxArgs A) {
  PAIR;
  // block prefix sums of two rows (slots 0 and 1) and their wave totals
  __shared__ double pf[2][BX_T];
  __shared__ double wt[2][BX_T / WV];
  __shared__ int pfc[CNT ? 2 : 1][CNT ? BX_T : 1];
  __shared__ int wtc[CNT ? 2 : 1][BX_T / WV];
  const int H = P.H, W = P.W, R = A.R;
  const int nout = BX_T - 2 * R;
  const int xo = bp.x * nout, y0 = bp.y * A.sy;
  if (xo >= W || y0 >= H) return;  // uniform per block
  const size_t N = (size_t)W * H;
  const int t = threadIdx.x, lane = t & (WV - 1), wave = t / WV, c = xo - R + t;
  const bool cin = c >= 0 && c < W;
  // input at row r of the column, and (CNT) whether it is a valid pixel
  auto px = [&](int r, int &cm) -> double {
    cm = 0;
    if (!(cin && r >= 0 && r < H)) return 0.0;
    const size_t k = (size_t)r * W + c;
    if constexpr (CNT) {
      // mask, disparity and offset loaded together (no load behind the mask)
      const uint8_t mk = gro(P.mb[A.src])[k];
      double sv;
      if (P.s_in) {
        sv = (double)gro(P.s_in)[k];
      } else {
        const double o = (double)gro(P.ob[A.osrc])[k];
        const double dl = A.use_delta ? (double)gro(P.delta)[k] : 0.0;
        sv = mk == 1 ? o + dl : o;
      }
      cm = mk ? 1 : 0;
      return mk ? sv : 0.0;
    } else {
      return box_in(P, A, N, k);
    }
  };
  double s = 0.0;
  int sc = 0;
#pragma unroll 8
  for (int r = y0 - R; r < y0 + R; ++r) {
    int cm;
    s += px(r, cm);
    sc += cm;
  }
  const bool out_col = c >= xo && c < xo + nout && c < W;  // then R <= t < BX_T - R
  const int y1 = min(y0 + A.sy, H);
  // a row's inputs (entering and leaving rows, output-stage operands) are
  // loaded two rows ahead
  struct RowIn {
    double add, sub;
    int addc, subc;
    BoxStoreIn st;
  };
  auto fetch = [&](int y) -> RowIn {
    RowIn q;
    q.add = px(y + R, q.addc);
    q.sub = px(y - R, q.subc);
    q.st = out_col ? box_store_in(P, A, N, (size_t)y * W + c) : BoxStoreIn{};
    return q;
  };
  // the column sums of a row, scanned along each wave; the wave totals go
  // to slot b
  auto stage = [&](int b, const RowIn &q, double &p, int &pc) {
    s += q.add;
    p = s;
    s -= q.sub;
    pc = 0;
    if constexpr (CNT) {
      sc += q.addc;
      pc = sc;
      sc -= q.subc;
    }
    p = wave_scan_incl(p);
    if constexpr (CNT) pc = wave_scan_incl(pc);
    if (lane == WV - 1) {
      wt[b][wave] = p;
      if constexpr (CNT) wtc[b][wave] = pc;
    }
  };
  // the block prefix: the totals of the waves before this one added
  auto finish = [&](int b, double p, int pc) {
    for (int w = 0; w < wave; ++w) {
      p += wt[b][w];
      if constexpr (CNT) pc += wtc[b][w];
    }
    pf[b][t] = p;
    if constexpr (CNT) pfc[b][t] = pc;
  };
  auto emit = [&](int b, int y, const RowIn &q) {
    if (!out_col) return;
    BoxStoreIn st = q.st;
    const size_t k = (size_t)y * W + c;
    if constexpr (CNT) {
      const int cnt = pfc[b][t + R] - (t - R - 1 >= 0 ? pfc[b][t - R - 1] : 0);
      st.cnt = (float)cnt;
      ((GLOBAL float *)(grw(P.f) + (size_t)F_CNT * N))[k] = st.cnt;
    }
    box_store(P, A, N, k, pf[b][t + R] - (t - R - 1 >= 0 ? pf[b][t - R - 1] : 0.0), st);
  };
  RowIn q0 = y0 < y1 ? fetch(y0) : RowIn{};
  RowIn q1 = y0 + 1 < y1 ? fetch(y0 + 1) : RowIn{};
  // y1 - y0 is uniform: every thread takes the same rows and barriers.  Slot
  // 0 row y, slot 1 row y + 1.  The first barrier: the wave totals are
  // written before they are read, and the previous pair's outputs have read
  // the prefix sums before they are written again.  The second: the prefix
  // sums are complete before the outputs read them, and the totals read
  // before the next pair writes them.
  for (int y = y0; y < y1; y += 2) {
    const RowIn c0 = q0, c1 = q1;
    const bool two = y + 1 < y1;
    if (y + 2 < y1) q0 = fetch(y + 2);
    if (y + 3 < y1) q1 = fetch(y + 3);
    double p0, p1 = 0.0;
    int pc0, pc1 = 0;
    stage(0, c0, p0, pc0);
    if (two) stage(1, c1, p1, pc1);
    __syncthreads();
    finish(0, p0, pc0);
    if (two) finish(1, p1, pc1);
    __syncthreads();
    emit(0, y, c0);
    if (two) emit(1, y + 1, c1);
  }
}

// Row pass over the column sums in F_TMP (one thread per row segment).
template <bool B>
__global__ void box_h_kernel(PostPair one, const PostPair *__restrict__ many, BoxArgs A, int seg) {
  PAIR;
  const int y = bp.x * blockDim.x + threadIdx.x;
  const int x0 = bp.y * seg;
  const int H = P.H, W = P.W, R = A.R;
  if (y >= H || x0 >= W) return;
  const size_t N = (size_t)W * H;
  const double *row = P.f + F_TMP * N + (size_t)y * W;
  double s = 0.0;
  for (int u = x0 - R; u <= x0 + R; ++u)
    if (u >= 0 && u < W) s += row[u];
  const int x1 = min(x0 + seg, W);
  for (int x = x0; x < x1; ++x) {
    box_store(P, A, N, (size_t)y * W + x, s);
    const int a = x + R + 1, b = x - R;
    if (a < W) s += row[a];
    if (b >= 0) s -= row[b];
  }
}

// Row pass over the column sums in F_TMP through LDS: one block per row
// stages the row, takes an inclusive prefix sum and writes out(x) =
// P(min(x+R, W-1)) - P(x-R-1), with coalesced loads and stores.  Rows up to
// BOXH_MAXW wide.
constexpr int BOXH_MAXW = 4096;
template <bool B>
__global__ __launch_bounds__(256) void box_h_lds_kernel(PostPair one, const PostPair *__restrict__ many,
                                                        BoxArgs A) {
  PAIR;
  __shared__ double row[BOXH_MAXW];
  __shared__ double part[256];
  const int y = bp.x;
  const int H = P.H, W = P.W, R = A.R;
  if (y >= H) return;
  const size_t N = (size_t)W * H;
  const double *rin = P.f + F_TMP * N + (size_t)y * W;
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
    box_store(P, A, N, (size_t)y * W + x, row[a] - (b >= 0 ? row[b] : 0.0));
  }
}

// ---- Eq. (4): re-search of the discrete disparities around d.  A block
// covers the sub-pixel kernel's band (SP_TX columns, SPB_TY rows) and builds
// the same packed stage: the L columns of the band's windows and the R
// columns from the block's largest candidate down to its smallest.  A lane
// takes a pixel's candidates four at a time; each window sum is exact
// (v_dot4_u32_u8 on aligned dwords), z and the cost in FP64, in ascending
// candidate order so that the first of equal costs is kept.

// Window sums of the candidates c0 .. c0 + 3 of a pixel whose window starts
// at packed row r0 and L stage column tx; rs is the R stage column of window
// column 0 at candidate c0 + 3 (candidate c0 + e at rs + 3 - e).  Reads
// stage columns rs .. rs + WIN + 2 of the R part.  When c0 + 3 is past the
// block's largest candidate, rs is down to -3: those reads land in the L
// part of the same packed row (inside the stage), and only the sums of the
// candidates past the pixel's last one, which are never used, take them.
template <int WIN, bool CH>
__device__ __forceinline__ void rs_sums4(const uint32_t *Pk, int S, int QL, int r0, int tx, int rs,
                                         uint32_t (&acc)[4]) {
  constexpr int NG = (WIN + 3) / 4, LAST = WIN - 4 * (NG - 1);
  constexpr uint32_t lastmask = LAST == 4 ? 0xFFFFFFFFu : (1u << (8 * LAST)) - 1u;
#pragma unroll
  for (int e = 0; e < 4; ++e) acc[e] = 0;
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    const uint32_t *lrow = Pk + (r0 + 4 * g) * S + tx;
    const uint32_t *rrow = Pk + (r0 + 4 * g) * S + 4 * QL + rs;
    uint32_t rv[WIN + 3];
#pragma unroll
    for (int u = 0; u < WIN + 3; ++u) rv[u] = rrow[u];
#pragma unroll
    for (int u = 0; u < WIN; ++u) {
      uint32_t m = g == NG - 1 ? lastmask : 0xFFFFFFFFu;
      if (CH) m &= (u & 1) ? 0xFF00FF00u : 0x00FF00FFu;
      const uint32_t l = m == 0xFFFFFFFFu ? lrow[u] : lrow[u] & m;
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[e] = __builtin_amdgcn_udot4(l, rv[u + 3 - e], acc[e], false);
    }
    asm volatile("" : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3]));
  }
}

// The re-searched disparity of pixel k (band row r0, L stage column tx):
// the candidate c in [lo, hi] of least cost 1 / max(z, 1e-3) + eta (c - d)^2,
// candidates whose right window has no variance skipped; o when none is left
// or the left window has no variance.
template <int WIN, bool CH>
__device__ __forceinline__ int rs_best(const PostPair &P, const uint32_t *Pk, int S, int QL, int r0,
                                       int tx, size_t k, int lo, int hi, double d, int cmax,
                                       double eta, int o) {
  const long long n = CH ? ((long long)WIN * WIN + 1) / 2 : (long long)WIN * WIN;
  const long long sl = P.SL[k];
  const long long varL = n * (long long)P.SSL[k] - sl * sl;
  if (varL <= 0) return o;
  double best = __builtin_inf();
  int onew = o;
  for (int c0 = lo; c0 <= hi; c0 += 4) {
    uint32_t acc[4];
    rs_sums4<WIN, CH>(Pk, S, QL, r0, tx, tx + cmax - (c0 + 3), acc);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int c = c0 + e;
      if (c > hi) break;
      const size_t kr = k - c;
      const long long sr = P.SR[kr];
      const long long varR = n * (long long)P.SSR[kr] - sr * sr;
      if (varR <= 0) continue;
      const double z = (double)(n * (long long)acc[e] - sl * sr) / sqrt((double)varL * (double)varR);
      const double ec = (double)c - d;
      const double cost = 1.0 / (z > 1e-3 ? z : 1e-3) + eta * ec * ec;
      if (cost < best) {
        best = cost;
        onew = c;
      }
    }
  }
  return onew;
}

// Pk: the packed stage in dynamic LDS, sp_lds_bytes(win, dmax - dmin + 1,
// TY) bytes at least (the block's candidates lie in [dmin, dmax]).  TY: rows
// per band, 8 as in the sub-pixel kernel, or 4 for launches with few blocks
// (a single pair), where the shorter bands' extra packing costs less than
// the idle SIMDs.  splane: also write the new o on valid pixels (0
// elsewhere) as FP64 into plane F_S, the next smoothing pass's input.
template <bool B, int TY>
__global__ __launch_bounds__(SPB_T) void research_kernel(PostPair one, const PostPair *__restrict__ many,
                                                         int osrc, int msrc, int odst, int dplane,
                                                         int range, double eta, int splane) {
  constexpr int NPT = TY * SP_TX / SPB_T;  // pixels per thread (rows ty + 2 j)
  PAIR;
  uint32_t *Pk = sp_dyn;
  __shared__ int s_cmin, s_cmax;
  const int tid = threadIdx.x, tx = tid & (SP_TX - 1), ty = tid / SP_TX;
  const int x0 = bp.x * SP_TX, y0 = bp.y * TY;
  if (x0 >= P.W || y0 >= P.H) return;  // uniform per block
  const int W = P.W, H = P.H, win = P.win, h = win / 2;
  const int x = x0 + tx;
  const size_t N = (size_t)W * H;
  int lo[NPT], hi[NPT];
  double dd[NPT];
  int cl = 1 << 30, chi = -(1 << 30);
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    const int y = y0 + ty + 2 * j;
    const size_t k = (size_t)y * W + x;
    // pixels whose own window is inside the image can have a defined
    // candidate; a candidate's right window must be inside as well
    const bool inside = x < W && y < H && x >= h && x <= W - 1 - h && y >= h && y <= H - 1 - h;
    const uint8_t mk = inside ? P.mb[msrc][k] : 0;
    dd[j] = mk ? P.f[(size_t)dplane * N + k] : 0.0;
    lo[j] = 0;
    hi[j] = -1;
    if (mk) {
      lo[j] = max(max(P.dmin, (int)ceil(dd[j] - range)), x - (W - 1 - h));
      hi[j] = min(min(P.dmax, (int)floor(dd[j] + range)), x - h);
    }
    if (lo[j] <= hi[j]) {
      cl = min(cl, lo[j]);
      chi = max(chi, hi[j]);
    }
  }
  if (tid == 0) {
    s_cmin = 1 << 30;
    s_cmax = -(1 << 30);
  }
  __syncthreads();
  cl = wave_min(cl);
  chi = wave_max(chi);
  if ((tid & (WV - 1)) == 0 && cl <= chi) {
    atomicMin(&s_cmin, cl);
    atomicMax(&s_cmax, chi);
  }
  __syncthreads();
  const int cmin = s_cmin, cmax = s_cmax;
  // stage column c of the R part is R(., x0 - cmax - h + c): window column u
  // of candidate c at pixel x is column tx + cmax - c + u
  const int QL = sp_quads_l(win), QR = cmin <= cmax ? sp_quads_r(win, cmax - cmin) : 0;
  const int S = 4 * (QL + QR);
  if (cmin <= cmax) {
    const int PR = min(TY, H - y0) + 4 * (sp_groups(win) - 1);
    sp_pack(Pk, S, PR, gro(P.left), gro(P.right), P.pitch, (long long)(H - 1) * P.pitch + W, y0 - h,
            x0 - h, QL, x0 - cmax - h, QR, tid);
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    const int r0 = ty + 2 * j, y = y0 + r0;
    if (x >= W || y >= H) continue;
    const size_t k = (size_t)y * W + x;
    int onew = P.ob[osrc][k];
    if (lo[j] <= hi[j]) {
#define RSB(w)                                                                                    \
  case w:                                                                                         \
    onew = P.chess ? rs_best<w, true>(P, Pk, S, QL, r0, tx, k, lo[j], hi[j], dd[j], cmax, eta, onew) \
                   : rs_best<w, false>(P, Pk, S, QL, r0, tx, k, lo[j], hi[j], dd[j], cmax, eta, onew); \
    break
      switch (win) {
        RSB(3);
        RSB(5);
        RSB(7);
        RSB(9);
        RSB(11);
        RSB(13);
        default:
          onew = P.chess ? rs_best<15, true>(P, Pk, S, QL, r0, tx, k, lo[j], hi[j], dd[j], cmax, eta, onew)
                         : rs_best<15, false>(P, Pk, S, QL, r0, tx, k, lo[j], hi[j], dd[j], cmax, eta, onew);
          break;
      }
#undef RSB
    }
    P.ob[odst][k] = (int16_t)onew;
    if (splane) P.f[(size_t)F_S * N + k] = P.mb[msrc][k] ? (double)onew : 0.0;
  }
}

// Output without smoothing (K = 0): s on valid pixels.
template <bool B>
__global__ void hc_copy_kernel(PostPair one, const PostPair *__restrict__ many, int src, int osrc,
                               int use_delta) {
  PAIR;
  const int W = P.W, H = P.H;
  (void)W;
  (void)H;
  for_pixels(P, bp, [&](int x, int y, size_t k) {
    const uint8_t mk = P.mb[src][k];
    P.disparity[k] = mk ? (float)hc_s_at(P, k, mk, osrc, use_delta) : __builtin_nanf("");
    if (P.valid_mask) P.valid_mask[k] = mk;
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
// the same with the batched and single-pair instantiations named
#define LAUNCH_K(kbatch, kone, grid, block, ...)                                         \
  do {                                                                                   \
    if (L.many)                                                                          \
      hipLaunchKernelGGL(kbatch, grid, block, 0, L.s, L.one, L.many, ##__VA_ARGS__);     \
    else                                                                                 \
      hipLaunchKernelGGL(kone, grid, block, 0, L.s, L.one, L.many, ##__VA_ARGS__);       \
  } while (0)

hipError_t launch_mark_invalid(const int16_t *o, const uint8_t *m, int16_t *out, size_t N,
                               hipStream_t s) {
  hipLaunchKernelGGL(mark_invalid_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, o, m, out, N);
  return hipGetLastError();
}
hipError_t post_decode(const PostLaunch &L) {
  LAUNCH(decode_kernel, pixgrid(L), dim3(PIX_T));
  return hipGetLastError();
}
hipError_t post_subpixel(const PostLaunch &L) {
  const dim3 grid(ceil_div(L.maxW, SP_TX), ceil_div(L.maxH, SPB_TY), L.npairs);
  const size_t lds = sp_lds_bytes(L.maxWin, L.maxD);
  if (L.many)
    hipLaunchKernelGGL(subpixel_kernel<true>, grid, dim3(SPB_T), lds, L.s, L.one, L.many);
  else
    hipLaunchKernelGGL(subpixel_kernel<false>, grid, dim3(SPB_T), lds, L.s, L.one, L.many);
  return hipGetLastError();
}
hipError_t post_subpixel_lr(const PostLaunch &L, int tol, int dst) {
  // 4-row bands when the sub-pixel blocks would be fewer than 1024 (a single
  // pair): the extra packing costs less than the idle SIMDs
  const int nspx = ceil_div(L.maxW, SP_TX);
  const bool shortb = (long long)nspx * ceil_div(L.maxH, SPB_TY) * L.npairs < 1024;
  const int ty = shortb ? 4 : SPB_TY, nsp = nspx * ceil_div(L.maxH, ty);
  const int nlrx = ceil_div(L.maxW, PIX_SEG), nlr = nlrx * L.maxH;
  const dim3 grid(nsp + nlr, 1, L.npairs);
  const size_t lds = sp_lds_bytes(L.maxWin, L.maxD, ty);
#define SPL(b, t) \
  hipLaunchKernelGGL((subpixel_lr_kernel<b, t>), grid, dim3(SPB_T), lds, L.s, L.one, L.many, nspx, nsp, nlrx, tol, dst)
  if (L.many) {
    if (shortb) SPL(true, 4); else SPL(true, SPB_TY);
  } else {
    if (shortb) SPL(false, 4); else SPL(false, SPB_TY);
  }
#undef SPL
  return hipGetLastError();
}
hipError_t post_lr(const PostLaunch &L, int tol, int dst) {
  LAUNCH(lr_check_kernel, pixgrid(L), dim3(PIX_T), tol, dst);
  return hipGetLastError();
}
// blocks of the row scans (4 rows each) and of the column / diagonal scans
static int rowblocks(const PostLaunch &L) { return ceil_div(L.maxH, 4); }
template <int SG>
static int vscanblocks(const PostLaunch &L) {
  int n = 0;
  for (int t = 1; t < 4; ++t) n += vscan_span<SG>(t, L.maxH, L.maxW);
  return ceil_div(n, 256);
}
// Segments of SEG rows, or SEG / 2 when a launch would have fewer than 1024
// blocks (a single pair): the shorter segments' longer relative look-ahead
// costs less than the idle CUs.
static bool short_segments(const PostLaunch &L) {
  return (long long)(rowblocks(L) + vscanblocks<SEG>(L)) * L.npairs < 1024;
}

hipError_t post_outlier(const PostLaunch &L, int r, float thresh, int src, int dst) {
  const int nrow = rowblocks(L);
  if (short_segments(L))
    LAUNCH_K((outlier_scan_kernel<true, SEG / 2>), (outlier_scan_kernel<false, SEG / 2>),
             dim3(nrow + vscanblocks<SEG / 2>(L), 1, L.npairs), dim3(256), r, thresh, src, nrow);
  else
    LAUNCH_K((outlier_scan_kernel<true, SEG>), (outlier_scan_kernel<false, SEG>),
             dim3(nrow + vscanblocks<SEG>(L), 1, L.npairs), dim3(256), r, thresh, src, nrow);
  LAUNCH(outlier_combine_kernel, pixgrid(L), dim3(PIX_T), src, dst);
  return hipGetLastError();
}
// radial fill src -> tmp, disk fill tmp -> dst (dst may equal src)
hipError_t post_fill(const PostLaunch &L, int radial_r, int min_lines, int disk_r, float frac,
                     int src, int tmp, int dst) {
  const int nrow = rowblocks(L);
  if (short_segments(L))
    LAUNCH_K((fill_scan_kernel<true, SEG / 2>), (fill_scan_kernel<false, SEG / 2>),
             dim3(nrow + vscanblocks<SEG / 2>(L), 1, L.npairs), dim3(256), radial_r, src, nrow);
  else
    LAUNCH_K((fill_scan_kernel<true, SEG>), (fill_scan_kernel<false, SEG>),
             dim3(nrow + vscanblocks<SEG>(L), 1, L.npairs), dim3(256), radial_r, src, nrow);
  // packed row prefixes when every pair of the launch allows them
  const int packed = disk_r <= DISK_RPK && L.maxW < 4096 ? 1 : 0;
  LAUNCH(fill_radial_kernel, dim3(L.maxH, 1, L.npairs), dim3(256), min_lines, src, tmp, packed);
  LAUNCH(fill_disk_kernel, pixgrid(L), dim3(PIX_T), disk_r, frac, tmp, dst, packed);
  return hipGetLastError();
}

// Box sum over the (2R+1)^2 window of the pass's input, stored by
// box_store's mode: one fused pass for R <= BX_RMAX, else a column pass into
// F_TMP and a row pass (the input and the written planes must then differ
// from F_TMP).
static void box2d(const PostLaunch &L, BoxArgs A) {
  if (A.R <= BX_RMAX) {
    // 32-row segments, shorter (down to BX_SYMIN rows) when that leaves
    // fewer than about 1024 blocks (a single pair): the seed of 2R rows per
    // segment is the price of more blocks in flight
    const int nout = BX_T - 2 * A.R, nx = ceil_div(L.maxW, nout);
    A.sy = BX_SY;
    while (A.sy > BX_SYMIN && (long long)nx * ceil_div(L.maxH, A.sy) * L.npairs < 1024) A.sy /= 2;
    const dim3 grid(nx, ceil_div(L.maxH, A.sy), L.npairs);
    if (A.counts) {
      LAUNCH_K((box2d_kernel<true, true>), (box2d_kernel<false, true>), grid, dim3(BX_T), A);
    } else {
      LAUNCH_K((box2d_kernel<true, false>), (box2d_kernel<false, false>), grid, dim3(BX_T), A);
    }
    return;
  }
  if (A.counts) {  // column and row passes: the counts first
    BoxArgs C = A;
    C.in = BOX_IN_MASK;
    C.mode = 0;
    C.counts = 0;
    box2d(L, C);
    A.counts = 0;
  }
  const int seg = 32;
  LAUNCH(box_v_kernel, dim3(ceil_div(L.maxW, 64), ceil_div(L.maxH, seg), L.npairs), dim3(64), A, seg);
  if (L.maxW <= BOXH_MAXW)
    LAUNCH(box_h_lds_kernel, dim3(L.maxH, 1, L.npairs), dim3(256), A);
  else
    LAUNCH(box_h_kernel, dim3(ceil_div(L.maxH, 64), ceil_div(L.maxW, seg), L.npairs), dim3(64), A, seg);
}

// Improved Laplacian smoothing of (ob[src], delta, mb[src]) or s_in; writes
// disparity (NaN where invalid) and valid_mask.
static void launch_research(const PostLaunch &L, int osrc, int msrc, int odst, int dplane, int range,
                            double eta, int splane) {
  const int gx = ceil_div(L.maxW, SP_TX);
  const bool shortb = (long long)gx * ceil_div(L.maxH, SPB_TY) * L.npairs < 1024;
  const int ty = shortb ? 4 : SPB_TY;
  const dim3 grid(gx, ceil_div(L.maxH, ty), L.npairs);
  const size_t lds = sp_lds_bytes(L.maxWin, L.maxD, ty);
#define RSL(b, t) \
  hipLaunchKernelGGL((research_kernel<b, t>), grid, dim3(SPB_T), lds, L.s, L.one, L.many, osrc, msrc, odst, dplane, range, eta, splane)
  if (L.many) {
    if (shortb) RSL(true, 4); else RSL(true, SPB_TY);
  } else {
    if (shortb) RSL(false, 4); else RSL(false, SPB_TY);
  }
#undef RSL
}
hipError_t post_research(const PostLaunch &L, int osrc, int msrc, int odst, int dplane, int range,
                         float eta) {
  launch_research(L, osrc, msrc, odst, dplane, range, (double)eta, 0);
  return hipGetLastError();
}

hipError_t post_hc(const PostLaunch &L, int src, int R, int K, float alpha, int use_delta,
                   int research, int range, float eta, const HcTrace *trace) {
  if (K == 0) {
    LAUNCH(hc_copy_kernel, pixgrid(L), dim3(PIX_T), src, src, use_delta);
    return hipGetLastError();
  }
  // research: Eqs. (1)-(4), the discrete o (no sub-pixel offset) is smoothed
  // and re-searched after every iteration but the last; o ping-pongs between
  // the two fill planes while the mask stays in plane src
  int ocur = src, oalt = src == 1 ? 2 : 1;
  if (research) use_delta = 0;
  auto args = [&](int in, int out, int mode) {
    BoxArgs A;
    A.R = R;
    A.in = in;
    A.out = out;
    A.mode = mode;
    A.src = src;
    A.osrc = ocur;
    A.use_delta = use_delta;
    A.sy = 32;
    A.counts = 0;
    A.alpha = (double)alpha;
    return A;
  };
  if (!research) {
    // a is fixed and s is formed on the fly from the disparities; every b
    // (Eq. 2) is formed in the output stage of the box pass before it.  b_1
    // = a - s stays in plane F_S: with c = alpha (a - s) = alpha b_1,
    // b_{k+1} = c + (1 - alpha) box(b_k m)/box(m), the later b alternating
    // between the planes F_D and F_IN, and only the last pass forms
    // d = a - box(b m)/box(m)
    BoxArgs first = args(BOX_IN_S, F_S, 4);  // a = box(s m) / box(m), b_1 -> F_S,
    first.counts = 1;                         // and the counts box(m) in the same pass
    box2d(L, first);
    int bin = F_S, bout = F_D;
    for (int it = 0; it < K; ++it) {
      box2d(L, args(bin, bout, it == K - 1 ? 3 : 5));  // d = a - box(b m) / box(m)
      bin = bout;
      bout = bout == F_D ? F_IN : F_D;
    }
    return hipGetLastError();
  }
  // per iteration two passes: a = box(o m) / box(m) from the current o
  // (formed on the fly from the map in the first iteration, later read from
  // the plane F_S that the re-search writes) with b = a - alpha o -
  // (1 - alpha) d_prev in its output stage (the first pass also boxes the
  // mask for the counts), then d = a - box(b m) / box(m)
  for (int it = 0; it < K; ++it) {
    BoxArgs ab = args(it == 0 ? (int)BOX_IN_S : (int)F_S, F_IN, it == 0 ? 4 : 6);
    ab.counts = it == 0 ? 1 : 0;
    box2d(L, ab);
    box2d(L, args(F_IN, F_IN, it == K - 1 ? 3 : 2));
    if (it < K - 1) {
      launch_research(L, ocur, src, oalt, (int)F_D, range, (double)eta, 1);
      if (trace && !L.many && it < trace->n) {
        const size_t N = (size_t)L.one.H * L.one.W;
        hipError_t e = hipMemcpyAsync(trace->o + it * N, L.one.ob[oalt], 2 * N,
                                      hipMemcpyDeviceToDevice, L.s);
        if (e == hipSuccess)
          e = hipMemcpyAsync(trace->d + it * N, L.one.f + (size_t)F_D * N, 8 * N,
                             hipMemcpyDeviceToDevice, L.s);
        if (e != hipSuccess) return e;
      }
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
