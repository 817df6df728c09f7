// Per-pair preparation for the matcher and the sub-pixel stages (Section
// II-A: ZNCC needs the window means and deviations of both images): the
// padded image planes the matcher streams, and the exact window sums with
// the inverse deviations, for the square or the chessboard window.
#include <type_traits>

#include "common.h"

namespace st {

// ---------------------------------------------------------------- preparation
// Padded image planes and the padding of the statistics planes of one pair
// (descriptor by value) or of a batch (table, pair from block_pos).
// A thread fills 4 consecutive plane columns (the strides are multiples of
// 16, so a group never straddles a row end) with one 8-byte store per L plane
// and one 4- or 8-byte store for R.
template <int PREC>
__device__ __forceinline__ uint16_t enc16(int v, int n) {
  if constexpr (PREC == P_I16) return (uint16_t)(int16_t)(n * v);
  else if constexpr (PREC == P_F16) return __builtin_bit_cast(uint16_t, (_Float16)(float)v);
  else return (uint16_t)(__builtin_bit_cast(uint32_t, (float)v) >> 16);
}
// Bytes x0 .. x0 + 3 of an image row of W bytes, byte j of the result (0
// outside the row).  Inside the row the bytes come from one aligned dword,
// or two realigned with v_alignbyte (the misalignment is that of the row
// base, the same for every thread of the row when x0 is a multiple of 4);
// near the row's ends byte by byte, so that no load leaves the row.
__device__ __forceinline__ uint32_t row4(const GLOBAL uint8_t *row, int x0, int W) {
  const int mis = (int)(((uintptr_t)row + (uintptr_t)(intptr_t)x0) & 3);
  const int lo = x0 - mis;
  if (lo >= 0 && lo + (mis ? 8 : 4) <= W) {
    const GLOBAL uint32_t *q = (const GLOBAL uint32_t *)(row + lo);
    return mis ? __builtin_amdgcn_alignbyte(q[1], q[0], mis) : q[0];
  }
  uint32_t v = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int x = x0 + j;
    if (x >= 0 && x < W) v |= (uint32_t)row[x] << (8 * j);
  }
  return v;
}

template <int PREC, bool B>
__global__ void prep_planes_kernel(PrepPair one, const PrepPair *many) {
  const BlockPos bp = block_pos();
  const PrepPair &P = B ? many[bp.pair] : one;
  const int y = bp.y;
  const int c0 = 4 * (bp.x * blockDim.x + threadIdx.x);
  if (y >= P.H) return;
  const int W = P.W;
  const int n = P.chess ? (P.win * P.win + 1) / 2 : P.win * P.win;
  const float qnan = __builtin_nanf("");
  const GLOBAL uint8_t *Lrow = gro(P.L) + (size_t)y * P.pitch;
  const GLOBAL uint8_t *Rrow = gro(P.R) + (size_t)y * P.pitch;
  if (c0 < P.strideL) {
    int v[4];
    bool in[4];
    const uint32_t w4 = row4(Lrow, c0 - P.padL, W);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int x = c0 + j - P.padL;
      in[j] = x >= 0 && x < W;
      v[j] = in[j] ? (int)((w4 >> (8 * j)) & 255u) - 128 : 0;
    }
    const size_t k = (size_t)y * P.strideL + c0;
    // mask: bit j keeps column j (all, or one chessboard colour)
    auto put = [&](size_t kk, int keep) {
      uint64_t a = 0, b = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int vj = (keep >> j) & 1 ? v[j] : 0;
        a |= (uint64_t)enc16<PREC>(vj, n) << (16 * j);
        b |= (uint64_t)enc16<PREC>(-vj, n) << (16 * j);
      }
      *(GLOBAL uint64_t *)((GLOBAL uint16_t *)P.Lp + kk) = a;
      *(GLOBAL uint64_t *)((GLOBAL uint16_t *)P.NLp + kk) = b;
    };
    if (!P.chess) {
      put(k, 15);
    } else {
      // colour copies: (x + y) even in the first, odd in the second
      const int even = ((c0 - P.padL + y) & 1) == 0 ? 0x5 : 0xA;
      put(k, even);
      put(k + (size_t)P.strideL * P.H, even ^ 0xF);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (!in[j]) {
        P.negSL[k + j] = 0;
        P.invL[k + j] = qnan;
      }
  }
  if (c0 < P.strideR) {
    int v[4];
    bool in[4];
    const uint32_t w4 = row4(Rrow, c0 - P.padR, W);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int x = c0 + j - P.padR;
      in[j] = x >= 0 && x < W;
      v[j] = in[j] ? (int)((w4 >> (8 * j)) & 255u) : 0;
    }
    const size_t k = (size_t)y * P.strideR + c0;
    if constexpr (PREC == P_I16) {
      *(GLOBAL uint32_t *)((GLOBAL uint8_t *)P.Rp + k) =
          (uint32_t)v[0] | ((uint32_t)v[1] << 8) | ((uint32_t)v[2] << 16) | ((uint32_t)v[3] << 24);
    } else {
      uint64_t a = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) a |= (uint64_t)enc16<PREC>(v[j], 1) << (16 * j);
      *(GLOBAL uint64_t *)((GLOBAL uint16_t *)P.Rp + k) = a;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (!in[j]) {
        P.SRp[k + j] = 0;
        P.invR[k + j] = qnan;
      }
  }
}

// Window sums S = sum I, SS = sum I^2 and 1/sqrt(n SS - S^2) of every pixel
// whose window lies inside the image (0 / NaN elsewhere).  side 0: left
// image (dense and padded planes), 1: right image, 2: dense planes only;
// NS = 2: both images of the pair in one pass (sides 0 and 1), so that the
// two share every barrier.  A block of WS_T threads owns WS_T columns; each
// thread keeps the vertical window sums of its column down a segment of
// sy rows and the horizontal sums are differences of a block prefix sum
// (wave scans, then the wave totals before each wave added through LDS).
// Two rows share each of the two barriers this takes.  Output columns of a
// block are WS_T - 2 WS_HMAX wide for every window.
// CH (chessboard window): a column keeps separate sums of its cells with
// x + y even and odd; a pixel takes the prefix sums of its own colour, since
// the cells u + v even around (x, y) are exactly those of the colour of
// (x, y).
// sy: 16 rows, halved down to 4 while a launch has fewer than 1024 blocks
// (one 960x540 pair: 4 rows, 544 blocks instead of 136).
constexpr int WS_T = 256, WS_SY = 16, WS_HMAX = 7, WS_NOUT = WS_T - 2 * WS_HMAX;
static dim3 ws_grid(int maxW, int maxH, int npairs, int &sy) {
  const int gx = ceil_div(maxW, WS_NOUT);
  sy = WS_SY;
  while (sy > 4 && (long long)gx * ceil_div(maxH, sy) * npairs < 1024) sy /= 2;
  return dim3(gx, ceil_div(maxH, sy), npairs);
}

template <bool B, bool CH, int NS>
__global__ __launch_bounds__(WS_T) void window_stats_kernel(PrepPair one, const PrepPair *many,
                                                            int side, int sy) {
  const BlockPos bp = block_pos();
  const PrepPair &P = B ? many[bp.pair] : one;
  constexpr int NV = CH ? 4 : 2;  // (S, SS) of each colour
  constexpr int NA = NS * NV;     // sums of a column: per image, per colour
  __shared__ int pf[2][NA][WS_T], wt[2][NA][WS_T / 64];
  const int H = P.H, W = P.W, win = P.win, h = win / 2;
  const int xo = bp.x * WS_NOUT, y0 = bp.y * sy;
  if (xo >= W || y0 >= H) return;  // uniform per block
  // the images of the pass and their sides
  const GLOBAL uint8_t *img[NS];
  int sd[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    sd[i] = NS == 2 ? i : side;
    img[i] = gro(sd[i] == 1 ? P.R : P.L);
  }
  const int t = threadIdx.x, c = xo - h + t;
  const bool cin = c >= 0 && c < W;
  using Px = typename std::conditional<NS == 2, int2, int>::type;
  // the pixel values of row r of the column (0 outside the image)
  auto px = [&](int r) -> Px {
    const bool in = cin && r >= 0 && r < H;
    const size_t k = (size_t)r * P.pitch + c;
    if constexpr (NS == 2) {
      return make_int2(in ? (int)img[0][k] : 0, in ? (int)img[1][k] : 0);
    } else {
      return in ? (int)img[0][k] : 0;
    }
  };
  auto val = [](const Px &p, int i) -> int {
    if constexpr (NS == 2) return i ? p.y : p.x;
    else return p;
  };
  int acc[NA];
#pragma unroll
  for (int i = 0; i < NA; ++i) acc[i] = 0;
  // add (sgn = 1) or remove (sgn = -1) row r of the column, whose pixel
  // values are p
  auto step_v = [&](int r, int sgn, const Px &p) {
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      const int v = sgn * val(p, i), vv = v * (sgn * v);
      int *a = acc + NV * i;
      if constexpr (CH) {
        const bool odd = ((c + r) & 1) != 0;
        a[0] += odd ? 0 : v;
        a[1] += odd ? 0 : vv;
        a[2] += odd ? v : 0;
        a[3] += odd ? vv : 0;
      } else {
        a[0] += v;
        a[1] += vv;
      }
    }
  };
  for (int r = y0 - h; r < y0 + h; ++r) step_v(r, 1, px(r));
  const bool out_col = c >= xo && c < xo + WS_NOUT && c < W;  // then h <= t < WS_T - h
  const int y1 = min(y0 + sy, H);
  const int n = CH ? (win * win + 1) / 2 : win * win;
  const int lane = t & 63, wave = t >> 6;
  // the window sums of row y (add row y + h, then drop row y - h for the
  // next; qa, qd: their pixel values), scanned along each wave; the wave
  // totals go to slot b
  auto stage = [&](int b, int y, const Px &qa, const Px &qd, int (&pv)[NA]) {
    step_v(y + h, 1, qa);
#pragma unroll
    for (int i = 0; i < NA; ++i) pv[i] = acc[i];
    step_v(y - h, -1, qd);
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      pv[i] = wave_scan_incl(pv[i]);
      if (lane == 63) wt[b][i][wave] = pv[i];
    }
  };
  // the block prefix: the totals of the waves before this one added
  auto finish = [&](int b, int (&pv)[NA]) {
    for (int w = 0; w < wave; ++w) {
#pragma unroll
      for (int i = 0; i < NA; ++i) pv[i] += wt[b][i][w];
    }
#pragma unroll
    for (int i = 0; i < NA; ++i) pf[b][i][t] = pv[i];
  };
  auto emit = [&](int b, int y) {
    if (!out_col) return;
    const int x = c;
    const bool inside = x >= h && x <= W - 1 - h && y >= h && y <= H - 1 - h;
    const size_t k = (size_t)y * W + x;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      const int q = NV * i + (CH ? 2 * ((x + y) & 1) : 0);
      int S = pf[b][q][t + h] - (t - h - 1 >= 0 ? pf[b][q][t - h - 1] : 0);
      int SS = pf[b][q + 1][t + h] - (t - h - 1 >= 0 ? pf[b][q + 1][t - h - 1] : 0);
      float iv = __builtin_nanf("");
      if (!inside) {
        S = 0;
        SS = 0;
      } else {
        const long long varN = (long long)n * SS - (long long)S * S;
        // FP64 reciprocal square root (within an ulp of 1/sqrt in FP64),
        // rounded once to float
        if (varN > 0) iv = (float)rsqrt((double)varN);
      }
      if (sd[i] == 1) {
        P.SR[k] = S;
        P.SSR[k] = SS;
        if (P.invRd) P.invRd[k] = iv;
        const size_t kp = (size_t)y * P.strideR + x + P.padR;
        P.SRp[kp] = S;
        P.invR[kp] = iv;
      } else {
        P.SL[k] = S;
        P.SSL[k] = SS;
        if (P.invLd) P.invLd[k] = iv;
        if (sd[i] == 0) {
          const size_t kp = (size_t)y * P.strideL + x + P.padL;
          P.negSL[kp] = 128 * n - S;
          P.invL[kp] = iv;
        }
      }
    }
  };
  // y1 - y0 is uniform: every thread takes the same rows and barriers
  // slot 0 row y, slot 1 row y + 1.  The first barrier: the wave totals are
  // written before they are read, and the previous pair's outputs have read
  // the prefix sums before they are written again.  The second: the prefix
  // sums are complete before the outputs read them, and the totals read
  // before the next pair writes them.
  // the pixels a row's stage adds and drops are loaded two rows ahead
  Px a0 = px(y0 + h), d0 = px(y0 - h);
  Px a1 = px(y0 + 1 + h), d1 = px(y0 + 1 - h);
  for (int y = y0; y < y1; y += 2) {
    const bool two = y + 1 < y1;
    const Px ca0 = a0, cd0 = d0, ca1 = a1, cd1 = d1;
    if (y + 2 < y1) {
      a0 = px(y + 2 + h);
      d0 = px(y + 2 - h);
    }
    if (y + 3 < y1) {
      a1 = px(y + 3 + h);
      d1 = px(y + 3 - h);
    }
    int p0[NA], p1[NA];
    stage(0, y, ca0, cd0, p0);
    if (two) stage(1, y + 1, ca1, cd1, p1);
    __syncthreads();
    finish(0, p0);
    if (two) finish(1, p1);
    __syncthreads();
    emit(0, y);
    if (two) emit(1, y + 1);
  }
}

// ---------------------------------------------------------------- host launchers
hipError_t launch_prep(const PrepPair &one, const PrepPair *many, int npairs, int maxH,
                       int maxCols, int maxW, int prec, hipStream_t s, hipStream_t s_stats) {
  // one block per row (4 columns a thread) up to 4096 columns: a second,
  // mostly idle block per row costs more than the wider block
  const int nt = std::min(1024, (ceil_div(maxCols, 4) + WV - 1) / WV * WV);
  const dim3 grid(ceil_div(maxCols, 4 * nt), maxH, npairs);
#define PP(pr)                                                                                \
  do {                                                                                        \
    if (many) hipLaunchKernelGGL((prep_planes_kernel<pr, true>), grid, dim3(nt), 0, s, one, many); \
    else hipLaunchKernelGGL((prep_planes_kernel<pr, false>), grid, dim3(nt), 0, s, one, many);     \
  } while (0)
  if (prec == P_I16) PP(P_I16); else if (prec == P_F16) PP(P_F16); else PP(P_BF16);
#undef PP
  // the window shape is shared by every pair of a batch (one parameter set);
  // both images in one pass
  int sy;
  const dim3 gs = ws_grid(maxW, maxH, npairs, sy);
  hipStream_t ss = s_stats ? s_stats : s;
#define WS(b, ch) hipLaunchKernelGGL((window_stats_kernel<b, ch, 2>), gs, dim3(WS_T), 0, ss, one, many, 0, sy)
  if (many) {
    if (one.chess) WS(true, true); else WS(true, false);
  } else {
    if (one.chess) WS(false, true); else WS(false, false);
  }
#undef WS
  return hipGetLastError();
}

hipError_t launch_window_stats_dense(const uint8_t *img, int H, int W, int pitch, int win,
                                     int chess, int32_t *S, int32_t *SS, float *inv, hipStream_t s) {
  PrepPair P = {};
  P.L = img;
  P.H = H;
  P.W = W;
  P.pitch = pitch;
  P.win = win;
  P.chess = chess;
  P.SL = S;
  P.SSL = SS;
  P.invLd = inv;
  int sy;
  const dim3 gs = ws_grid(W, H, 1, sy);
  if (chess)
    hipLaunchKernelGGL((window_stats_kernel<false, true, 1>), gs, dim3(WS_T), 0, s, P, (const PrepPair *)nullptr, 2, sy);
  else
    hipLaunchKernelGGL((window_stats_kernel<false, false, 1>), gs, dim3(WS_T), 0, s, P, (const PrepPair *)nullptr, 2, sy);
  return hipGetLastError();
}

}  // namespace st
