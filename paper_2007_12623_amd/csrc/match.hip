// Dense ZNCC matching with winner-take-all in the left and right reference
// (Section II-A of the paper: every pixel tests every candidate disparity over
// a square window).  The paper's kernel gives one thread per pixel and
// caches image rows in shared memory; this one is laid out for gfx950:
//
//  * a wave owns a span of 64*8 columns, one chunk of 8 disparities and a
//    band of rows; lane l owns columns x0 .. x0+7 (x0 = xs + 8 l);
//  * vertical window sums V(c, d) = sum_v n(L-128)(c, y+v) * R(c-d, y+v) are
//    running sums in registers: one v_dot2_i32_i16 adds the entering row and
//    removes the leaving one;
//  * horizontal window sums come from prefix sums over the lane's 8 columns;
//    the h columns on either side arrive as one partial sum from each
//    neighbouring lane through the LDS crossbar (lanes 0 and 63 are halos);
//  * the ZNCC numerator n*S_LR - S_L*S_R is exact in int32 (24-bit mads);
//    normalisation by the FP64-computed 1/sqrt(varN) happens in fp32;
//  * the winner-take-all key is z + 2 in fp32 with the disparity index in the
//    4 low mantissa bits, so one v_max3 updates a running argmax with two
//    candidates; invalid candidates carry NaN, which v_max ignores;
//  * right-reference maxima accumulate along the diagonals x - d and are
//    merged across neighbouring lanes;
//  * a workgroup of 4 waves owns one (band, span) and a group of disparity
//    chunks; its waves merge their keys (quantised z, then 255 - (d - dmin))
//    with LDS atomic max into key tiles of the band, which go to global
//    memory once per band: plain stores for the left keys when the group
//    holds every chunk, one atomic max per right column otherwise.
#include <algorithm>
#include <type_traits>

#include "common.h"

namespace st {

// ---------------------------------------------------------------- helpers
// Neighbour-lane terms through DPP wave shifts, an operand modifier of the
// add (or max) that consumes the value: no LDS round trip and no wait.
// add_left(a, v) = a + v of lane i-1 (wave_shr:1), add_right(a, v) = a + v
// of lane i+1 (wave_shl:1).  Lane 0 (left) and lane 63 (right) read 0;
// both are halo lanes whose outputs are unused.  The instructions are
// written out (the compiler folds only some of its DPP moves into the adds,
// and keeps the rest as separate moves); a DPP read of a VGPR needs two
// wait states after the VALU write of it, hence the s_nop 1 in front.
__device__ __forceinline__ int add_left(int a, int v) {
  int r;
  asm("s_nop 1\n\tv_add_u32_dpp %0, %1, %2 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
      : "=v"(r) : "v"(v), "v"(a));
  return r;
}
__device__ __forceinline__ int add_right(int a, int v) {
  int r;
  asm("s_nop 1\n\tv_add_u32_dpp %0, %1, %2 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
      : "=v"(r) : "v"(v), "v"(a));
  return r;
}
__device__ __forceinline__ float add_left(float a, float v) {
  float r;
  asm("s_nop 1\n\tv_add_f32_dpp %0, %1, %2 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
      : "=v"(r) : "v"(v), "v"(a));
  return r;
}
__device__ __forceinline__ float add_right(float a, float v) {
  float r;
  asm("s_nop 1\n\tv_add_f32_dpp %0, %1, %2 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
      : "=v"(r) : "v"(v), "v"(a));
  return r;
}
// max(a, v of lane i+1), ignoring quiet NaNs like kmax below.  Lane 63 has
// no right neighbour and keeps a: without bound_ctrl the shift leaves that
// lane unwritten, and the result is a's own register.  (A zero read there
// would be the key of z + 3 = 0, a valid key, for columns no lane covers.)
__device__ __forceinline__ float max_right(float a, float v) {
  asm("s_nop 1\n\tv_max_f32_dpp %0, %1, %0 wave_shl:1 row_mask:0xf bank_mask:0xf"
      : "+v"(a) : "v"(v));
  return a;
}
// Maxima of keys that ignore quiet-NaN operands (the keys of invalid
// candidates), as single v_max_f32 / v_max3_f32 instructions: written as
// builtins the compiler first canonicalises every operand that comes out of
// integer bit operations (one more v_max_f32 per key).  The keys are normal
// floats or quiet NaNs, for which the instruction returns an operand's bits
// unchanged.
__device__ __forceinline__ float kmax(float a, float b) {
  float r;
  asm("v_max_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ float kmax3(float a, float b, float c) {
  float r;
  asm("v_max3_f32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}
__device__ __forceinline__ int s24(int v) { return __builtin_amdgcn_sbfe(v, 0, 24); }

typedef short short2v __attribute__((ext_vector_type(2)));
typedef _Float16 half2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));

// byte selectors for v_perm_b32(S0 = hi source, S1 = lo source)
// 16-bit halves: lo16 <- S1 half h, hi16 <- S0 half h
__device__ __forceinline__ constexpr uint32_t sel16(int h) { return h ? 0x07060302u : 0x05040100u; }
// 8-bit lanes zero-extended: lo16 <- S1 byte b, hi16 <- S0 byte b
__device__ __forceinline__ constexpr uint32_t sel8(int b) {
  return (uint32_t)b | 0x0C00u | ((uint32_t)(4 + b) << 16) | 0x0C000000u;
}

template <int PREC> struct Img;
template <> struct Img<P_I16> {
  using Acc = int;
  static constexpr int RB = 1;  // bytes per R element
  __device__ static Acc dot(uint32_t l, uint32_t r, Acc c) {
    return __builtin_amdgcn_sdot2(__builtin_bit_cast(short2v, l), __builtin_bit_cast(short2v, r), c, false);
  }
};
template <> struct Img<P_F16> {
  using Acc = float;
  static constexpr int RB = 2;
  __device__ static Acc dot(uint32_t l, uint32_t r, Acc c) {
    return __builtin_amdgcn_fdot2(__builtin_bit_cast(half2v, l), __builtin_bit_cast(half2v, r), c, false);
  }
};
template <> struct Img<P_BF16> {
  using Acc = float;
  static constexpr int RB = 2;
  __device__ static Acc dot(uint32_t l, uint32_t r, Acc c) {
    return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2v, l), __builtin_bit_cast(bf16x2v, r), c, false);
  }
};

// Lane keys are the bits of z + 3 (in [2, 4] up to rounding: non-negative
// floats compare like unsigned integers, and one binade keeps the
// quantisation uniform) with the low nibble replaced by 15 - j, j the
// disparity's index in its chunk.  The global key of a lane key b with
// nibble m is 0x80000000 | q << 8 | 255 - (d - dmin), q the bits of z + 3
// above the nibble, so that ties prefer the smaller disparity.  With
// c = 0x80001000 + 240 - (d0 - dmin) it is ((b & ~15) << 4) + c + m,
// computed as ((b << 4) + c) - 15 m: for b in [2, 4] the 32-bit shift gives
// a signed value in [-4096, 0x08001000], so the key has bit 31 set and
// keeps the order of z.  A lane without a valid candidate keeps the start
// value KEY_START, a negative float (below every z + 3 and ignored by none
// of the maxima) whose shifted bits are 0x80000000: its key, 0x1000 +
// 240 - (d0 - dmin), has bit 31 clear.  So bit 31 marks a valid key, and a
// key without it never wins a merge.
constexpr float KEY_OFFSET = 3.0f;
constexpr uint32_t KEY_START = 0xB8000000u;
__device__ __forceinline__ uint32_t key_base(int dd0) { return 0x80001000u + 240u - (uint32_t)dd0; }
__device__ __forceinline__ uint32_t global_key(float k, uint32_t c) {
  const uint32_t b = __builtin_bit_cast(uint32_t, k);
  // three instructions; left to itself the compiler takes four (a separate
  // shift, the product -15 m, then a three-way add)
  uint32_t t, key;
  asm("v_lshl_add_u32 %0, %1, 4, %2" : "=v"(t) : "v"(b), "v"(c));
  asm("v_mad_i32_i24 %0, %1, -15, %2" : "=v"(key) : "v"(b & 15u), "v"(t));
  return key;
}
__device__ __forceinline__ bool key_valid(uint32_t v) { return (int)v < 0; }

__device__ __forceinline__ void gmax(GLOBAL uint32_t *p, uint32_t v) {
  __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void lmax(LDS uint32_t *p, uint32_t v) {
  __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Key tiles of one workgroup task in LDS.
//   left:  key of lane l, column c of row r at lt[r*8*LTP + c*LTP + l]
//   right: tile column q (image column rbase + q) of row r at
//          rt[r*8*rp + (q & 7)*rp + (q >> 3)]
// LTP and rp are 4 (mod 8): a wave's atomics (lanes at consecutive slots)
// and the write-out (threads at consecutive columns) are both free of bank
// conflicts.
constexpr int LTP = 68;
struct KeyTile {
  LDS uint32_t *lt;
  LDS uint32_t *rt;
  int rp, y0, rbase;
};

// Load N dwords at byte offset `off` (a multiple of 4) of a wave-uniform
// base: the base stays in scalar registers and each lane keeps a 32-bit
// offset.
template <int N>
__device__ __forceinline__ void load_dw(uint32_t (&dst)[N], const GLOBAL char *base, uint32_t off) {
  const GLOBAL uint32_t *q = (const GLOBAL uint32_t *)(base + off);
#pragma unroll
  for (int i = 0; i < N; ++i) dst[i] = q[i];
}

// Load N dwords starting `sh` bytes (0..3, uniform) after byte offset `off`
// (a multiple of 4): one extra dword, then v_alignbyte per dword.
template <int N, bool SH>
__device__ __forceinline__ void load_dw_shifted(uint32_t (&dst)[N], const GLOBAL char *base,
                                                uint32_t off, int sh) {
  if constexpr (!SH) {
    load_dw(dst, base, off);
    return;
  }
  const GLOBAL uint32_t *q = (const GLOBAL uint32_t *)(base + off);
  uint32_t t[N + 1];
#pragma unroll
  for (int i = 0; i <= N; ++i) t[i] = q[i];
#pragma unroll
  for (int i = 0; i < N; ++i) dst[i] = __builtin_amdgcn_alignbyte(t[i + 1], t[i], sh);
}

// ---------------------------------------------------------------- one task
// Rows [y0, y1) of the span starting at column xs, disparities d0 .. d0+DC-1;
// keys go to the workgroup's tiles.  With the chessboard window the pass
// takes colour `par`: its L planes hold only the pixels with (x + y) & 1 ==
// par, so the window sums of a pixel of that colour run over exactly its
// chessboard cells, and the pixels of the other colour produce no keys.
template <int WIN, int DC, int PREC, bool SH>
__device__ __forceinline__ void match_rows(const MatchPair &P, int y0, int y1, int xs, int d0,
                                           int par, int lane, const KeyTile &kt) {
  constexpr int H = WIN / 2;
  constexpr int K = KC;
  constexpr int T = K + DC - 1;                 // R columns touched by a lane
  using IM = Img<PREC>;
  using Acc = typename IM::Acc;
  constexpr int RB = IM::RB;
  constexpr int NLD = K / 2;                    // dwords of one L row segment (int16/fp16)
  constexpr int NRD = (T * RB + 3) / 4;         // dwords of one R row segment
  const int n = P.nwin;

  const int x0 = xs + lane * K;
  const int colL = x0 + P.padL;                 // multiple of 8
  const int colR = x0 - d0 - (DC - 1) + P.padR;
  // byte misalignment of the right segments (wave-uniform; 0 unless SH, the
  // shifted last chunk of some ranges)
  const int rsh = SH ? (RB * colR) & 3 : 0;
  const bool halo = (lane == 0) || (lane == WV - 1);
  // planes are under 4 GiB: byte offsets of the lane's segments fit 32 bits
  const GLOBAL char *Lg = (const GLOBAL char *)P.Lp + par * P.lplane;
  const GLOBAL char *NLg = (const GLOBAL char *)P.NLp + par * P.lplane;
  const GLOBAL char *Rg = (const GLOBAL char *)P.Rp;
  const uint32_t Lo = 2u * (uint32_t)colL, Ro = (uint32_t)(RB * colR - rsh);
  const uint32_t sL = 2u * (uint32_t)P.strideL, sR = (uint32_t)(RB * P.strideR);

  Acc V[DC][K];
#pragma unroll
  for (int j = 0; j < DC; ++j)
#pragma unroll
    for (int c = 0; c < K; ++c) V[j][c] = 0;

  // ---- vertical sums of the first row: rows y0-H .. y0+H, two at a time
  for (int r = y0 - H; r <= y0 + H; r += 2) {
    const bool two = r + 1 <= y0 + H;
    uint32_t la[NLD], lb[NLD], ra[NRD], rb[NRD];
    load_dw(la, Lg, Lo + sL * r);
    load_dw_shifted<NRD, SH>(ra, Rg, Ro + sR * r, rsh);
    if (two) {
      load_dw(lb, Lg, Lo + sL * (r + 1));
      load_dw_shifted<NRD, SH>(rb, Rg, Ro + sR * (r + 1), rsh);
    } else {
#pragma unroll
      for (int i = 0; i < NLD; ++i) lb[i] = 0;
#pragma unroll
      for (int i = 0; i < NRD; ++i) rb[i] = 0;
    }
    uint32_t lp[K], rp[T];
#pragma unroll
    for (int c = 0; c < K; ++c) lp[c] = __builtin_amdgcn_perm(lb[c / 2], la[c / 2], sel16(c & 1));
#pragma unroll
    for (int t = 0; t < T; ++t) {
      if constexpr (RB == 1) rp[t] = __builtin_amdgcn_perm(rb[t / 4], ra[t / 4], sel8(t & 3));
      else rp[t] = __builtin_amdgcn_perm(rb[t / 2], ra[t / 2], sel16(t & 1));
    }
#pragma unroll
    for (int j = 0; j < DC; ++j)
#pragma unroll
      for (int c = 0; c < K; ++c) V[j][c] = IM::dot(lp[c], rp[c - j + DC - 1], V[j][c]);
  }

  const uint32_t kc = key_base(d0 - P.dmin);
  for (int y = y0; y < y1; ++y) {
    if (y > y0) {
      // entering row y+H (+), leaving row y-H-1 (-)
      const int ra_ = y + H, rl_ = y - H - 1;
      uint32_t la[NLD], lo[NLD], ra[NRD], ro[NRD];
      load_dw(la, Lg, Lo + sL * ra_);
      load_dw(lo, NLg, Lo + sL * rl_);
      load_dw_shifted<NRD, SH>(ra, Rg, Ro + sR * ra_, rsh);
      load_dw_shifted<NRD, SH>(ro, Rg, Ro + sR * rl_, rsh);
      uint32_t lp[K], rp[T];
#pragma unroll
      for (int c = 0; c < K; ++c) lp[c] = __builtin_amdgcn_perm(lo[c / 2], la[c / 2], sel16(c & 1));
#pragma unroll
      for (int t = 0; t < T; ++t) {
        if constexpr (RB == 1) rp[t] = __builtin_amdgcn_perm(ro[t / 4], ra[t / 4], sel8(t & 3));
        else rp[t] = __builtin_amdgcn_perm(ro[t / 2], ra[t / 2], sel16(t & 1));
      }
#pragma unroll
      for (int j = 0; j < DC; ++j)
#pragma unroll
        for (int c = 0; c < K; ++c) V[j][c] = IM::dot(lp[c], rp[c - j + DC - 1], V[j][c]);
    }

    // ---- per-row statistics: left pixels of the lane, right columns of the segment
    int nsl[K];
    float il[K];
    {
      // 32-byte aligned: colL is a multiple of 8, strideL of 16
      const uint32_t o = 4u * (uint32_t)(y * P.strideL + colL);
      const GLOBAL uint32_t *ns = (const GLOBAL uint32_t *)((const GLOBAL char *)P.negSL + o);
      const GLOBAL uint32_t *iv = (const GLOBAL uint32_t *)((const GLOBAL char *)P.invL + o);
      uint32_t nsw[K], ivw[K];
      load_dw(nsw, (const GLOBAL char *)ns, 0);
      load_dw(ivw, (const GLOBAL char *)iv, 0);
      // chessboard: column x0 + c has colour par when c & 1 == cpar (x0 has
      // the parity of xs, so cpar is wave-uniform)
      const int cpar = (xs + y + par) & 1;
      // bit c set: column c is of the other colour (uniform)
      const int cm = P.chess ? (cpar ? 0x55 : 0xAA) : 0;
#pragma unroll
      for (int c = 0; c < K; ++c) {
        nsl[c] = (int)nsw[c];
        const bool off = halo | (((cm >> c) & 1) != 0);
        il[c] = off ? __builtin_nanf("") : __builtin_bit_cast(float, ivw[c]);
      }
    }
    int sr[T];
    float ir[T];
    {
      const uint32_t o = 4u * (uint32_t)(y * P.strideR + colR);
      const GLOBAL int32_t *srp = (const GLOBAL int32_t *)((const GLOBAL char *)P.SR + o);
      const GLOBAL float *irp = (const GLOBAL float *)((const GLOBAL char *)P.invR + o);
#pragma unroll
      for (int t = 0; t < T; ++t) {
        sr[t] = srp[t];
        ir[t] = irp[t];
      }
    }

    float bestL[K];
    float Pd[T];
#pragma unroll
    for (int c = 0; c < K; ++c) bestL[c] = __builtin_bit_cast(float, KEY_START);
#pragma unroll
    for (int t = 0; t < T; ++t) Pd[t] = __builtin_bit_cast(float, KEY_START);

    // ---- per chunk disparity j: horizontal window sums of the lane's
    //      columns (own columns through prefix sums; the h columns beyond each
    //      side as one partial sum from the neighbouring lane: suffix sums of
    //      the left lane, prefix sums of the right lane), then the keys.
    //      Evaluation (i, j) uses right column t = i - j + DC - 1.  The
    //      disparities go in pairs (j, j + 1): key (i, j) and key (i, j + 1)
    //      meet in the left maximum of pixel i, keys (i, j) and (i + 1, j + 1)
    //      on diagonal t, so every merge takes two keys (v_max3).
    const int nn = s24(n);
#pragma unroll
    for (int j0 = 0; j0 < DC; j0 += 2) {
      float kp[2][K];
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) {
        const int j = j0 + jj;
        Acc Pf[K + 1];
        Pf[0] = 0;
#pragma unroll
        for (int c = 0; c < K; ++c) Pf[c + 1] = c == 0 ? V[j][0] : Pf[c] + V[j][c];
        Acc Sf[H + 1];
        Sf[0] = 0;
#pragma unroll
        for (int k = 1; k <= H; ++k) Sf[k] = k == 1 ? V[j][K - 1] : Sf[k - 1] + V[j][K - k];
#pragma unroll
        for (int i = 0; i < K; ++i) {
          const int lo = i - H, hi = i + H + 1;   // own columns [max(lo,0), min(hi,K))
          Acc Sij = (lo > 0) ? Pf[hi < K ? hi : K] - Pf[lo] : Pf[hi < K ? hi : K];
          if (lo < 0) Sij = add_left(Sij, Sf[-lo]);    // suffix sums of the left lane
          if (hi > K) Sij = add_right(Sij, Pf[hi - K]);  // prefix sums of the right lane
          const int t = i - j + DC - 1;
          int num;
          if constexpr (PREC == P_I16) {
            num = s24(nsl[i]) * s24(sr[t]) + Sij;
          } else {
            // Sij is an exact integer below 2^23 in fp32
            num = s24((int)Sij) * nn + s24(nsl[i]) * s24(sr[t]);
          }
          const float zl = (float)num * ir[t];
          float zq;
          if constexpr (PREC == P_I16) {
            zq = __builtin_fmaf(zl, il[i], KEY_OFFSET);
          } else if constexpr (PREC == P_F16) {
            // the cost slice: z rounded to fp16 (v_fma_mixlo_f16), widened
            // and offset in one v_fma_mix_f32
            const _Float16 zh = (_Float16)(zl * il[i]);
            asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel_hi:[1,0,0]" : "=v"(zq) : "v"(zh), "v"(KEY_OFFSET));
          } else {
            // the cost slice: z rounded to bf16 (to nearest even) into the
            // high half of a dword whose low half is 0, which is then that
            // value as an fp32 (one v_cvt_pk_bf16_f32)
            float zb;
            asm("v_cvt_pk_bf16_f32 %0, 0, %1" : "=v"(zb) : "v"(zl * il[i]));
            zq = zb + KEY_OFFSET;
          }
          kp[jj][i] = __builtin_bit_cast(
              float, (__builtin_bit_cast(uint32_t, zq) & ~15u) | (uint32_t)(15 - j));
        }
      }
#pragma unroll
      for (int i = 0; i < K; ++i) bestL[i] = kmax3(bestL[i], kp[0][i], kp[1][i]);
      // diagonal t = i - j0 + DC - 1 holds (i, j0) and (i + 1, j0 + 1)
#pragma unroll
      for (int i = 0; i < K - 1; ++i) {
        const int t = i - j0 + DC - 1;
        Pd[t] = kmax3(Pd[t], kp[0][i], kp[1][i + 1]);
      }
      Pd[K - 1 - j0 + DC - 1] = kmax(Pd[K - 1 - j0 + DC - 1], kp[0][K - 1]);
      Pd[DC - 2 - j0] = kmax(Pd[DC - 2 - j0], kp[1][0]);
    }

    // ---- right reference: fold diagonals of higher lanes into this lane's
    //      home diagonals t in [DC-1, T).  Increasing t order chains the
    //      contributions of several lanes in one pass.
#pragma unroll
    for (int t = 0; t < DC - 1; ++t) Pd[t + K] = max_right(Pd[t + K], Pd[t]);

    // ---- emit into the tiles: left reference per pixel, right reference
    //      per home column.  Branch-free: a lane without a valid candidate
    //      merges a key below 0x80000000.  The halo lanes' keys are all of
    //      that kind, their normalisers being NaN; so are lane 0's diagonals
    //      left of its home, the columns that the previous span covers.
    LDS uint32_t *lrow = kt.lt + (y - kt.y0) * (8 * LTP) + lane;
#pragma unroll
    for (int c = 0; c < K; ++c) lmax(lrow + c * LTP, global_key(bestL[c], kc));
    LDS uint32_t *rrow = kt.rt + (y - kt.y0) * (8 * kt.rp);
    const int q0 = x0 - d0 - kt.rbase;  // tile column of home diagonal 0; q0 & 7 is wave-uniform
#pragma unroll
    for (int m = 0; m < K; ++m) {
      const int q = q0 + m;
      lmax(rrow + (q & 7) * kt.rp + (q >> 3), global_key(Pd[m + DC - 1], kc));
    }
  }
}

// ---------------------------------------------------------------- workgroup task
// Band `g` (band * nspan + span) of a pair, chunk group `cg`: the chunks
// cg*CG .. min((cg+1)*CG, nchunk)-1, rows rlo .. rhi-1 of the band (all of
// it, or one half of it for the tasks that end a queue).  The 4 waves take
// (chunk, sub-band) items in turn; with fewer chunks than waves the rows
// are cut into sub-bands so that every wave has work.
template <int WIN, int DC, int PREC>
__device__ __forceinline__ void wg_task(const MatchPair &P, int g, int cg, int rlo, int rhi,
                                        LDS uint32_t *lds) {
  // the wave index is uniform: in a scalar register every quantity derived
  // from it (chunk, colour, rows of the item) stays scalar as well
  const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & (WV - 1);
  constexpr int NT = NWAVE * WV;
  const int h = WIN / 2;
  const int band = g / P.nspan, span = g - band * P.nspan;
  const int y0 = h + band * P.TY + rlo;
  const int y1 = min(h + band * P.TY + rhi, P.H - h);
  if (y0 >= y1) {
    // uniform over the workgroup (no half band past the image is queued):
    // still one barrier, which the persistent loop's reuse of its task
    // index relies on
    __syncthreads();
    return;
  }
  const int rows = y1 - y0;
  const int xs = P.xs0 + span * (OUT_LANES * KC);
  const int D = P.dmax - P.dmin + 1;
  const int cf = cg * P.CG, cl = min(cf + P.CG, P.nchunk) - 1, nc = cl - cf + 1;
  const int d0f = P.dmin + min(cf * DC, D - DC), d0l = P.dmin + min(cl * DC, D - DC);
  KeyTile kt;
  kt.lt = lds;
  kt.rt = lds + P.TY * 8 * LTP;
  kt.rp = P.rp;
  kt.y0 = y0;
  kt.rbase = xs - d0l - (DC - 1);
  const int RW = WV * KC + (DC - 1) + (d0l - d0f);  // right tile columns in use

  for (int i = tid; i < rows * 8 * LTP; i += NT) kt.lt[i] = 0u;
  for (int i = tid; i < rows * 8 * kt.rp; i += NT) kt.rt[i] = 0u;
  __syncthreads();

  // units: (chunk, colour) pairs, one colour unless the window is a
  // chessboard.  Items: the units in whole rounds of NWAVE over the band's
  // rows, then those of an incomplete last round (one or two) cut into
  // sub-bands, NWAVE / rem each, so that every wave has work there too
  // (three keep whole rows: a quarter band costs its own restart)
  const int units = nc * (P.chess ? 2 : 1);
  const int full = units / NWAVE * NWAVE, rem = units - full;
  const int SB = rem == 0 ? 1 : NWAVE / rem;
  const int TYs = ceil_div(rows, SB);
  const int items = full + rem * SB;
  for (int it = wave; it < items; it += NWAVE) {
    const int r = it - full;
    const int u = r < 0 ? it : full + r % rem, sb = r < 0 ? 0 : r / rem;
    const int c = cf + u % nc, par = u / nc;
    const int ya = r < 0 ? y0 : y0 + sb * TYs, yb = r < 0 ? y1 : min(ya + TYs, y1);
    if (ya < yb) {
      const int d0 = P.dmin + min(c * DC, D - DC);
      // right segments start on a dword unless the chunk was shifted
      if (((Img<PREC>::RB * (xs - d0 - (DC - 1) + P.padR)) & 3) != 0)
        match_rows<WIN, DC, PREC, true>(P, ya, yb, xs, d0, par, lane, kt);
      else
        match_rows<WIN, DC, PREC, false>(P, ya, yb, xs, d0, par, lane, kt);
    }
  }
  __syncthreads();

  // write-out: output columns xs+8 .. xs+503 of the left tile; every used
  // column of the right tile
  const bool whole = P.ncg == 1;
  GLOBAL uint32_t *kl = (GLOBAL uint32_t *)P.keyL;
  GLOBAL uint32_t *kr = (GLOBAL uint32_t *)P.keyR;
  for (int r = 0; r < rows; ++r) {
    const size_t rowoff = (size_t)(y0 + r) * P.W;
    for (int xr = KC + tid; xr < (OUT_LANES + 1) * KC; xr += NT) {
      const int x = xs + xr;
      if (x < 0 || x >= P.W) continue;
      const uint32_t v = kt.lt[r * 8 * LTP + (xr & 7) * LTP + (xr >> 3)];
      if (whole) kl[rowoff + x] = v;
      else if (key_valid(v)) gmax(kl + rowoff + x, v);
    }
    for (int q = tid; q < RW; q += NT) {
      const uint32_t v = kt.rt[r * 8 * kt.rp + (q & 7) * kt.rp + (q >> 3)];
      const int x = kt.rbase + q;
      if (key_valid(v) && x >= 0 && x < P.W) gmax(kr + rowoff + x, v);
    }
  }
}

// One workgroup per task.  Blocks b with equal b % 8 run on one XCD; each
// XCD gets whole (band, span) groups so that their chunk groups share its L2.
template <int WIN, int DC, int PREC>
__global__ __launch_bounds__(NWAVE * WV) __attribute__((amdgpu_waves_per_eu(3)))
void match_kernel(MatchPair P, int ngroups) {
  extern __shared__ uint32_t lds_dyn[];
  const int b = blockIdx.x;
  const int xcd = b & 7;
  const int r = b >> 3;
  const int cg = r % P.ncg;
  const int g = (r / P.ncg) * 8 + xcd;
  if (g >= ngroups) return;
  wg_task<WIN, DC, PREC>(P, g, cg, 0, P.TY, (LDS uint32_t *)lds_dyn);
}

// Persistent form: workgroups pull tasks (pair, group, chunk group, rows) of
// one window size from a queue until it is empty.  Every workgroup reaches the
// exit once the counter passes ntasks.
template <int WIN, int DC, int PREC>
__global__ __launch_bounds__(NWAVE * WV) __attribute__((amdgpu_waves_per_eu(3)))
void match_persistent_kernel(const MatchPair *__restrict__ pairs, const int4 *__restrict__ tasks,
                             int ntasks, int *__restrict__ counter) {
  extern __shared__ uint32_t lds_dyn[];
  __shared__ int next;
  for (;;) {
    // the previous task's barriers keep this store behind every read of `next`
    if (threadIdx.x == 0) next = atomicAdd(counter, 1);
    __syncthreads();
    const int t = __builtin_amdgcn_readfirstlane(next);
    if (t >= ntasks) break;
    const int4 tk = tasks[t];
    const MatchPair P = pairs[tk.x];
    // tk.w: 0 for the whole band, else rows (w & 0xFFFF) .. (w >> 16) - 1
    const int rlo = tk.w ? (tk.w & 0xFFFF) : 0, rhi = tk.w ? (tk.w >> 16) : P.TY;
    wg_task<WIN, DC, PREC>(P, tk.y, tk.z, rlo, rhi, (LDS uint32_t *)lds_dyn);
  }
}

__global__ void reset_counter_kernel(int *counter) { *counter = 0; }

// ---------------------------------------------------------------- host launchers
size_t match_lds_bytes(const MatchPair &P) { return 4 * (size_t)P.TY * 8 * (LTP + P.rp); }

template <class F>
static hipError_t allow_lds(F *kern, size_t bytes) {
  return hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int WIN, int DC, int PREC>
static hipError_t launch_match_t(const MatchPair &P, hipStream_t s) {
  const int ngroups = P.nband * P.nspan;
  const int blocks = 8 * ceil_div(ngroups, 8) * P.ncg;
  const size_t lds = match_lds_bytes(P);
  hipError_t e = allow_lds(match_kernel<WIN, DC, PREC>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((match_kernel<WIN, DC, PREC>), dim3(blocks), dim3(NWAVE * WV), lds, s, P, ngroups);
  return hipGetLastError();
}

// Calls f(window, disparities per thread, precision) with the three as
// compile-time constants: windows 3..15 (odd), chunks of 4 or 8
// disparities, the three image precisions.
template <class F>
static auto with_config(int win, int dc, int prec, F &&f) {
  auto by_prec = [&](auto W, auto D) {
    if (prec == P_I16) return f(W, D, std::integral_constant<int, P_I16>{});
    if (prec == P_F16) return f(W, D, std::integral_constant<int, P_F16>{});
    return f(W, D, std::integral_constant<int, P_BF16>{});
  };
  auto by_dc = [&](auto W) {
    if (dc == 4) return by_prec(W, std::integral_constant<int, 4>{});
    return by_prec(W, std::integral_constant<int, 8>{});
  };
  switch (win) {
    case 3: return by_dc(std::integral_constant<int, 3>{});
    case 5: return by_dc(std::integral_constant<int, 5>{});
    case 7: return by_dc(std::integral_constant<int, 7>{});
    case 9: return by_dc(std::integral_constant<int, 9>{});
    case 11: return by_dc(std::integral_constant<int, 11>{});
    case 13: return by_dc(std::integral_constant<int, 13>{});
    default: return by_dc(std::integral_constant<int, 15>{});
  }
}

static bool config_ok(int win, int dc) { return win >= 3 && win <= 15 && (win & 1) && (dc == 4 || dc == 8); }

hipError_t launch_match(const MatchPair &P, int prec, hipStream_t s) {
  if (!config_ok(P.win, P.DC)) return hipErrorInvalidValue;
  return with_config(P.win, P.DC, prec, [&](auto W, auto D, auto Pr) {
    return launch_match_t<decltype(W)::value, decltype(D)::value, decltype(Pr)::value>(P, s);
  });
}

// One persistent launch over the tasks of one window size.
hipError_t launch_match_persistent(const MatchPair *pairs_dev, const int4 *tasks_dev, int ntasks,
                                   int *counter_dev, int win, int dc, int prec, int nblocks,
                                   size_t lds, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  if (!config_ok(win, dc)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, s, counter_dev);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (ev0) (void)hipEventRecord(ev0, s);
  e = with_config(win, dc, prec, [&](auto W, auto D, auto Pr) {
    auto *k = match_persistent_kernel<decltype(W)::value, decltype(D)::value, decltype(Pr)::value>;
    hipError_t x = allow_lds(k, lds);
    if (x != hipSuccess) return x;
    hipLaunchKernelGGL(k, dim3(nblocks), dim3(NWAVE * WV), lds, s, pairs_dev, tasks_dev, ntasks,
                       counter_dev);
    return hipGetLastError();
  });
  if (ev1) (void)hipEventRecord(ev1, s);
  return e;
}

int match_persistent_occupancy(int win, int dc, int prec, size_t lds) {
  if (!config_ok(win, dc)) return 1;
  return with_config(win, dc, prec, [&](auto W, auto D, auto Pr) {
    auto *k = match_persistent_kernel<decltype(W)::value, decltype(D)::value, decltype(Pr)::value>;
    int n = 0;
    if (allow_lds(k, lds) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, NWAVE * WV, lds) != hipSuccess) {
      (void)hipGetLastError();
      return 1;
    }
    return std::max(1, n);
  });
}

}  // namespace st
