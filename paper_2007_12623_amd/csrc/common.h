// Shared device/host definitions of the MI355X ZNCC stereo library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace st {

// Explicit address spaces for device code: loads through generic pointers
// become flat instructions, which count on the LDS wait counter as well and
// may alias LDS, so the compiler can neither overlap them with LDS traffic
// nor move them past LDS stores.
#define GLOBAL __attribute__((address_space(1)))
#define LDS __attribute__((address_space(3)))
template <class T>
__device__ __forceinline__ const GLOBAL T *gro(const T *p) { return (const GLOBAL T *)p; }
template <class T>
__device__ __forceinline__ GLOBAL T *grw(T *p) { return (GLOBAL T *)p; }

constexpr int WV = 64;        // wavefront size on gfx950
constexpr int KC = 8;         // image columns owned by one lane of the matcher
constexpr int OUT_LANES = 62; // lanes 1..62 of a wave produce output; 0 and 63 are halos
constexpr int NWAVE = 4;      // waves of a matcher workgroup

// Inclusive prefix sum over the 64 lanes of a wave through DPP moves, with
// no LDS round trip: Hillis-Steele over each row of 16 lanes with row shifts
// of 1, 2, 4 and 8 (lanes shifted in from outside the row read 0), then the
// total of row 0 added to row 1 and of row 2 to row 3 (row_bcast:15), and
// the total of rows 0-1 to rows 2 and 3 (row_bcast:31).  Lanes a step does
// not write keep 0, so the step adds 0 there.
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_take(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xF, true);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_take(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)dpp_take<CTRL, ROWS>((int)(unsigned)b);
  const unsigned hi = (unsigned)dpp_take<CTRL, ROWS>((int)(unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <class T>
__device__ __forceinline__ T wave_scan_incl(T v) {
  v += dpp_take<0x111, 0xF>(v);  // row_shr:1
  v += dpp_take<0x112, 0xF>(v);  // row_shr:2
  v += dpp_take<0x114, 0xF>(v);  // row_shr:4
  v += dpp_take<0x118, 0xF>(v);  // row_shr:8
  v += dpp_take<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_take<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
  return v;
}

enum Prec { P_I16 = 0, P_F16 = 1, P_BF16 = 2 };

// Disparity stored at pixels without a valid one in the integer disparity
// maps of the post-processing (decode, left-right check, outlier removal,
// fills): the radial scans then tell validity from the disparity alone and
// read one 2-byte value per step.  Disparities lie within +-4096.
constexpr int16_t O_NONE = -32768;

// Geometry and device pointers of one prepared pair, as the matcher sees it.
// Planes are padded row-major arrays: image column x lives at index x + pad.
// With the chessboard window the L planes come twice, lplane bytes apart:
// copy c keeps the pixels with (x + y) & 1 == c and holds 0 elsewhere.
//   L planes / L stats: stride strideL, pad padL  (padL chosen so that the
//                       first column of every lane is 16-byte aligned)
//   R plane  / R stats: stride strideR, pad padR  (multiple of 4)
struct MatchPair {
  const void *Lp;      // int16 n*(L-128) | fp16/bf16 (L-128)
  const void *NLp;     // the negation of Lp
  const void *Rp;      // uint8 R | fp16/bf16 R
  const int32_t *negSL;  // 128*n - S_L (int path) or 128*n - S_L as well (fp path)
  const float *invL;     // 1/sqrt(varN_L), NaN where the candidate set is empty
  const int32_t *SR;     // S_R
  const float *invR;     // 1/sqrt(varN_R), NaN where invalid
  uint32_t *keyL;        // H*W merged left-reference keys
  uint32_t *keyR;        // H*W merged right-reference keys
  int32_t H, W, win, dmin, dmax;
  int32_t strideL, padL, strideR, padR;
  int32_t xs0;          // first column of lane 0 of span 0
  int32_t nspan, nband, nchunk, TY, DC;
  int32_t CG, ncg;      // chunks per workgroup task, chunk groups
  int32_t rp;           // slot stride of the right key tile (4 mod 8)
  int32_t first_task;   // index of this pair's first task in a batched queue
  int32_t chess;        // 1: chessboard window (cells u + v even around the centre)
  int32_t nwin;         // cells of the window: win^2, or (win^2 + 1) / 2 for the chessboard
  uint32_t lplane;      // bytes from the colour-0 copy of Lp / NLp to the colour-1 copy
};

// Dense per-pair view used by the post-processing kernels.  A batched
// launch reads entry blockIdx.z of a device table; a single-pair launch gets
// the descriptor by value.
struct PostPair {
  const uint8_t *left, *right;
  int32_t H, W, pitch, win, dmin, dmax;
  int32_t chess;                       // 1: chessboard window
  const int32_t *SL, *SSL, *SR, *SSR;  // dense window sums (0 outside)
  uint32_t *keyL, *keyR;               // merged WTA keys (cleared by decode)
  int16_t *oR;
  uint8_t *mR;
  int16_t *ob[3];                      // [0] WTA disparity, [1] [2] ping-pong
  uint8_t *mb[3];                      // masks, same roles
  double *zbest, *zm, *zp;             // may be null
  float *delta;
  int32_t *pc, *ps;                    // row prefix sums (count, sum), H x (W+1)
  uint32_t *hits;                      // 8 planes: nearest valid pixel per direction
  uint8_t *pass;                       // 4 planes: outlier runs per line type
  double *f;                           // 6 smoothing planes of H x W
  const float *s_in;                   // optional smoothing input (stage entry)
  float *disparity;
  uint8_t *valid_mask;
};

// Inputs and outputs of the plane/statistics preparation of one pair.
struct PrepPair {
  const uint8_t *L, *R;
  int32_t H, W, pitch, win;
  int32_t chess;                         // 1: chessboard window, two L plane copies
  void *Lp, *NLp, *Rp;                   // padded image planes
  int32_t *negSL, *SRp;                  // padded statistics planes
  float *invL, *invR;
  int32_t strideL, padL, strideR, padR;
  int32_t *SL, *SSL, *SR, *SSR;          // dense window sums
  float *invLd, *invRd;                  // dense inverse deviations (may be null)
};

// A pixel-parallel launch over one pair (descriptor by value) or a batch
// (device table, grid.z = pair, grid sized for the largest pair).
struct PostLaunch {
  PostPair one;
  const PostPair *many;  // null for a single pair
  int npairs, maxH, maxW;
  int maxWin, maxD;  // largest window and disparity count over the pairs
  hipStream_t s;
};

struct RefineArgs {
  const uint8_t *L, *R;
  const float *d;
  const uint8_t *mask;
  int H, W, pitch, win;
  int sy;           // rows per block of the fused passes (set by the launchers)
  double lambda;
  double *f;        // planes of H*W doubles
  double *partial;  // one double per block of the energy kernel
  float *Z;         // may be null
  double *E;
  float *grad;
};

__host__ __device__ inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

// Block coordinates (x, y, pair) of a launch with grid (X, Y, pairs).  The
// launched blocks are spread over the 8 XCDs round-robin (block b runs on
// XCD b % 8); they are renumbered so that each XCD takes one contiguous
// eighth of the blocks in (pair, y, x) order.  An XCD then works through a
// few neighbouring row bands of one or two pairs at a time, and data that
// neighbouring blocks share (scan look-aheads, window halos, staged rows)
// stays in its L2.
struct BlockPos {
  int x, y, pair;
};
__device__ __forceinline__ BlockPos block_pos() {
  const int X = gridDim.x, Y = gridDim.y;
  const int T = X * Y * gridDim.z;
  const int b = blockIdx.x + X * (blockIdx.y + Y * blockIdx.z);
  const int xcd = b & 7, s = b >> 3;
  const int g = xcd * (T >> 3) + min(xcd, T & 7) + s;
  BlockPos q;
  q.x = g % X;
  const int r = g / X;
  q.y = r % Y;
  q.pair = r / Y;
  return q;
}

// ---- host launchers (one per stage); all return hipGetLastError()
// The padded planes on s, the window statistics on s_stats (s when null; the
// two write disjoint parts of the planes and may run side by side).
hipError_t launch_prep(const PrepPair &one, const PrepPair *many, int npairs, int maxH,
                       int maxCols, int maxW, int prec, hipStream_t s,
                       hipStream_t s_stats = nullptr);
hipError_t launch_match(const MatchPair &P, int prec, hipStream_t s);
// One persistent matcher launch over the tasks of one window size and one
// chunk width dc (4 or 8 disparities per lane); ev0/ev1 (may be null) are
// recorded on s just before and after it.
hipError_t launch_match_persistent(const MatchPair *pairs_dev, const int4 *tasks_dev, int ntasks,
                                   int *counter_dev, int win, int dc, int prec, int nblocks,
                                   size_t lds, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1);
// resident matcher workgroups per CU with `lds` bytes of key tiles each
int match_persistent_occupancy(int win, int dc, int prec, size_t lds);
size_t match_lds_bytes(const MatchPair &P);  // key tiles of one workgroup
hipError_t launch_window_stats_dense(const uint8_t *img, int H, int W, int pitch, int win,
                                     int chess, int32_t *S, int32_t *SS, float *inv, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, int N, uint32_t v, hipStream_t s);
// out = m ? o : O_NONE over N pixels (a caller's map in the form the radial
// scans read)
hipError_t launch_mark_invalid(const int16_t *o, const uint8_t *m, int16_t *out, size_t N,
                               hipStream_t s);
struct Mat4 {
  double q[16];
};
hipError_t launch_reproject(const float *disp, int H, int W, const Mat4 &Q, float *xyz, hipStream_t s);
hipError_t post_decode(const PostLaunch &L);
hipError_t post_subpixel(const PostLaunch &L);
hipError_t post_lr(const PostLaunch &L, int tol, int dst);
// post_subpixel and post_lr in one launch
hipError_t post_subpixel_lr(const PostLaunch &L, int tol, int dst);
hipError_t post_outlier(const PostLaunch &L, int r, float thresh, int src, int dst);
hipError_t post_fill(const PostLaunch &L, int radial_r, int min_lines, int disk_r, float frac,
                     int src, int tmp, int dst);
// Per-iteration state of the Eq. (4) loop kept for a debug readout (single
// pair): after re-search j (j = 0 .. n-1) the new o goes to o + j N and the
// d it was centred on to d + j N.
struct HcTrace {
  int16_t *o;
  double *d;
  int n;
};
hipError_t post_hc(const PostLaunch &L, int src, int R, int K, float alpha, int use_delta,
                   int research, int range, float eta, const HcTrace *trace = nullptr);
// one Eq. (4) re-search: o from ob[osrc], mask mb[msrc], d from FP64 plane
// dplane of f; the new o goes to ob[odst]
hipError_t post_research(const PostLaunch &L, int osrc, int msrc, int odst, int dplane, int range,
                         float eta);
int refine_planes();
int refine_partials(int H, int W);
hipError_t launch_refine_forward(const RefineArgs &A, hipStream_t s);
hipError_t launch_refine_backward(const RefineArgs &A, hipStream_t s);
hipError_t launch_refine_step(float *d, const float *g, const uint8_t *mask, int N, float tau,
                              float ms, hipStream_t s);

}  // namespace st
