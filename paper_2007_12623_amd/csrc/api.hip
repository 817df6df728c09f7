// C ABI of the stereo library (declared in include/stereo.h): argument
// checks, handle and scratch management, orchestration of the stages of the
// paper's Section II pipeline, the batched persistent launch with graph
// replay, the matcher autotuner and the refinement entry points.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "common.h"
#include "stereo.h"

using namespace st;

// ---------------------------------------------------------------- profiler ranges
// A named range of the host timeline (the enqueueing of a stage, shown by
// rocprofv3 --marker-trace); without a profiler attached it is a no-op.
struct Range {
  explicit Range(const char *name) { roctxRangePushA(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range &) = delete;
  Range &operator=(const Range &) = delete;
};

// ---------------------------------------------------------------- errors
static thread_local std::string g_err;

static st_status fail(st_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define ARG(cond, ...)                          \
  do {                                          \
    if (!(cond)) return fail(ST_EINVAL, __VA_ARGS__); \
  } while (0)

#define HIPCK(call)                                                                       \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) {                                                               \
      if (h) h->keys_dirty = true;                                                        \
      return fail(ST_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));                \
    }                                                                                     \
  } while (0)

// Make the handle's device current for the calling thread.
#define SETDEV(h)                                                                  \
  do {                                                                             \
    const hipError_t e_ = hipSetDevice((h)->device);                               \
    if (e_ != hipSuccess)                                                          \
      return fail(ST_EHIP, "hipSetDevice(%d) failed: %s", (h)->device, hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------- variants
// Matcher tilings: band height TY, chunks per workgroup task CG and
// disparities per lane DC (the chunk width), in the order the default
// choice prefers them.  Bands of 8 rows come first: their key tiles (about
// 37 KB) leave room for three workgroups per CU, which the matcher's
// register budget (three waves per SIMD) is sized for; among them fewer key
// merges and fewer vertical-sum restarts first.  Chunks of 4 disparities
// halve the registers of the running sums but convert and merge twice as
// many keys per evaluation; the autotuners try them like any other tiling.
struct Variant {
  int TY, CG, DC;
};
static const Variant kVariants[] = {{8, 16, 8}, {8, 8, 8},  {16, 16, 8}, {16, 8, 8}, {8, 4, 8},
                                    {16, 4, 8}, {8, 2, 8},  {16, 2, 8},  {4, 4, 8},  {4, 2, 8},
                                    {8, 32, 4}, {8, 16, 4}, {16, 32, 4}, {8, 8, 4}, {10, 16, 8},
                                    {6, 16, 8}};
static const int kNumVariants = (int)(sizeof kVariants / sizeof kVariants[0]);

// ---------------------------------------------------------------- handle
struct DevBuf {
  void *p = nullptr;
  size_t n = 0;
};

struct BatchCache {
  std::vector<st_pair> pairs;
  st_params params{};
  int variant = -2;
  unsigned tune_gen = 0;  // the tuning table's generation the graph was built with
  // what the matcher launches of this batch need, for stereo_time_matcher:
  // one persistent launch per window size present in the batch
  struct Group {
    int win, dc, variant, off, ntasks, nblocks;
    size_t lds;
  };
  std::vector<Group> groups;
  MatchPair *tM = nullptr;
  int4 *tT = nullptr;
  int *tC = nullptr;
  int prec = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  DevBuf ws, keys, tables;
};

struct st_handle_s {
  int device = 0;
  int ncu = 256;
  hipStream_t cap_stream = nullptr;
  // a second capture stream and its fork / join events: the persistent
  // launches of a batch's window sizes after the first run beside it
  hipStream_t side_stream = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr, post_fork = nullptr;
  // the window statistics of a batch beside its plane preparation
  hipEvent_t prep_fork = nullptr, prep_join = nullptr;
  // capture streams of the post-processing of a batch's image sizes after
  // the first (created when a batch first needs them), their join events
  std::vector<hipStream_t> post_streams;
  std::vector<hipEvent_t> post_done;
  DevBuf ws, keys, rws, dbgrs;
  bool keys_dirty = false;
  int variant = -1;
  std::map<std::string, int> tune;
  unsigned tune_gen = 0;  // bumped whenever the tuning table changes
  std::map<std::string, void *> dbg;
  BatchCache batch;
};

// ---------------------------------------------------------------- fixed scratch
// The scratch of stereo_match_noalloc: a file-scope device array, of which
// every GPU the library runs on holds its own copy until the process ends.
// In host code the array's name is only a host-side stand-in: kernels get the
// device address that hipGetSymbolAddress returns for the current device,
// looked up once per device when the first handle on it is created.
static __device__ __align__(256) unsigned char scratch[ST_NOALLOC_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch[kMaxDevices];

// This device's copy of `scratch` (the device must be current).
static st_status scratch_lookup(int device) {
  if (device >= kMaxDevices) return fail(ST_EUNSUPPORTED, "device %d: at most %d devices", device, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[device]) return ST_OK;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    return fail(ST_EHIP, "hipGetSymbolAddress(scratch) on device %d failed: %s", device,
                hipGetErrorString(e));
  }
  g_scratch[device] = p;
  return ST_OK;
}

static bool fault_alloc() {
  const char *e = getenv("STEREO_FAULT");
  return e && strcmp(e, "alloc") == 0;
}

// Grow a device buffer to at least `need` bytes (contents are not kept).
static st_status grow(st_handle h, DevBuf &b, size_t need, bool zero) {
  if (b.n >= need && b.p) return ST_OK;
  if (fault_alloc()) return fail(ST_ENOMEM, "device allocation of %zu bytes failed (injected)", need);
  if (b.p) {
    (void)hipDeviceSynchronize();  // the buffer may still be in use by queued work
    (void)hipFree(b.p);
    b.p = nullptr;
    b.n = 0;
  }
  void *p = nullptr;
  if (hipMalloc(&p, need) != hipSuccess || !p) {
    (void)hipGetLastError();
    return fail(ST_ENOMEM, "device allocation of %zu bytes failed", need);
  }
  if (zero && hipMemset(p, 0, need) != hipSuccess) {
    (void)hipFree(p);
    return fail(ST_EHIP, "hipMemset of scratch failed");
  }
  b.p = p;
  b.n = need;
  (void)h;
  return ST_OK;
}

static void release(DevBuf &b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.n = 0;
}

// ---------------------------------------------------------------- checks
static st_status check_shape(int H, int W, int pitch, int dmin, int dmax, int win) {
  ARG(win >= 3 && win <= 15 && (win & 1), "win must be odd and in [3, 15] (got %d)", win);
  // bounds first, so that the range below is computed without overflow
  ARG(dmin >= -4096 && dmax <= 4096, "disparities beyond +-4096 are not supported");
  ARG(dmax >= dmin, "dmax < dmin (%d < %d)", dmax, dmin);
  const int D = dmax - dmin + 1;
  ARG(D <= 256, "dmax - dmin + 1 must be at most 256 (got %d)", D);
  // a valid request: the matcher's disparity chunks are 8 wide
  if (D < 8)
    return fail(ST_EUNSUPPORTED, "ranges of fewer than 8 disparities are not implemented (got %d)", D);
  ARG(H >= win && W >= win, "image %dx%d smaller than the window %d", W, H, win);
  ARG((long long)H * W <= (1LL << 28), "image too large");
  ARG(pitch >= W, "pitch %d < width %d", pitch, W);
  return ST_OK;
}

static st_status check_params(const st_params *p) {
  ARG(p, "params is NULL");
  ARG(p->struct_size == (int32_t)sizeof(st_params), "params.struct_size %d != %d", p->struct_size,
      (int)sizeof(st_params));
  ARG(p->precision >= 0 && p->precision <= 2, "unknown precision %d", p->precision);
  ARG(p->lr_tol >= 0, "lr_tol < 0");
  ARG(p->radial_iters >= 0 && p->radial_iters <= 64, "radial_iters out of range");
  ARG(p->radial_r0 >= 1 && p->radial_dr >= 0 && p->radial_r0 + 64 * p->radial_dr <= 4096,
      "radial radii out of range");
  ARG(p->fill_radial_r >= 0 && p->fill_radial_r <= 4096, "fill_radial_r out of range");
  ARG(p->fill_min_lines >= 1 && p->fill_min_lines <= 4, "fill_min_lines must be in [1, 4]");
  ARG(p->fill_disk_r >= 0 && p->fill_disk_r <= 2048, "fill_disk_r out of range");
  ARG(p->fill_disk_min_frac >= 0.0f && p->fill_disk_min_frac <= 1.0f, "fill_disk_min_frac not in [0,1]");
  ARG(p->smooth_radius >= 0 && p->smooth_radius <= 2048, "smooth_radius out of range");
  ARG(p->smooth_iters >= 0 && p->smooth_iters <= 64, "smooth_iters out of range");
  ARG(p->research == 0 || p->research == 1, "research must be 0 or 1");
  ARG(p->research_range >= 0 && p->research_range <= 64, "research_range out of range");
  ARG(p->research_eta >= 0.0f, "research_eta < 0");
  ARG(!p->research || p->smooth_radius <= 64, "the Eq. (4) re-search needs smooth_radius <= 64");
  ARG(p->chessboard == 0 || p->chessboard == 1, "chessboard must be 0 or 1");
  return ST_OK;
}

// ---------------------------------------------------------------- geometry
static int round_up(int v, int m) { return ((v + m - 1) / m) * m; }
static int pmod(int a, int m) { return ((a % m) + m) % m; }

// Spans, bands, chunks and plane padding of one pair for the matcher.
static void make_geom(MatchPair &P, int H, int W, int win, int dmin, int dmax, int DC, int TY,
                      int CG, int chess) {
  const int h = win / 2, K = KC;
  P.H = H;
  P.W = W;
  P.win = win;
  P.chess = chess;
  P.nwin = chess ? (win * win + 1) / 2 : win * win;
  P.lplane = 0;
  P.dmin = dmin;
  P.dmax = dmax;
  P.DC = DC;
  P.TY = TY;
  // lane columns x0 = xs + 8 l with xs = dmin - 1 (mod 8): the right-image
  // segment of every lane then starts on a 4-column boundary, except in a
  // last chunk that had to be shifted down to end at dmax
  const int target = h - K, r = pmod(dmin - 1, 8);
  P.xs0 = target - pmod(target - r, 8);
  const int span = OUT_LANES * K;
  P.nspan = std::max(1, ceil_div(W - h - (P.xs0 + K), span));
  P.nband = ceil_div(H - 2 * h, TY);
  const int D = dmax - dmin + 1;
  P.nchunk = ceil_div(D, DC);
  const int xs_last = P.xs0 + (P.nspan - 1) * span;
  const int Lmax = xs_last + WV * K;
  P.padL = P.xs0 < 0 ? -P.xs0 : pmod(-P.xs0, 8);
  P.strideL = round_up(P.padL + std::max(W, Lmax), 16);
  const int d0_last = dmin + std::min((P.nchunk - 1) * DC, D - DC);
  const int Rmin = P.xs0 - d0_last - (DC - 1);
  const int Rmax = xs_last + WV * K - dmin + 8;  // dword-rounded segment reads
  P.padR = round_up(std::max(0, -Rmin), 4);
  P.strideR = round_up(P.padR + std::max(W, Rmax), 16);
  P.first_task = 0;
  // chunk groups and the right key tile: 512 + 7 + (d0 of the group's last
  // chunk - d0 of its first) columns in slots of rp, rp = 4 (mod 8)
  P.CG = std::max(1, std::min(CG, P.nchunk));
  P.ncg = ceil_div(P.nchunk, P.CG);
  const int rw = WV * KC + (DC - 1) + DC * (P.CG - 1);
  P.rp = ceil_div(rw, 8);
  P.rp += (4 - P.rp % 8 + 8) % 8;
}

static int pick_variant(st_handle h, int H, int W, int win, int dmin, int dmax, int prec);

// ---------------------------------------------------------------- scratch layout
struct Carve {
  size_t off = 0;
  size_t take(size_t bytes) {
    off = (off + 255) & ~(size_t)255;
    const size_t o = off;
    off += bytes;
    return o;
  }
};

// Offsets of every per-pair buffer inside one scratch region.
struct PairLayout {
  size_t Lp, NLp, Rp, negSL, invL, SRp, invR, SL, SSL, SR, SSR, oR, mR, ob[3], mb[3], zbest,
      zm, zp, delta, pc, ps, f, dbg_mlr, dbg_o, dbg_m;
  size_t total;
};

static PairLayout layout(const MatchPair &P, int prec, bool debug) {
  PairLayout Lo{};
  Carve c;
  const size_t N = (size_t)P.H * P.W;
  const size_t nl = (size_t)P.strideL * P.H, nr = (size_t)P.strideR * P.H;
  const int RB = prec == P_I16 ? 1 : 2;
  // two colour copies of the L planes for the chessboard window
  const size_t ncopy = P.chess ? 2 : 1;
  Lo.Lp = c.take(2 * nl * ncopy);
  Lo.NLp = c.take(2 * nl * ncopy);
  Lo.Rp = c.take(RB * nr + 64);
  Lo.negSL = c.take(4 * nl);
  Lo.invL = c.take(4 * nl);
  Lo.SRp = c.take(4 * nr);
  Lo.invR = c.take(4 * nr);
  Lo.SL = c.take(4 * N);
  Lo.SSL = c.take(4 * N);
  Lo.SR = c.take(4 * N);
  Lo.SSR = c.take(4 * N);
  Lo.oR = c.take(2 * N);
  Lo.mR = c.take(N);
  for (int i = 0; i < 3; ++i) {
    Lo.ob[i] = c.take(2 * N);
    Lo.mb[i] = c.take(N);
  }
  Lo.delta = c.take(4 * N);
  Lo.pc = c.take(4 * (size_t)P.H * (P.W + 1));
  Lo.ps = c.take(4 * (size_t)P.H * (P.W + 1));
  // the smoothing's FP64 planes; before the smoothing starts the same bytes
  // hold the radial scans (8 x 4 bytes of nearest hits, 4 x 1 byte of runs)
  Lo.f = c.take(6 * 8 * N);
  if (debug) {
    // the FP64 scores of the sub-pixel step are written for the debug
    // readout only
    Lo.zbest = c.take(8 * N);
    Lo.zm = c.take(8 * N);
    Lo.zp = c.take(8 * N);
    Lo.dbg_mlr = c.take(N);
    Lo.dbg_o = c.take(2 * N);
    Lo.dbg_m = c.take(N);
  }
  Lo.total = c.take(0);
  return Lo;
}

template <class T>
static T *at(void *base, size_t off) {
  return (T *)((char *)base + off);
}

static void fill_views(const PairLayout &Lo, void *base, uint32_t *keys, MatchPair &M, PrepPair &Pp,
                       PostPair &Q, const uint8_t *left, const uint8_t *right, int pitch) {
  const size_t N = (size_t)M.H * M.W;
  M.Lp = at<void>(base, Lo.Lp);
  M.NLp = at<void>(base, Lo.NLp);
  M.lplane = M.chess ? (uint32_t)(2 * (size_t)M.strideL * M.H) : 0u;
  M.Rp = at<void>(base, Lo.Rp);
  M.negSL = at<int32_t>(base, Lo.negSL);
  M.invL = at<float>(base, Lo.invL);
  M.SR = at<int32_t>(base, Lo.SRp);
  M.invR = at<float>(base, Lo.invR);
  M.keyL = keys;
  M.keyR = keys + N;

  Pp = PrepPair{};
  Pp.L = left;
  Pp.R = right;
  Pp.H = M.H;
  Pp.W = M.W;
  Pp.pitch = pitch;
  Pp.win = M.win;
  Pp.chess = M.chess;
  Pp.Lp = at<void>(base, Lo.Lp);
  Pp.NLp = at<void>(base, Lo.NLp);
  Pp.Rp = at<void>(base, Lo.Rp);
  Pp.negSL = at<int32_t>(base, Lo.negSL);
  Pp.invL = at<float>(base, Lo.invL);
  Pp.SRp = at<int32_t>(base, Lo.SRp);
  Pp.invR = at<float>(base, Lo.invR);
  Pp.strideL = M.strideL;
  Pp.padL = M.padL;
  Pp.strideR = M.strideR;
  Pp.padR = M.padR;
  Pp.SL = at<int32_t>(base, Lo.SL);
  Pp.SSL = at<int32_t>(base, Lo.SSL);
  Pp.SR = at<int32_t>(base, Lo.SR);
  Pp.SSR = at<int32_t>(base, Lo.SSR);

  Q = PostPair{};
  Q.left = left;
  Q.right = right;
  Q.H = M.H;
  Q.W = M.W;
  Q.pitch = pitch;
  Q.win = M.win;
  Q.chess = M.chess;
  Q.dmin = M.dmin;
  Q.dmax = M.dmax;
  Q.SL = Pp.SL;
  Q.SSL = Pp.SSL;
  Q.SR = Pp.SR;
  Q.SSR = Pp.SSR;
  Q.keyL = keys;
  Q.keyR = keys + N;
  Q.oR = at<int16_t>(base, Lo.oR);
  Q.mR = at<uint8_t>(base, Lo.mR);
  for (int i = 0; i < 3; ++i) {
    Q.ob[i] = at<int16_t>(base, Lo.ob[i]);
    Q.mb[i] = at<uint8_t>(base, Lo.mb[i]);
  }
  // offset 0 is the first L plane, so 0 marks a buffer left out
  Q.zbest = Lo.zbest ? at<double>(base, Lo.zbest) : nullptr;
  Q.zm = Lo.zm ? at<double>(base, Lo.zm) : nullptr;
  Q.zp = Lo.zp ? at<double>(base, Lo.zp) : nullptr;
  Q.delta = at<float>(base, Lo.delta);
  Q.pc = at<int32_t>(base, Lo.pc);
  Q.ps = at<int32_t>(base, Lo.ps);
  Q.f = at<double>(base, Lo.f);
  Q.hits = at<uint32_t>(base, Lo.f);
  Q.pass = at<uint8_t>(base, Lo.f + 32 * N);
}

// ---------------------------------------------------------------- pipeline
// Where the single-pair path copies intermediates for stereo_debug_get.
struct DebugSink {
  void *mlr, *o, *m;
  size_t N;
  HcTrace trace;  // the Eq. (4) loop's states (trace.n = 0: none kept)
};

// Every stage after the matcher, identical for the single and the batched
// path: decode, sub-pixel, left-right check, outlier removal / hole filling
// (ping-pong buffers 1 and 2; buffer 0 keeps the WTA result), smoothing.
static hipError_t post_stages(const PostLaunch &L, const st_params &p, const DebugSink *dbg) {
  hipError_t e = hipSuccess;
  auto ck = [&](hipError_t x) {
    if (x != hipSuccess && e == hipSuccess) e = x;
  };
  ck(post_decode(L));
  int cur = 0;
  if (p.subpixel && p.lr_check) {
    ck(post_subpixel_lr(L, p.lr_tol, 1));
    cur = 1;
  } else {
    if (p.subpixel) ck(post_subpixel(L));
    if (p.lr_check) {
      ck(post_lr(L, p.lr_tol, 1));
      cur = 1;
    }
  }
  if (dbg) ck(hipMemcpyAsync(dbg->mlr, L.one.mb[cur], dbg->N, hipMemcpyDeviceToDevice, L.s));
  if (p.radial_iters <= 0) {
    const int tmp = cur == 1 ? 2 : 1, dst = cur == 0 ? 2 : cur;
    ck(post_fill(L, p.fill_radial_r, p.fill_min_lines, p.fill_disk_r, p.fill_disk_min_frac, cur,
                 tmp, dst));
    cur = dst;
  } else {
    for (int it = 0; it < p.radial_iters; ++it) {
      const int r = p.radial_r0 + it * p.radial_dr;
      const int nxt = cur == 1 ? 2 : 1;
      ck(post_outlier(L, r, p.radial_thresh, cur, nxt));
      const int tmp = nxt == 1 ? 2 : 1;
      ck(post_fill(L, p.fill_radial_r, p.fill_min_lines, p.fill_disk_r, p.fill_disk_min_frac, nxt,
                   tmp, nxt));
      cur = nxt;
    }
  }
  if (dbg) {
    ck(hipMemcpyAsync(dbg->o, L.one.ob[cur], 2 * dbg->N, hipMemcpyDeviceToDevice, L.s));
    ck(hipMemcpyAsync(dbg->m, L.one.mb[cur], dbg->N, hipMemcpyDeviceToDevice, L.s));
  }
  ck(post_hc(L, cur, p.smooth_radius, p.smooth_iters, p.smooth_alpha, p.subpixel, p.research,
             p.research_range, p.research_eta, dbg && dbg->trace.n > 0 ? &dbg->trace : nullptr));
  return e;
}

static int variant_TY(int v) { return kVariants[v].TY; }
static int variant_CG(int v) { return kVariants[v].CG; }
static int variant_DC(int v) { return kVariants[v].DC; }

extern "C" {

void st_default_params(st_params *p) {
  if (!p) return;
  memset(p, 0, sizeof *p);
  p->struct_size = sizeof(st_params);
  p->subpixel = 1;
  p->lr_check = 1;
  p->lr_tol = 1;
  p->radial_iters = 3;
  p->radial_r0 = 10;
  p->radial_dr = 10;
  p->radial_thresh = 2.5f;
  p->fill_radial_r = 50;
  p->fill_min_lines = 2;
  p->fill_disk_r = 20;
  p->fill_disk_min_frac = 0.25f;
  p->smooth_radius = 15;
  p->smooth_iters = 3;
  p->smooth_alpha = 0.1f;
  p->precision = ST_FP32;
  p->debug_outputs = 0;
  p->research = 0;
  p->research_range = 5;
  p->research_eta = 0.01f;
  p->chessboard = 0;
}

const char *st_last_error(void) { return g_err.c_str(); }

const char *st_version(void) { return "stereo_mi355x 1.0 (gfx950, HIP)"; }

int st_num_variants(void) { return kNumVariants; }

const char *st_variant_name(int v) {
  static thread_local char buf[64];
  if (v < 0 || v >= kNumVariants) return "";
  snprintf(buf, sizeof buf, "TY=%d,CG=%d,DC=%d", kVariants[v].TY, kVariants[v].CG,
           kVariants[v].DC);
  return buf;
}

static void load_tune(st_handle h);
static void save_tune(st_handle h);

st_status st_create(st_handle *out, int device) {
  ARG(out, "out is NULL");
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
    (void)hipGetLastError();
    return fail(ST_ENODEV, "no HIP device");
  }
  ARG(device >= 0, "device < 0");
  if (device >= n) return fail(ST_ENODEV, "device %d does not exist (%d devices)", device, n);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess)
    return fail(ST_ENODEV, "cannot query device %d", device);
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(ST_ENODEV, "device %d is %s, this library is built for gfx950", device,
                prop.gcnArchName);
  if (hipSetDevice(device) != hipSuccess) return fail(ST_ENODEV, "cannot select device %d", device);
  st_handle h = new st_handle_s();
  h->device = device;
  h->ncu = prop.multiProcessorCount;
  const st_status rs = scratch_lookup(device);
  if (rs != ST_OK) {
    delete h;
    return rs;
  }
  if (hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&h->side_stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&h->fork_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->join_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->post_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->prep_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->prep_join, hipEventDisableTiming) != hipSuccess) {
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    if (h->side_stream) (void)hipStreamDestroy(h->side_stream);
    if (h->fork_ev) (void)hipEventDestroy(h->fork_ev);
    if (h->join_ev) (void)hipEventDestroy(h->join_ev);
    if (h->post_fork) (void)hipEventDestroy(h->post_fork);
    if (h->prep_fork) (void)hipEventDestroy(h->prep_fork);
    delete h;
    return fail(ST_EHIP, "cannot create the capture streams");
  }
  load_tune(h);
  *out = h;
  return ST_OK;
}

static void drop_batch(BatchCache &b) {
  if (b.exec) (void)hipGraphExecDestroy(b.exec);
  if (b.graph) (void)hipGraphDestroy(b.graph);
  b.exec = nullptr;
  b.graph = nullptr;
  b.pairs.clear();
  b.variant = -2;
}

void st_destroy(st_handle h) {
  if (!h) return;
  // teardown is best effort: a failing call cannot be reported from here
  (void)hipSetDevice(h->device);
  (void)hipDeviceSynchronize();
  drop_batch(h->batch);
  release(h->batch.ws);
  release(h->batch.keys);
  release(h->batch.tables);
  release(h->ws);
  release(h->keys);
  release(h->rws);
  release(h->dbgrs);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  if (h->side_stream) (void)hipStreamDestroy(h->side_stream);
  if (h->fork_ev) (void)hipEventDestroy(h->fork_ev);
  if (h->join_ev) (void)hipEventDestroy(h->join_ev);
  if (h->post_fork) (void)hipEventDestroy(h->post_fork);
  if (h->prep_fork) (void)hipEventDestroy(h->prep_fork);
  if (h->prep_join) (void)hipEventDestroy(h->prep_join);
  for (hipStream_t ps : h->post_streams) (void)hipStreamDestroy(ps);
  for (hipEvent_t pe : h->post_done) (void)hipEventDestroy(pe);
  delete h;
}

// Prepare scratch for one pair and fill the device views.
static st_status setup_single(st_handle h, const uint8_t *left, const uint8_t *right, int H, int W,
                              int pitch, int dmin, int dmax, int win, int chess, int prec,
                              int variant, bool debug, MatchPair &M, PrepPair &Pp, PostPair &Q,
                              PairLayout &Lo, hipStream_t s) {
  make_geom(M, H, W, win, dmin, dmax, variant_DC(variant), variant_TY(variant), variant_CG(variant),
            chess);
  Lo = layout(M, prec, debug);
  st_status rc = grow(h, h->ws, Lo.total, false);
  if (rc) return rc;
  const size_t N = (size_t)H * W;
  if (h->keys.n < 8 * N) {
    rc = grow(h, h->keys, 8 * N, true);
    if (rc) return rc;
    h->keys_dirty = false;
  }
  if (h->keys_dirty) {
    HIPCK(launch_fill_u32((uint32_t *)h->keys.p, (int)(2 * N), 0u, s));
    h->keys_dirty = false;
  }
  fill_views(Lo, h->ws.p, (uint32_t *)h->keys.p, M, Pp, Q, left, right, pitch);
  return ST_OK;
}

static st_status run_front(st_handle h, const MatchPair &M, const PrepPair &Pp, int prec,
                           hipStream_t s) {
  HIPCK(launch_prep(Pp, nullptr, 1, M.H, std::max(M.strideL, M.strideR), M.W, prec, s));
  HIPCK(launch_match(M, prec, s));
  return ST_OK;
}

static PostLaunch single_launch(const PostPair &Q, hipStream_t s) {
  PostLaunch L;
  L.one = Q;
  L.many = nullptr;
  L.npairs = 1;
  L.maxH = Q.H;
  L.maxW = Q.W;
  L.maxWin = Q.win;
  L.maxD = Q.dmax - Q.dmin + 1;
  L.s = s;
  return L;
}

st_status stereo_match(st_handle h, const uint8_t *left, const uint8_t *right, int H, int W,
                       int pitch, int dmin, int dmax, int win, const st_params *params,
                       float *disparity, uint8_t *valid_mask, void *stream) {
  st_status rc = check_shape(H, W, pitch, dmin, dmax, win);
  if (rc) return rc;
  rc = check_params(params);
  if (rc) return rc;
  ARG(left && right && disparity && valid_mask, "NULL image or output pointer");
  ARG(h, "NULL handle");
  SETDEV(h);
  hipStream_t s = (hipStream_t)stream;
  const int prec = params->precision;
  const bool debug = params->debug_outputs != 0;
  const int v = pick_variant(h, H, W, win, dmin, dmax, prec);
  MatchPair M;
  PrepPair Pp;
  PostPair Q;
  PairLayout Lo;
  rc = setup_single(h, left, right, H, W, pitch, dmin, dmax, win, params->chessboard, prec, v,
                    debug, M, Pp, Q, Lo, s);
  if (rc) return rc;
  h->dbg.clear();
  Range whole("stereo_match");
  {
    Range r("stereo_match: planes, statistics, matcher");
    rc = run_front(h, M, Pp, prec, s);
  }
  if (rc) return rc;
  Q.disparity = disparity;
  Q.valid_mask = valid_mask;
  PostLaunch L = single_launch(Q, s);
  const size_t N = (size_t)H * W;
  DebugSink sink{at<void>(h->ws.p, Lo.dbg_mlr), at<void>(h->ws.p, Lo.dbg_o),
                 at<void>(h->ws.p, Lo.dbg_m), N, HcTrace{nullptr, nullptr, 0}};
  const int nrs = debug && params->research ? std::max(0, params->smooth_iters - 1) : 0;
  if (nrs > 0) {
    // the state after every re-search: o (int16) and the d it was centred on
    rc = grow(h, h->dbgrs, (size_t)nrs * 10 * N + 256, false);
    if (rc) return rc;
    sink.trace.d = (double *)h->dbgrs.p;
    sink.trace.o = (int16_t *)((double *)h->dbgrs.p + (size_t)nrs * N);
    sink.trace.n = nrs;
  }
  {
    Range r("stereo_match: decode, sub-pixel, left-right, outliers, fills, smoothing");
    HIPCK(post_stages(L, *params, debug ? &sink : nullptr));
  }
  if (debug) {
    h->dbg["o_wta"] = Q.ob[0];
    h->dbg["m_wta"] = Q.mb[0];
    h->dbg["o_r"] = Q.oR;
    h->dbg["m_r"] = Q.mR;
    h->dbg["zbest"] = Q.zbest;
    h->dbg["zm"] = Q.zm;
    h->dbg["zp"] = Q.zp;
    h->dbg["delta"] = Q.delta;
    h->dbg["m_lr"] = at<void>(h->ws.p, Lo.dbg_mlr);
    h->dbg["o_post"] = at<void>(h->ws.p, Lo.dbg_o);
    h->dbg["m_post"] = at<void>(h->ws.p, Lo.dbg_m);
    for (int j = 0; j < nrs; ++j) {
      h->dbg["o_rs" + std::to_string(j + 1)] = sink.trace.o + (size_t)j * N;
      h->dbg["d_rs" + std::to_string(j + 1)] = sink.trace.d + (size_t)j * N;
    }
  }
  return ST_OK;
}

st_status stereo_match_noalloc(st_handle h, const uint8_t *left, const uint8_t *right, int H,
                               int W, int pitch, int dmin, int dmax, int win,
                               const st_params *params, float *disparity, uint8_t *valid_mask,
                               void *stream) {
  st_status rc = check_shape(H, W, pitch, dmin, dmax, win);
  if (rc) return rc;
  rc = check_params(params);
  if (rc) return rc;
  ARG(left && right && disparity && valid_mask, "NULL image or output pointer");
  ARG(h, "NULL handle");
  ARG(!params->debug_outputs,
      "debug_outputs needs handle-owned buffers: use stereo_match for a debug run");
  void *base = h->device < kMaxDevices ? g_scratch[h->device] : nullptr;
  if (!base) return fail(ST_EHIP, "no scratch address for device %d", h->device);
  const int prec = params->precision;
  const int v = pick_variant(h, H, W, win, dmin, dmax, prec);
  MatchPair M;
  PrepPair Pp;
  PostPair Q;
  make_geom(M, H, W, win, dmin, dmax, variant_DC(v), variant_TY(v), variant_CG(v),
            params->chessboard);
  const PairLayout Lo = layout(M, prec, false);
  const size_t N = (size_t)H * W;
  const size_t koff = (Lo.total + 255) & ~(size_t)255, need = koff + 8 * N;
  if (need > (size_t)ST_NOALLOC_SCRATCH_BYTES)
    return fail(ST_EUNSUPPORTED,
                "a %dx%d pair with %d disparities needs %zu bytes of scratch; the fixed scratch "
                "of stereo_match_noalloc holds %zu",
                W, H, dmax - dmin + 1, need, (size_t)ST_NOALLOC_SCRATCH_BYTES);
  SETDEV(h);
  hipStream_t s = (hipStream_t)stream;
  uint32_t *keys = at<uint32_t>(base, koff);
  // the merged keys must start at zero whatever the last call left: cleared
  // by a kernel (no memset node if the caller captures the stream)
  HIPCK(launch_fill_u32(keys, (int)(2 * N), 0u, s));
  fill_views(Lo, base, keys, M, Pp, Q, left, right, pitch);
  Range whole("stereo_match_noalloc");
  rc = run_front(h, M, Pp, prec, s);
  if (rc) return rc;
  Q.disparity = disparity;
  Q.valid_mask = valid_mask;
  HIPCK(post_stages(single_launch(Q, s), *params, nullptr));
  return ST_OK;
}

st_status stereo_debug_get(st_handle h, const char *name, void **dev_ptr) {
  ARG(h && name && dev_ptr, "NULL argument");
  auto it = h->dbg.find(name);
  ARG(it != h->dbg.end(), "no debug buffer '%s' (run stereo_match with debug_outputs = 1)", name);
  *dev_ptr = it->second;
  return ST_OK;
}

// ---------------------------------------------------------------- single stages
st_status st_window_stats(st_handle h, const uint8_t *img, int H, int W, int pitch, int win,
                          int chess, int32_t *S, int32_t *SS, float *inv, void *stream) {
  ARG(win >= 3 && win <= 15 && (win & 1), "win must be odd and in [3, 15]");
  ARG(chess == 0 || chess == 1, "chess must be 0 or 1");
  ARG(H >= 1 && W >= 1 && pitch >= W, "bad image shape");
  ARG(img && S && SS && inv, "NULL pointer");
  ARG(h, "NULL handle");
  SETDEV(h);
  HIPCK(launch_window_stats_dense(img, H, W, pitch, win, chess, S, SS, inv, (hipStream_t)stream));
  return ST_OK;
}

st_status st_match_wta(st_handle h, const uint8_t *left, const uint8_t *right, int H, int W,
                       int pitch, int dmin, int dmax, int win, int chess, int precision,
                       int16_t *oL, uint8_t *mL, int16_t *oR, uint8_t *mR, void *stream) {
  st_status rc = check_shape(H, W, pitch, dmin, dmax, win);
  if (rc) return rc;
  ARG(chess == 0 || chess == 1, "chess must be 0 or 1");
  ARG(precision >= 0 && precision <= 2, "unknown precision %d", precision);
  ARG(left && right && oL && mL && oR && mR, "NULL pointer");
  ARG(h, "NULL handle");
  SETDEV(h);
  hipStream_t s = (hipStream_t)stream;
  const int v = pick_variant(h, H, W, win, dmin, dmax, precision);
  MatchPair M;
  PrepPair Pp;
  PostPair Q;
  PairLayout Lo;
  rc = setup_single(h, left, right, H, W, pitch, dmin, dmax, win, chess, precision, v, false, M, Pp,
                    Q, Lo, s);
  if (rc) return rc;
  rc = run_front(h, M, Pp, precision, s);
  if (rc) return rc;
  Q.ob[0] = oL;
  Q.mb[0] = mL;
  Q.oR = oR;
  Q.mR = mR;
  HIPCK(post_decode(single_launch(Q, s)));
  return ST_OK;
}

st_status st_subpixel(st_handle h, const uint8_t *left, const uint8_t *right, int H, int W,
                      int pitch, int dmin, int dmax, int win, int chess, const int16_t *oL,
                      const uint8_t *mL, double *zbest, double *zm, double *zp, float *delta,
                      void *stream) {
  st_status rc = check_shape(H, W, pitch, dmin, dmax, win);
  if (rc) return rc;
  ARG(chess == 0 || chess == 1, "chess must be 0 or 1");
  ARG(left && right && oL && mL && delta, "NULL pointer");
  ARG(h, "NULL handle");
  SETDEV(h);
  hipStream_t s = (hipStream_t)stream;
  const size_t N = (size_t)H * W;
  HIPCK(grow(h, h->ws, 16 * N + 1024, false) == ST_OK ? hipSuccess : hipErrorOutOfMemory);
  PostPair Q{};
  Q.left = left;
  Q.right = right;
  Q.H = H;
  Q.W = W;
  Q.pitch = pitch;
  Q.win = win;
  Q.chess = chess;
  Q.dmin = dmin;
  Q.dmax = dmax;
  int32_t *base = (int32_t *)h->ws.p;
  Q.SL = base;
  Q.SSL = base + N;
  Q.SR = base + 2 * N;
  Q.SSR = base + 3 * N;
  HIPCK(launch_window_stats_dense(left, H, W, pitch, win, chess, base, base + N, nullptr, s));
  HIPCK(launch_window_stats_dense(right, H, W, pitch, win, chess, base + 2 * N, base + 3 * N, nullptr, s));
  Q.ob[0] = const_cast<int16_t *>(oL);
  Q.mb[0] = const_cast<uint8_t *>(mL);
  Q.zbest = zbest;
  Q.zm = zm;
  Q.zp = zp;
  Q.delta = delta;
  HIPCK(post_subpixel(single_launch(Q, s)));
  return ST_OK;
}

st_status st_lr_check(st_handle h, const int16_t *oL, const uint8_t *mL, const int16_t *oR,
                      const uint8_t *mR, int H, int W, int tol, uint8_t *mask_out, void *stream) {
  ARG(H >= 1 && W >= 1 && tol >= 0, "bad shape or tolerance");
  ARG(oL && mL && oR && mR && mask_out, "NULL pointer");
  ARG(h, "NULL handle");
  SETDEV(h);
  const size_t N = (size_t)H * W;
  HIPCK(grow(h, h->ws, 2 * N + 256, false) == ST_OK ? hipSuccess : hipErrorOutOfMemory);
  PostPair Q{};
  Q.H = H;
  Q.W = W;
  Q.ob[0] = const_cast<int16_t *>(oL);
  Q.mb[0] = const_cast<uint8_t *>(mL);
  Q.oR = const_cast<int16_t *>(oR);
  Q.mR = const_cast<uint8_t *>(mR);
  Q.ob[1] = (int16_t *)h->ws.p;
  Q.mb[1] = mask_out;
  HIPCK(post_lr(single_launch(Q, (hipStream_t)stream), tol, 1));
  return ST_OK;
}

st_status st_radial_outlier(st_handle h, const int16_t *o, const uint8_t *m_in, int H, int W,
                            int r, float thresh, uint8_t *m_out, void *stream) {
  ARG(H >= 1 && W >= 1 && r >= 1 && r <= 4096, "bad shape or radius");
  ARG(o && m_in && m_out, "NULL pointer");
  ARG(m_out != m_in, "m_out aliases m_in");
  ARG(h, "NULL handle");
  SETDEV(h);
  const size_t N = (size_t)H * W;
  Carve c;
  const size_t ot = c.take(2 * N), it = c.take(2 * N), pt = c.take(4 * N), tot = c.take(0);
  HIPCK(grow(h, h->ws, tot, false) == ST_OK ? hipSuccess : hipErrorOutOfMemory);
  hipStream_t s = (hipStream_t)stream;
  // the scans read validity from the disparity: O_NONE where m_in == 0
  HIPCK(launch_mark_invalid(o, m_in, at<int16_t>(h->ws.p, it), N, s));
  PostPair Q{};
  Q.H = H;
  Q.W = W;
  Q.ob[1] = at<int16_t>(h->ws.p, it);
  Q.mb[1] = const_cast<uint8_t *>(m_in);
  Q.ob[2] = at<int16_t>(h->ws.p, ot);
  Q.pass = at<uint8_t>(h->ws.p, pt);
  Q.mb[2] = m_out;
  HIPCK(post_outlier(single_launch(Q, s), r, thresh, 1, 2));
  return ST_OK;
}

st_status st_fill(st_handle h, const int16_t *o_in, const uint8_t *m_in, int H, int W,
                  int radial_r, int min_lines, int disk_r, float min_frac, int16_t *o_out,
                  uint8_t *m_out, void *stream) {
  ARG(H >= 1 && W >= 1 && radial_r >= 0 && disk_r >= 0 && min_lines >= 1 && min_lines <= 4,
      "bad shape or fill parameters");
  ARG(min_frac >= 0.0f && min_frac <= 1.0f, "min_frac not in [0, 1]");
  ARG(o_in && m_in && o_out && m_out, "NULL pointer");
  ARG((const void *)o_out != (const void *)o_in && (const void *)m_out != (const void *)m_in,
      "outputs alias inputs");
  ARG(h, "NULL handle");
  SETDEV(h);
  const size_t N = (size_t)H * W;
  Carve c;
  const size_t ot = c.take(2 * N), mt = c.take(N), pc = c.take(4 * (size_t)H * (W + 1)),
               ps = c.take(4 * (size_t)H * (W + 1)), ht = c.take(32 * N), it = c.take(2 * N),
               tot = c.take(0);
  HIPCK(grow(h, h->ws, tot, false) == ST_OK ? hipSuccess : hipErrorOutOfMemory);
  hipStream_t s = (hipStream_t)stream;
  // the scans read validity from the disparity: O_NONE where m_in == 0
  HIPCK(launch_mark_invalid(o_in, m_in, at<int16_t>(h->ws.p, it), N, s));
  PostPair Q{};
  Q.H = H;
  Q.W = W;
  Q.ob[0] = at<int16_t>(h->ws.p, it);
  Q.mb[0] = const_cast<uint8_t *>(m_in);
  Q.ob[1] = at<int16_t>(h->ws.p, ot);
  Q.mb[1] = at<uint8_t>(h->ws.p, mt);
  Q.ob[2] = o_out;
  Q.mb[2] = m_out;
  Q.pc = at<int32_t>(h->ws.p, pc);
  Q.ps = at<int32_t>(h->ws.p, ps);
  Q.hits = at<uint32_t>(h->ws.p, ht);
  HIPCK(post_fill(single_launch(Q, s), radial_r, min_lines, disk_r, min_frac, 0, 1, 2));
  return ST_OK;
}

st_status st_research(st_handle h, const uint8_t *left, const uint8_t *right, int H, int W,
                      int pitch, int dmin, int dmax, int win, int chess, const int16_t *o_in,
                      const uint8_t *m, const double *d, int range, float eta, int16_t *o_out,
                      void *stream) {
  st_status rc = check_shape(H, W, pitch, dmin, dmax, win);
  if (rc) return rc;
  ARG(chess == 0 || chess == 1, "chess must be 0 or 1");
  ARG(range >= 0 && range <= 64 && eta >= 0.0f, "bad range or eta");
  ARG(left && right && o_in && m && d && o_out, "NULL pointer");
  ARG((const void *)o_in != (const void *)o_out, "o_out aliases o_in");
  ARG(h, "NULL handle");
  SETDEV(h);
  hipStream_t s = (hipStream_t)stream;
  const size_t N = (size_t)H * W;
  HIPCK(grow(h, h->ws, 16 * N + 1024, false) == ST_OK ? hipSuccess : hipErrorOutOfMemory);
  PostPair Q{};
  Q.left = left;
  Q.right = right;
  Q.H = H;
  Q.W = W;
  Q.pitch = pitch;
  Q.win = win;
  Q.chess = chess;
  Q.dmin = dmin;
  Q.dmax = dmax;
  int32_t *base = (int32_t *)h->ws.p;
  Q.SL = base;
  Q.SSL = base + N;
  Q.SR = base + 2 * N;
  Q.SSR = base + 3 * N;
  HIPCK(launch_window_stats_dense(left, H, W, pitch, win, chess, base, base + N, nullptr, s));
  HIPCK(launch_window_stats_dense(right, H, W, pitch, win, chess, base + 2 * N, base + 3 * N, nullptr, s));
  Q.ob[0] = const_cast<int16_t *>(o_in);
  Q.mb[0] = const_cast<uint8_t *>(m);
  Q.ob[1] = o_out;
  Q.f = const_cast<double *>(d);
  HIPCK(post_research(single_launch(Q, s), 0, 0, 1, 0, range, eta));
  return ST_OK;
}

st_status st_reproject(st_handle h, const float *disparity, int H, int W, const double *Q,
                       float *xyz, void *stream) {
  ARG(H >= 1 && W >= 1 && (long long)H * W <= (1LL << 28), "bad shape");
  ARG(disparity && Q && xyz, "NULL pointer");
  ARG(h, "NULL handle");
  SETDEV(h);
  Mat4 M;
  for (int i = 0; i < 16; ++i) M.q[i] = Q[i];
  HIPCK(launch_reproject(disparity, H, W, M, xyz, (hipStream_t)stream));
  return ST_OK;
}

st_status st_hc_smooth(st_handle h, const float *s_in, const uint8_t *m, int H, int W, int R,
                       int K, float alpha, float *out, void *stream) {
  ARG(H >= 1 && W >= 1 && R >= 0 && R <= 2048 && K >= 0 && K <= 64, "bad shape or parameters");
  ARG(s_in && m && out, "NULL pointer");
  ARG(h, "NULL handle");
  SETDEV(h);
  const size_t N = (size_t)H * W;
  HIPCK(grow(h, h->ws, 6 * 8 * N + 256, false) == ST_OK ? hipSuccess : hipErrorOutOfMemory);
  PostPair Q{};
  Q.H = H;
  Q.W = W;
  Q.mb[0] = const_cast<uint8_t *>(m);
  Q.s_in = s_in;
  Q.f = (double *)h->ws.p;
  Q.disparity = out;
  Q.valid_mask = nullptr;
  HIPCK(post_hc(single_launch(Q, (hipStream_t)stream), 0, R, K, alpha, 0, 0, 0, 0.0f));
  return ST_OK;
}

// ---------------------------------------------------------------- batched
// Tuning-table key of the persistent launch of one window size of a batch:
// window, precision, window shape and the size and range of each of that
// window's pairs in order (64-bit FNV-1a).
static std::string batch_key(const st_pair *pairs, int n, int win, int prec, int chess) {
  uint64_t x = 1469598103934665603ull;
  auto mix = [&](int v) {
    for (int b = 0; b < 4; ++b) {
      x ^= (uint8_t)((uint32_t)v >> (8 * b));
      x *= 1099511628211ull;
    }
  };
  for (int i = 0; i < n; ++i)
    if (pairs[i].win == win) {
      mix(pairs[i].H);
      mix(pairs[i].W);
      mix(pairs[i].dmin);
      mix(pairs[i].dmax);
    }
  char b[96];
  snprintf(b, sizeof b, "b_w%d_p%d_c%d_%016llx", win, prec, chess, (unsigned long long)x);
  return b;
}

// The persistent matcher launches of the current batch on stream s, one per
// window size: the first on s, the others one after another on the side
// stream, forked from s after the work already on it and joined back into
// it, so that each launch's workgroups take the CUs that the launch beside
// it frees at its tail.  ev0 / ev1 (may be null) bracket all of them on s.
static hipError_t launch_groups(st_handle h, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  BatchCache &B = h->batch;
  hipError_t e = hipSuccess;
  auto ck = [&](hipError_t x) {
    if (x != hipSuccess && e == hipSuccess) e = x;
  };
  if (ev0) ck(hipEventRecord(ev0, s));
  if (B.groups.size() > 1) {
    ck(hipEventRecord(h->fork_ev, s));
    ck(hipStreamWaitEvent(h->side_stream, h->fork_ev, 0));
  }
  for (size_t gi = 0; gi < B.groups.size(); ++gi) {
    const BatchCache::Group &g = B.groups[gi];
    ck(launch_match_persistent(B.tM, B.tT + g.off, g.ntasks, B.tC + gi, g.win, g.dc, B.prec,
                               g.nblocks, g.lds, gi == 0 ? s : h->side_stream, nullptr, nullptr));
  }
  if (B.groups.size() > 1) {
    ck(hipEventRecord(h->join_ev, h->side_stream));
    ck(hipStreamWaitEvent(s, h->join_ev, 0));
  }
  if (ev1) ck(hipEventRecord(ev1, s));
  return e;
}

st_status stereo_match_batched(st_handle h, const st_pair *pairs, int n_pairs,
                               const st_params *params, void *stream) {
  ARG(pairs && n_pairs >= 1 && n_pairs <= 65535, "bad pair list");
  st_status rc = check_params(params);
  if (rc) return rc;
  for (int i = 0; i < n_pairs; ++i) {
    const st_pair &q = pairs[i];
    rc = check_shape(q.H, q.W, q.pitch, q.dmin, q.dmax, q.win);
    if (rc) {
      const std::string why = g_err;
      return fail(rc, "pair %d: %s", i, why.c_str());
    }
    ARG(q.left && q.right && q.disparity && q.valid_mask, "pair %d: NULL pointer", i);
  }
  ARG(h, "NULL handle");
  SETDEV(h);
  hipStream_t s = (hipStream_t)stream;
  const int prec = params->precision;
  BatchCache &B = h->batch;
  const int vforce = h->variant;
  bool same = B.exec && (int)B.pairs.size() == n_pairs && B.variant == vforce &&
              B.tune_gen == h->tune_gen &&
              memcmp(&B.params, params, sizeof(st_params)) == 0 &&
              memcmp(B.pairs.data(), pairs, sizeof(st_pair) * n_pairs) == 0;
  if (same) {
    Range r("stereo_match_batched: graph replay");
    HIPCK(hipGraphLaunch(B.exec, s));
    return ST_OK;
  }
  Range build("stereo_match_batched: layout, tables, capture");
  // a replay of the previous layout may still be queued (on this or another
  // stream): its graph and the device tables it reads are replaced below
  HIPCK(hipDeviceSynchronize());
  drop_batch(B);
  // the matcher variant of each window size: forced, tuned for this batch
  // layout, or the first in preference order
  std::map<int, int> wvar;
  for (int i = 0; i < n_pairs; ++i) {
    const int w = pairs[i].win;
    if (wvar.count(w)) continue;
    int v = vforce >= 0 ? vforce : 0;
    if (vforce < 0) {
      auto it = h->tune.find(batch_key(pairs, n_pairs, w, prec, params->chessboard));
      if (it != h->tune.end()) v = it->second;
    }
    wvar[w] = v;
  }
  std::vector<MatchPair> M(n_pairs);
  std::vector<PrepPair> Pp(n_pairs);
  std::vector<PostPair> Q(n_pairs);
  std::vector<PairLayout> Lo(n_pairs);
  std::vector<size_t> base(n_pairs), kbase(n_pairs);
  size_t total = 0, ktotal = 0;
  int maxH = 0, maxW = 0, maxCols = 0;
  for (int i = 0; i < n_pairs; ++i) {
    const st_pair &q = pairs[i];
    const int v = wvar[q.win];
    make_geom(M[i], q.H, q.W, q.win, q.dmin, q.dmax, variant_DC(v), variant_TY(v), variant_CG(v),
              params->chessboard);
    Lo[i] = layout(M[i], prec, false);
    total = (total + 255) & ~(size_t)255;
    base[i] = total;
    total += Lo[i].total;
    kbase[i] = ktotal;
    ktotal += 2 * (size_t)q.H * q.W;
    maxH = std::max(maxH, q.H);
    maxW = std::max(maxW, q.W);
    maxCols = std::max(maxCols, std::max(M[i].strideL, M[i].strideR));
  }
  rc = grow(h, B.ws, total, false);
  if (rc) return rc;
  rc = grow(h, B.keys, 4 * ktotal, true);
  if (rc) return rc;
  // task queues, one per window size: (pair, group, chunk group), longest
  // first; the cost counts rows evaluated plus vertical-sum restarts
  std::map<int, std::vector<std::pair<int, int4>>> byw;
  std::map<int, long long> wcost;
  std::map<int, size_t> wlds;
  for (int i = 0; i < n_pairs; ++i) {
    const MatchPair &P = M[i];
    const int hh = P.win / 2;
    wlds[P.win] = std::max(wlds[P.win], match_lds_bytes(P));
    for (int g = 0; g < P.nband * P.nspan; ++g) {
      const int band = g / P.nspan;
      const int rows = std::min(P.TY, P.H - hh - (hh + band * P.TY));
      for (int c = 0; c < P.ncg; ++c) {
        const int nc = std::min(P.CG, P.nchunk - c * P.CG);
        const int cost = nc * (rows + 2 * hh);
        byw[P.win].push_back({cost, make_int4(i, g, c, 0)});
        wcost[P.win] += cost;
      }
    }
  }
  std::vector<int> wins;
  for (auto &kv : byw) wins.push_back(kv.first);
  std::sort(wins.begin(), wins.end(), [&](int a, int b) { return wcost[a] > wcost[b]; });
  std::vector<int4> sorted;
  std::vector<BatchCache::Group> groups;
  for (int w : wins) {
    auto &v = byw[w];
    std::stable_sort(v.begin(), v.end(), [](const std::pair<int, int4> &a,
                                            const std::pair<int, int4> &b) { return a.first > b.first; });
    BatchCache::Group gr;
    gr.win = w;
    gr.variant = wvar[w];
    gr.dc = variant_DC(gr.variant);
    gr.off = (int)sorted.size();
    gr.lds = wlds[w];
    gr.nblocks = h->ncu * match_persistent_occupancy(w, gr.dc, prec, gr.lds);
    // the queue's last round: its tasks (the cheapest, at the end) go in
    // two halves of their band's rows, so that the workgroups run out of
    // work at most half a task apart (tk.w = first row | end row << 16)
    const int nsplit = std::min((int)v.size(), gr.nblocks);
    const int nfull = (int)v.size() - nsplit;
    for (int i = 0; i < nfull; ++i) sorted.push_back(v[i].second);
    for (int i = nfull; i < (int)v.size(); ++i) {
      const int4 tk = v[i].second;
      const MatchPair &P = M[tk.x];
      const int hh = P.win / 2, band = tk.y / P.nspan;
      const int rows = std::min(P.TY, P.H - 2 * hh - band * P.TY);
      if (rows < 2) {
        sorted.push_back(tk);
        continue;
      }
      const int mid = rows / 2;
      sorted.push_back(make_int4(tk.x, tk.y, tk.z, mid << 16));
      sorted.push_back(make_int4(tk.x, tk.y, tk.z, mid | (rows << 16)));
    }
    gr.ntasks = (int)sorted.size() - gr.off;
    groups.push_back(gr);
  }
  // device tables
  Carve c;
  const size_t tM = c.take(sizeof(MatchPair) * n_pairs), tP = c.take(sizeof(PrepPair) * n_pairs),
               tQ = c.take(sizeof(PostPair) * n_pairs), tT = c.take(sizeof(int4) * sorted.size()),
               tC = c.take(4 * groups.size() + 16), tTot = c.take(0);
  rc = grow(h, B.tables, tTot, false);
  if (rc) return rc;
  for (int i = 0; i < n_pairs; ++i) {
    fill_views(Lo[i], at<void>(B.ws.p, base[i]), (uint32_t *)B.keys.p + kbase[i], M[i], Pp[i], Q[i],
               pairs[i].left, pairs[i].right, pairs[i].pitch);
    Q[i].disparity = pairs[i].disparity;
    Q[i].valid_mask = pairs[i].valid_mask;
  }
  HIPCK(hipMemcpy(at<void>(B.tables.p, tM), M.data(), sizeof(MatchPair) * n_pairs, hipMemcpyHostToDevice));
  HIPCK(hipMemcpy(at<void>(B.tables.p, tP), Pp.data(), sizeof(PrepPair) * n_pairs, hipMemcpyHostToDevice));
  // post-processing by image size: the pairs of one size are consecutive in
  // the table and run each stage as one launch whose grid fits that size
  // (one grid for the largest pair would leave most blocks of a small pair
  // empty); sizes by pixel count, largest first
  std::map<std::pair<int, int>, std::vector<int>> byshape;
  for (int i = 0; i < n_pairs; ++i) byshape[{pairs[i].H, pairs[i].W}].push_back(i);
  // a size with many pairs is cut in two halves on two streams, so that the
  // tail of one half's launch overlaps the other's (each stage is a chain
  // of short launches whose last blocks leave most of the chip idle)
  std::vector<std::vector<int>> shapes;
  for (auto &kv : byshape) {
    const size_t n = kv.second.size(), cut = n >= 8 ? n / 2 : n;
    shapes.emplace_back(kv.second.begin(), kv.second.begin() + cut);
    if (cut < n) shapes.emplace_back(kv.second.begin() + cut, kv.second.end());
  }
  std::stable_sort(shapes.begin(), shapes.end(), [&](const std::vector<int> &a, const std::vector<int> &b) {
    return (long long)pairs[a[0]].H * pairs[a[0]].W > (long long)pairs[b[0]].H * pairs[b[0]].W;
  });
  std::vector<PostPair> Qs;
  for (auto &g : shapes)
    for (int i : g) Qs.push_back(Q[i]);
  HIPCK(hipMemcpy(at<void>(B.tables.p, tQ), Qs.data(), sizeof(PostPair) * n_pairs, hipMemcpyHostToDevice));
  // streams for the groups after the first (at most kPostStreams, shared
  // round robin beyond that)
  constexpr int kPostStreams = 7;
  const int nps = std::min((int)shapes.size() - 1, kPostStreams);
  while ((int)h->post_streams.size() < nps) {
    hipStream_t ps = nullptr;
    hipEvent_t pe = nullptr;
    HIPCK(hipStreamCreateWithFlags(&ps, hipStreamNonBlocking));
    if (hipEventCreateWithFlags(&pe, hipEventDisableTiming) != hipSuccess) {
      (void)hipStreamDestroy(ps);
      return fail(ST_EHIP, "cannot create a post-processing event");
    }
    h->post_streams.push_back(ps);
    h->post_done.push_back(pe);
  }
  HIPCK(hipMemcpy(at<void>(B.tables.p, tT), sorted.data(), sizeof(int4) * sorted.size(), hipMemcpyHostToDevice));
  // resident waves of the persistent matcher
  // capture the whole sequence once, replay it on later calls
  hipStream_t cs = h->cap_stream;
  HIPCK(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
  hipError_t e = hipSuccess;
  auto ck = [&](hipError_t x) { if (x != hipSuccess && e == hipSuccess) e = x; };
  // the window statistics on the side stream beside the plane preparation
  // (disjoint parts of the planes), joined before the matcher
  ck(hipEventRecord(h->prep_fork, cs));
  ck(hipStreamWaitEvent(h->side_stream, h->prep_fork, 0));
  ck(launch_prep(Pp[0], at<PrepPair>(B.tables.p, tP), n_pairs, maxH, maxCols, maxW, prec, cs,
                 h->side_stream));
  ck(hipEventRecord(h->prep_join, h->side_stream));
  ck(hipStreamWaitEvent(cs, h->prep_join, 0));
  B.tM = at<MatchPair>(B.tables.p, tM);
  B.tT = at<int4>(B.tables.p, tT);
  B.tC = at<int>(B.tables.p, tC);
  B.groups = groups;
  B.prec = prec;
  ck(launch_groups(h, cs, nullptr, nullptr));
  // the post-processing of each group; groups after the first on streams
  // forked after the matcher and joined back at the end
  if (nps > 0) {
    ck(hipEventRecord(h->post_fork, cs));
    for (int k = 0; k < nps; ++k) ck(hipStreamWaitEvent(h->post_streams[k], h->post_fork, 0));
  }
  int first = 0;
  for (size_t g = 0; g < shapes.size(); ++g) {
    const std::vector<int> &ids = shapes[g];
    PostLaunch L;
    L.one = Qs[first];
    L.many = at<PostPair>(B.tables.p, tQ) + first;
    L.npairs = (int)ids.size();
    L.maxH = pairs[ids[0]].H;
    L.maxW = pairs[ids[0]].W;
    L.maxWin = 0;
    L.maxD = 0;
    for (int i : ids) {
      L.maxWin = std::max(L.maxWin, Q[i].win);
      L.maxD = std::max(L.maxD, Q[i].dmax - Q[i].dmin + 1);
    }
    L.s = g == 0 ? cs : h->post_streams[(g - 1) % kPostStreams];
    ck(post_stages(L, *params, nullptr));
    first += (int)ids.size();
  }
  for (int k = 0; k < nps; ++k) {
    ck(hipEventRecord(h->post_done[k], h->post_streams[k]));
    ck(hipStreamWaitEvent(cs, h->post_done[k], 0));
  }
  hipGraph_t g = nullptr;
  hipError_t ee = hipStreamEndCapture(cs, &g);
  if (e != hipSuccess || ee != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    h->keys_dirty = true;
    return fail(ST_EHIP, "capture of the batched launch failed: %s",
                hipGetErrorString(e != hipSuccess ? e : ee));
  }
  hipGraphExec_t ex = nullptr;
  if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(ST_EHIP, "hipGraphInstantiate failed");
  }
  B.graph = g;
  B.exec = ex;
  B.pairs.assign(pairs, pairs + n_pairs);
  B.params = *params;
  B.variant = vforce;
  B.tune_gen = h->tune_gen;
  HIPCK(hipGraphLaunch(B.exec, s));
  return ST_OK;
}

// Mean ms of each window size's persistent launch alone (reps launches each,
// HIP events on s); the batch must have been built and run.
static hipError_t time_each_group(st_handle h, int reps, hipStream_t s, std::vector<double> &ms) {
  BatchCache &B = h->batch;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  ms.assign(B.groups.size(), 0.0);
  for (size_t gi = 0; gi < B.groups.size() && e == hipSuccess; ++gi) {
    const BatchCache::Group &g = B.groups[gi];
    for (int r = 0; r < reps && e == hipSuccess; ++r) {
      e = launch_match_persistent(B.tM, B.tT + g.off, g.ntasks, B.tC + gi, g.win, g.dc, B.prec,
                                  g.nblocks, g.lds, s, e0, e1);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float t = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
      ms[gi] += t / reps;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return e;
}

st_status stereo_time_matcher(st_handle h, const st_pair *pairs, int n_pairs,
                              const st_params *params, int reps, float *ms_out, void *stream) {
  ARG(ms_out && reps >= 1 && reps <= 100000, "bad reps or NULL output");
  ARG(h, "NULL handle");
  // (re)build the batch if needed and run it once: prepares every plane
  st_status rc = stereo_match_batched(h, pairs, n_pairs, params, stream);
  if (rc) return rc;
  BatchCache &B = h->batch;
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  HIPCK(hipEventCreate(&e0));
  HIPCK(hipEventCreate(&e1));
  double total = 0.0;
  hipError_t e = hipSuccess;
  // the matcher phase as the graph runs it: every window size's launch,
  // side by side, between two events on the stream
  for (int r = 0; r < reps && e == hipSuccess; ++r) {
    e = launch_groups(h, s, e0, e1);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    total += ms;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIPCK(e);
  // the keys now hold the merged maxima again; the next decode clears them,
  // so replay the batch once to leave every output consistent
  HIPCK(hipGraphLaunch(B.exec, s));
  *ms_out = (float)(total / reps);
  return ST_OK;
}

st_status st_autotune_batched(st_handle h, const st_pair *pairs, int n_pairs,
                              const st_params *params, int reps, int *best_cfg, void *stream) {
  ARG(h, "NULL handle");
  ARG(reps >= 1 && reps <= 1000, "reps must be in [1, 1000]");
  ARG(pairs && n_pairs >= 1, "bad pair list");
  hipStream_t s = (hipStream_t)stream;
  const int saved = h->variant;
  std::map<int, std::pair<double, int>> best;  // window -> (ms, variant)
  st_status rc = ST_OK;
  for (int v = 0; v < kNumVariants && rc == ST_OK; ++v) {
    h->variant = v;
    rc = stereo_match_batched(h, pairs, n_pairs, params, stream);  // builds and runs it
    if (rc) break;
    std::vector<double> ms;
    const hipError_t e = time_each_group(h, reps, s, ms);
    if (e != hipSuccess) {
      rc = fail(ST_EHIP, "timing the persistent launches failed: %s", hipGetErrorString(e));
      break;
    }
    const BatchCache &B = h->batch;
    for (size_t gi = 0; gi < B.groups.size(); ++gi) {
      auto it = best.find(B.groups[gi].win);
      if (it == best.end() || ms[gi] < it->second.first) best[B.groups[gi].win] = {ms[gi], v};
    }
  }
  h->variant = saved;
  if (rc) {
    h->keys_dirty = true;
    drop_batch(h->batch);
    return rc;
  }
  const int prec = params->precision;
  for (auto &kv : best) h->tune[batch_key(pairs, n_pairs, kv.first, prec, params->chessboard)] = kv.second.second;
  ++h->tune_gen;
  save_tune(h);
  if (best_cfg)
    for (int i = 0; i < n_pairs; ++i) best_cfg[i] = best[pairs[i].win].second;
  // rebuild with the tuned variants; the outputs come from them
  return stereo_match_batched(h, pairs, n_pairs, params, stream);
}

int st_batch_variant(st_handle h, int win) {
  if (!h || !h->batch.exec) return -1;
  for (const BatchCache::Group &g : h->batch.groups)
    if (g.win == win) return g.variant;
  return -1;
}

// ---------------------------------------------------------------- refinement
static st_status refine_setup(st_handle h, const uint8_t *left, const uint8_t *right,
                              const float *d, const uint8_t *mask, int H, int W, int pitch,
                              int win, float lambda_tv, RefineArgs &A) {
  ARG(win >= 3 && win <= 15 && (win & 1), "win must be odd and in [3, 15]");
  ARG(H >= win && W >= win && pitch >= W && (long long)H * W <= (1LL << 26), "bad image shape");
  ARG(left && right && d && mask, "NULL pointer");
  ARG(lambda_tv >= 0.0f, "lambda_tv < 0");
  ARG(h, "NULL handle");
  SETDEV(h);
  const size_t N = (size_t)H * W;
  const size_t need = (size_t)refine_planes() * 8 * N + 8 * (size_t)refine_partials(H, W) + 512;
  st_status rc = grow(h, h->rws, need, false);
  if (rc) return rc;
  A = RefineArgs{};
  A.L = left;
  A.R = right;
  A.d = d;
  A.mask = mask;
  A.H = H;
  A.W = W;
  A.pitch = pitch;
  A.win = win;
  A.lambda = lambda_tv;
  A.f = (double *)h->rws.p;
  A.partial = A.f + (size_t)refine_planes() * N;
  return ST_OK;
}

st_status stereo_refine_forward(st_handle h, const uint8_t *left, const uint8_t *right,
                                const float *d, const uint8_t *mask, int H, int W, int pitch,
                                int win, float lambda_tv, float *Z, double *E, void *stream) {
  ARG(E, "E is NULL");
  RefineArgs A;
  st_status rc = refine_setup(h, left, right, d, mask, H, W, pitch, win, lambda_tv, A);
  if (rc) return rc;
  A.Z = Z;
  A.E = E;
  Range r("stereo_refine_forward");
  HIPCK(launch_refine_forward(A, (hipStream_t)stream));
  return ST_OK;
}

st_status stereo_refine_backward(st_handle h, const uint8_t *left, const uint8_t *right,
                                 const float *d, const uint8_t *mask, int H, int W, int pitch,
                                 int win, float lambda_tv, float *grad_d, void *stream) {
  ARG(grad_d, "grad_d is NULL");
  RefineArgs A;
  st_status rc = refine_setup(h, left, right, d, mask, H, W, pitch, win, lambda_tv, A);
  if (rc) return rc;
  A.grad = grad_d;
  Range r("stereo_refine_backward");
  HIPCK(launch_refine_backward(A, (hipStream_t)stream));
  return ST_OK;
}

st_status stereo_refine_step(st_handle h, float *d, const float *grad_d, const uint8_t *mask,
                             int H, int W, float tau, float max_step, void *stream) {
  ARG(d && grad_d && mask, "NULL pointer");
  ARG(H >= 1 && W >= 1 && (long long)H * W <= (1LL << 28), "bad shape");
  ARG(tau >= 0.0f && max_step >= 0.0f, "negative step parameters");
  ARG(h, "NULL handle");
  SETDEV(h);
  HIPCK(launch_refine_step(d, grad_d, mask, H * W, tau, max_step, (hipStream_t)stream));
  return ST_OK;
}

// ---------------------------------------------------------------- tuning
st_status st_set_variant(st_handle h, int variant) {
  ARG(h, "NULL handle");
  ARG(variant >= -1 && variant < kNumVariants, "variant %d out of range", variant);
  h->variant = variant;
  return ST_OK;
}

}  // extern "C"

static std::string tune_key(int H, int W, int win, int dmin, int dmax, int prec) {
  (void)H;
  const int D = dmax - dmin + 1;
  char b[96];
  snprintf(b, sizeof b, "w%d_D%d_W%d_p%d", win, round_up(D, 32), round_up(W, 256), prec);
  return b;
}

// Variant used when nothing is forced: the tuned one for this shape bucket,
// else the first in preference order that gives every CU two workgroups.
static int pick_variant(st_handle h, int H, int W, int win, int dmin, int dmax, int prec) {
  if (h->variant >= 0) return h->variant;
  auto it = h->tune.find(tune_key(H, W, win, dmin, dmax, prec));
  if (it != h->tune.end()) return it->second;
  int best = 0;
  long long best_n = -1;
  for (int v = 0; v < kNumVariants; ++v) {
    MatchPair P;
    make_geom(P, H, W, win, dmin, dmax, variant_DC(v), variant_TY(v), variant_CG(v), 0);
    const long long n = (long long)P.nspan * P.nband * P.ncg;
    if (n >= 2LL * h->ncu) return v;
    if (n > best_n) {
      best_n = n;
      best = v;
    }
  }
  return best;
}

static void save_tune(st_handle h) {
  const char *path = getenv("STEREO_TUNE_CACHE");
  if (!path || !*path) return;
  std::ofstream f(path);
  if (!f) return;
  f << "{\n";
  size_t i = 0;
  for (auto &kv : h->tune) {
    f << "  \"" << kv.first << "\": " << kv.second << (++i < h->tune.size() ? "," : "") << "\n";
  }
  f << "}\n";
}

// Reads the flat {"key": int, ...} object written by save_tune.
static void load_tune(st_handle h) {
  const char *path = getenv("STEREO_TUNE_CACHE");
  if (!path || !*path) return;
  std::ifstream f(path);
  if (!f) return;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  size_t p = 0;
  while ((p = s.find('"', p)) != std::string::npos) {
    const size_t q = s.find('"', p + 1);
    if (q == std::string::npos) break;
    const std::string key = s.substr(p + 1, q - p - 1);
    const size_t colon = s.find(':', q);
    if (colon == std::string::npos) break;
    const int v = atoi(s.c_str() + colon + 1);
    if (v >= 0 && v < kNumVariants) h->tune[key] = v;
    p = colon + 1;
  }
}

extern "C" st_status st_autotune(st_handle h, int H, int W, int dmin, int dmax, int win,
                                 int precision, int *best_cfg, void *stream) {
  st_status rc = check_shape(H, W, W, dmin, dmax, win);
  if (rc) return rc;
  ARG(precision >= 0 && precision <= 2, "unknown precision");
  ARG(h, "NULL handle");
  SETDEV(h);
  hipStream_t s = (hipStream_t)stream;
  // seeded test pattern: a smooth texture and its shift by a quarter range
  const size_t N = (size_t)H * W;
  std::vector<uint8_t> img(2 * N);
  uint32_t st = 12345u;
  for (size_t i = 0; i < N; ++i) {
    st = st * 1664525u + 1013904223u;
    img[i] = (uint8_t)(st >> 24);
  }
  const int shift = (dmin + dmax) / 2;
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      const int xs = std::min(std::max(x + shift, 0), W - 1);
      img[N + (size_t)y * W + x] = img[(size_t)y * W + xs];
    }
  uint8_t *dimg = nullptr;
  HIPCK(hipMalloc(&dimg, 2 * N));
  hipError_t e = hipMemcpy(dimg, img.data(), 2 * N, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(dimg);
    HIPCK(e);
  }
  int best = -1;
  double best_ms = 1e30;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  auto ck = [&](hipError_t x) {
    if (x != hipSuccess && e == hipSuccess) e = x;
  };
  for (int v = 0; v < kNumVariants && e == hipSuccess; ++v) {
    MatchPair M;
    PrepPair Pp;
    PostPair Q;
    PairLayout Lo;
    rc = setup_single(h, dimg, dimg + N, H, W, W, dmin, dmax, win, 0, precision, v, false, M, Pp,
                      Q, Lo, s);
    if (rc) break;
    ck(launch_prep(Pp, nullptr, 1, H, std::max(M.strideL, M.strideR), W, precision, s));
    PostLaunch L = single_launch(Q, s);
    double ms_min = 1e30;
    for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {
      ck(hipEventRecord(e0, s));
      ck(launch_match(M, precision, s));
      ck(hipEventRecord(e1, s));
      ck(post_decode(L));
      ck(hipEventSynchronize(e1));
      float ms = 0;
      ck(hipEventElapsedTime(&ms, e0, e1));
      if (rep > 0) ms_min = std::min(ms_min, (double)ms);
    }
    if (ms_min < best_ms) {
      best_ms = ms_min;
      best = v;
    }
  }
  ck(hipStreamSynchronize(s));
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(dimg);
  if (rc) return rc;
  HIPCK(e);
  if (best < 0) return fail(ST_EUNSUPPORTED, "no matcher variant fits this shape");
  h->tune[tune_key(H, W, win, dmin, dmax, precision)] = best;
  ++h->tune_gen;
  save_tune(h);
  if (best_cfg) *best_cfg = best;
  return ST_OK;
}
