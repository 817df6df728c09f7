/*
 * stereo.h - C ABI of the MI355X dense ZNCC stereo library (libstereo_mi355x.so).
 *
 * Method: Zhou & Jagadeesan, "Real-time Dense Reconstruction of Tissue
 * Surface from Stereo Optical Video" (arXiv 2007.12623), Section II:
 * ZNCC local matching over a square window for every pixel and candidate
 * disparity (II-A), winner-take-all, outlier removal and hole filling
 * (II-B), improved Laplacian smoothing (II-C, Eqs. 1-3).  On top: a
 * parabola sub-pixel offset, a left-right consistency check, a batched
 * persistent launch, FP16/BF16 storage and a differentiable refinement.
 *
 * Conventions shared by every entry point
 *  - Images are rectified 8-bit grey levels, row-major with a row pitch in
 *    bytes (pitch >= W).  Left pixel (x, y) at disparity d matches right
 *    pixel (x - d, y); d may be negative.  A window of odd size win lies
 *    around each pixel (half size h = win / 2).
 *  - Unless stated otherwise every data pointer is a DEVICE pointer owned by
 *    the caller; outputs are written densely (row stride W elements).
 *    Host pointers are marked "host".
 *  - Work is enqueued on `stream` (a hipStream_t passed as void*, NULL = the
 *    default stream) and the call returns without synchronising; results are
 *    valid once the stream has reached that point.
 *  - Arguments are checked on the host before any device call; invalid ones
 *    return ST_EINVAL and touch nothing.  Launch failures return ST_EHIP.
 *    st_last_error() describes the last failure of the calling thread.
 *  - A handle owns its scratch memory (grown on demand, ST_ENOMEM if it
 *    cannot grow).  Calls on one handle must not run concurrently from
 *    several host threads or overlap on several streams.
 */
#ifndef STEREO_MI355X_H
#define STEREO_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ST_OK = 0,
  ST_EINVAL = -1,       /* bad argument (checked before any device work) */
  ST_ENOMEM = -2,       /* device scratch could not be allocated */
  ST_EHIP = -3,         /* a HIP runtime call or kernel launch failed */
  ST_ENODEV = -4,       /* no usable gfx950 device */
  ST_EUNSUPPORTED = -5  /* valid request the library does not implement */
} st_status;

typedef enum { ST_FP32 = 0, ST_FP16 = 1, ST_BF16 = 2 } st_precision;

typedef struct st_handle_s *st_handle;

/* Pipeline parameters.  st_default_params() fills the paper's constants. */
typedef struct {
  int32_t struct_size;        /* sizeof(st_params): ABI guard */
  int32_t subpixel;           /* 1: parabola offset added to matched pixels */
  int32_t lr_check;           /* 1: left-right consistency check */
  int32_t lr_tol;             /* max |oL - oR| kept (1 px) */
  int32_t radial_iters;       /* outlier/fill alternations (3, Section II-B);
                                 0 = a single fill pass, no outlier removal */
  int32_t radial_r0;          /* first outlier radius (10 px) */
  int32_t radial_dr;          /* radius step per alternation (10 px) */
  float radial_thresh;        /* neighbour disparity step bound (2.5) */
  int32_t fill_radial_r;      /* radial fill search radius (50 px) */
  int32_t fill_min_lines;     /* complete lines needed by the radial fill (2) */
  int32_t fill_disk_r;        /* disk fill radius (20 px) */
  float fill_disk_min_frac;   /* valid fraction of in-image disk cells (0.25) */
  int32_t smooth_radius;      /* half size R of the (2R+1)^2 smoothing window (15) */
  int32_t smooth_iters;       /* improved Laplacian iterations K (3; 0 = none) */
  float smooth_alpha;         /* Eq. (2) weight (0.1) */
  int32_t precision;          /* st_precision of image and cost storage */
  int32_t debug_outputs;      /* 1: keep intermediates for stereo_debug_get */
  int32_t research;           /* 1: Eq. (4) - the discrete disparities o are
                                 re-searched around d in every smoothing
                                 iteration and Eqs. (1)-(2) use o (Section
                                 II-C); 0: smoothing of s = o + delta */
  int32_t research_range;     /* half width of the re-search window (5) */
  float research_eta;         /* weight of (o* - d)^2 in Eq. (4) (0.01) */
  int32_t chessboard;         /* 1: the chessboard window of Section II-A - only
                                 the cells (u, v) around the centre with u + v
                                 even (61 of 121 at 11x11) enter every ZNCC,
                                 in matching, sub-pixel fit and re-search;
                                 0: the full square window (default) */
} st_params;

/* Fill *p with the paper's constants (Section II, Appendix of constants):
 * 3 alternations r = 10, 20, 30, threshold 2.5, fill radii 50 and 20,
 * smoothing radius 15, alpha 0.1, K = 3, FP32. */
void st_default_params(st_params *p);

/* Create a handle bound to HIP device `device`.  *out receives the handle.
 * ST_ENODEV when the device does not exist or is not gfx950. */
st_status st_create(st_handle *out, int device);
/* Release a handle and its scratch (synchronises the device first). */
void st_destroy(st_handle h);

/* Message for the last failing call of this thread ("" if none). */
const char *st_last_error(void);

/*
 * Whole stereo path of Section II for one rectified pair.
 *  left, right : H x W uint8 with row pitch `pitch` bytes
 *  dmin..dmax  : candidate disparities within +-4096, 8 <= dmax - dmin + 1
 *                <= 256; a range of 1..7 disparities is valid but not
 *                implemented here (ST_EUNSUPPORTED)
 *  win         : odd window size, 3..15 (15 keeps every window sum exact in
 *                24 bits and the ZNCC numerator inside int32)
 *  disparity   : H x W float out; NaN where invalid
 *  valid_mask  : H x W uint8 out; 0 invalid, 1 matched, 2 filled
 * Requires H >= win and W >= win.
 */
st_status stereo_match(st_handle h, const uint8_t *left, const uint8_t *right, int H, int W,
                       int pitch, int dmin, int dmax, int win, const st_params *params,
                       float *disparity, uint8_t *valid_mask, void *stream);

/* Bytes of the fixed per-GPU scratch array behind stereo_match_noalloc. */
#define ST_NOALLOC_SCRATCH_BYTES (64u << 20)

/*
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * computation and result as stereo_match (same arguments, same kernels),
 * but every intermediate lives in one static device array of
 * ST_NOALLOC_SCRATCH_BYTES (64 MiB) that each GPU the library runs on holds
 * until the process ends; the call allocates and frees nothing.  The caller
 * still owns the images and the outputs.
 *  - Enough for a 960x540 pair at up to 256 disparities and any window, the
 *    chessboard window included, and for every smaller pair.  A pair whose
 *    planes, maps and keys need more returns ST_EUNSUPPORTED before any
 *    device call, with the bytes needed in st_last_error().
 *  - params->debug_outputs must be 0 (the debug buffers belong to the
 *    handle): ST_EINVAL otherwise.
 *  - Every call on one GPU shares that GPU's array and it keeps the last
 *    call's contents (the call clears what must start at zero itself).
 *    Calls that overlap on one GPU - from several handles, host threads or
 *    streams without ordering between them - race on it.
 */
st_status stereo_match_noalloc(st_handle h, const uint8_t *left, const uint8_t *right, int H,
                               int W, int pitch, int dmin, int dmax, int win,
                               const st_params *params, float *disparity, uint8_t *valid_mask,
                               void *stream);

/* One pair of a batch: same meaning as the stereo_match arguments. */
typedef struct {
  const uint8_t *left, *right;
  int32_t H, W, pitch, dmin, dmax, win;
  float *disparity;
  uint8_t *valid_mask;
} st_pair;

/*
 * Many pairs of uneven size, disparity range and window in one persistent
 * matcher launch (a work queue over row bands, column spans and disparity
 * chunks, longest tasks first) followed by batched post-processing.  The
 * sequence of launches for a given batch layout is captured once into a
 * HIP graph and replayed on later calls with the same layout and pointers.
 *  pairs : host array of n_pairs descriptors (device image/output pointers)
 * Results equal stereo_match on each pair, bit for bit.
 */
st_status stereo_match_batched(st_handle h, const st_pair *pairs, int n_pairs,
                               const st_params *params, void *stream);

/*
 * Differentiable sub-pixel refinement: energy of a float disparity field
 *   E(d) = sum_{p in Omega} (1 - Z_p(d)) + lambda_tv * TV(d)
 * R_w(q) is the right row linearly interpolated at q_x - d(q) (clamped to
 * [0, W-1]); Z_p is the ZNCC of the left window and the R_w window around p;
 * Omega holds the pixels with mask != 0 whose whole window is inside the
 * image, has mask != 0 everywhere and non-zero left variance; TV sums
 * |d(q+e) - d(q)| over right and down neighbours that both have mask != 0.
 *  d     : H x W float (device)        mask : H x W uint8 (device)
 *  Z     : H x W float out, NaN outside Omega (may be NULL)
 *  E     : one double out (device)
 */
st_status stereo_refine_forward(st_handle h, const uint8_t *left, const uint8_t *right,
                                const float *d, const uint8_t *mask, int H, int W, int pitch,
                                int win, float lambda_tv, float *Z, double *E, void *stream);
/* dE/dd for the same energy (hand-written backward), H x W float out.
 * At an integer interpolation coordinate the slope of the segment to the
 * right is used; |.| contributes 0 where a difference is exactly 0. */
st_status stereo_refine_backward(st_handle h, const uint8_t *left, const uint8_t *right,
                                 const float *d, const uint8_t *mask, int H, int W, int pitch,
                                 int win, float lambda_tv, float *grad_d, void *stream);
/* One clamped gradient step d <- d - clamp(tau * g, -max_step, max_step) on
 * pixels with mask != 0 (device arrays, H x W). */
st_status stereo_refine_step(st_handle h, float *d, const float *grad_d, const uint8_t *mask,
                             int H, int W, float tau, float max_step, void *stream);

/*
 * Device pointer of an intermediate of the last stereo_match call made with
 * debug_outputs = 1 (the handle owns the memory; valid until the next call):
 *  "o_wta" int16 H x W   left-reference WTA disparity
 *  "m_wta" uint8         1 where some candidate is valid
 *  "o_r"   int16         right-reference WTA disparity (indexed by xr)
 *  "m_r"   uint8
 *  "zbest" double        exact ZNCC at o_wta      "zm", "zp" double: at o_wta -+ 1 (NaN if none)
 *  "delta" float         parabola offset
 *  "m_lr"  uint8         mask after the left-right check
 *  "o_post" int16, "m_post" uint8   disparity and mask after outlier removal/fills
 *  with research = 1 and K = smooth_iters >= 2, for j = 1 .. K-1:
 *  "o_rs<j>" int16  the discrete disparities after the j-th Eq. (4) re-search
 *  "d_rs<j>" double the smoothed d^j that re-search was centred on
 * (integer disparities are -32768 where their mask is 0)
 * ST_EINVAL for an unknown name or when no debug run is held.
 */
st_status stereo_debug_get(st_handle h, const char *name, void **dev_ptr);

/* ---- single stages, for stage-wise checks; all arrays H x W, dense ---- */

/* Window statistics (Section II-A): S = sum I, SS = sum I^2 over the window
 * of every pixel whose window lies inside the image (0 elsewhere), and
 * inv = 1/sqrt(n*SS - S^2) computed in FP64 (NaN where the window leaves
 * the image or has zero variance).  chess = 0: the square window, n = win^2;
 * chess = 1: its chessboard cells (u + v even around the centre),
 * n = (win^2 + 1) / 2.  The same flag has this meaning in st_match_wta,
 * st_subpixel and st_research. */
st_status st_window_stats(st_handle h, const uint8_t *img, int H, int W, int pitch, int win,
                          int chess, int32_t *S, int32_t *SS, float *inv, void *stream);

/* ZNCC matching and winner-take-all in both references (Section II-A).
 *  oL, mL : argmax_d z(x, y, d) and 1 if any candidate is valid
 *           (oL = -32768 where mL = 0)
 *  oR, mR : for right pixel xr, argmax_d z(xr + d, y, d) (-32768 where
 *           mR = 0)
 * Candidates whose windows leave the image or have zero variance are
 * invalid; ties within 2^-18 of each other may resolve to either.
 * precision selects FP32 or FP16/BF16 image and cost storage. */
st_status st_match_wta(st_handle h, const uint8_t *left, const uint8_t *right, int H, int W,
                       int pitch, int dmin, int dmax, int win, int chess, int precision,
                       int16_t *oL, uint8_t *mL, int16_t *oR, uint8_t *mR, void *stream);

/* Exact ZNCC at oL-1, oL, oL+1 (int32 sums, FP64 normalisation) and the
 * parabola offset delta; zm/zp NaN where the neighbour is not a valid
 * candidate.  Any of zbest/zm/zp may be NULL.  A pixel with mL != 0 must
 * have oL in [dmin, dmax]; one outside is treated as unmatched (NaN z,
 * delta 0). */
st_status st_subpixel(st_handle h, const uint8_t *left, const uint8_t *right, int H, int W,
                      int pitch, int dmin, int dmax, int win, int chess, const int16_t *oL,
                      const uint8_t *mL, double *zbest, double *zm, double *zp, float *delta,
                      void *stream);

/* Left-right check: mask_out = mL && |oL(x) - oR(x - oL(x))| <= tol. */
st_status st_lr_check(st_handle h, const int16_t *oL, const uint8_t *mL, const int16_t *oR,
                      const uint8_t *mR, int H, int W, int tol, uint8_t *mask_out, void *stream);

/* Radial outlier removal with radius r (Section II-B); mask codes of kept
 * pixels are preserved.  m_out must not alias m_in. */
st_status st_radial_outlier(st_handle h, const int16_t *o, const uint8_t *m_in, int H, int W,
                            int r, float thresh, uint8_t *m_out, void *stream);

/* Hole filling (Section II-B): radial then disk; filled pixels get code 2.
 * o_out/m_out must not alias the inputs; o_out is -32768 where m_out = 0. */
st_status st_fill(st_handle h, const int16_t *o_in, const uint8_t *m_in, int H, int W,
                  int radial_r, int min_lines, int disk_r, float min_frac, int16_t *o_out,
                  uint8_t *m_out, void *stream);

/* Improved Laplacian smoothing (Section II-C, Eqs. 1-3) of s over pixels
 * with m != 0 and a (2R+1)^2 window, K iterations, computed in FP64;
 * out is NaN where m == 0. */
st_status st_hc_smooth(st_handle h, const float *s, const uint8_t *m, int H, int W, int R, int K,
                       float alpha, float *out, void *stream);

/* One Eq. (4) re-search (Section II-C) of every pixel with m != 0: among the
 * integers c in [d - range, d + range] and [dmin, dmax] whose ZNCC is
 * defined (both windows inside the image, non-zero variances), the c
 * minimising 1/max(z, 1e-3) + eta (c - d)^2, ties to the smaller c (the
 * paper's reciprocal ZNCC held finite where z <= 0); a pixel without a
 * defined candidate keeps o_in.  z is exact (integer window sums, FP64
 * normalisation).  left/right: device uint8 with pitch; o_in, o_out: device
 * int16 H x W (must not alias); m: device uint8 H x W; d: device FP64 H x W.
 * ST_EINVAL for bad shapes, range outside [0, 64], eta < 0 or NULL pointers. */
st_status st_research(st_handle h, const uint8_t *left, const uint8_t *right, int H, int W,
                      int pitch, int dmin, int dmax, int win, int chess, const int16_t *o_in,
                      const uint8_t *m, const double *d, int range, float eta, int16_t *o_out,
                      void *stream);

/* ---- disparity to 3-D points ---- */

/* Reprojection of a disparity map to 3-D points (Section II: after stereo
 * calibration the depths follow directly from the disparities; the paper's
 * conversion is the one of Matlab's reconstructScene).  Q is the 4x4
 * reprojection matrix of the rectified pair (host memory, 16 doubles,
 * row-major): pixel (x, y) with disparity d gives
 *   [X Y Z W]^T = Q [x y d 1]^T,   point = (X/W, Y/W, Z/W),
 * so that for a horizontal rig (focal length f, baseline B, principal point
 * (cx, cy)) Z = f B / d.  disparity: device, H x W float, NaN = invalid;
 * xyz: device, H x W x 3 float (x, y, z interleaved), written by the call.
 * A point is NaN where d is NaN or W == 0.  Arithmetic in FP64, stored as
 * float.  ST_EINVAL for NULL pointers or a bad shape. */
st_status st_reproject(st_handle h, const float *disparity, int H, int W, const double *Q,
                       float *xyz, void *stream);

/* ---- tuning ---- */

/* Time the matcher's tile variants (band height, disparity chunks per
 * workgroup, disparities per lane) for one problem shape on the handle's
 * device (a seeded texture and its shift: the matcher's work does not
 * depend on the image content) and remember the
 * fastest for that (win, disparity-count bucket, width bucket, precision).  The table
 * is saved to / loaded from the JSON file named by the environment variable
 * STEREO_TUNE_CACHE when it is set.  *best_cfg (host, may be NULL) receives
 * the chosen variant id. */
st_status st_autotune(st_handle h, int H, int W, int dmin, int dmax, int win, int precision,
                      int *best_cfg, void *stream);

/*
 * Autotuner of the batched launch: for every window size in the batch, the
 * persistent matcher launch of that window's pairs is timed (reps launches,
 * HIP events on `stream`) under each matcher variant - band height, chunks
 * per workgroup task and disparities per lane, st_variant_name() - and the
 * fastest is kept in the handle's tuning table under a key of the batch
 * layout (the window, precision, window shape and every pair's size and
 * range), which stereo_match_batched reads when it builds the graph of a
 * batch with that layout (and the STEREO_TUNE_CACHE file keeps).  Runs the
 * whole batch once per variant, so it writes the pairs' outputs; they end
 * as stereo_match_batched leaves them with the tuned choice.
 *  best_cfg : host array of n_pairs ints (may be NULL): the variant chosen
 *             for each pair's window size
 * Same argument errors as stereo_match_batched; reps outside [1, 1000]
 * gives ST_EINVAL.
 */
st_status st_autotune_batched(st_handle h, const st_pair *pairs, int n_pairs,
                              const st_params *params, int reps, int *best_cfg, void *stream);
/* The variant the handle's current batched graph uses for window size win
 * (-1 if no batch is held or none of its pairs has that window). */
int st_batch_variant(st_handle h, int win);

/* Average duration in milliseconds (*ms_out, host) of the batched matcher
 * kernel alone, timed with HIP events on `stream` around each of `reps`
 * launches, for the batch described as in stereo_match_batched (which is run
 * first, so every output is also produced).  For measurement harnesses. */
st_status stereo_time_matcher(st_handle h, const st_pair *pairs, int n_pairs,
                              const st_params *params, int reps, float *ms_out, void *stream);

/* Force a matcher variant for later calls on this handle (-1 = automatic).
 * Variant ids are 0..st_num_variants()-1. */
st_status st_set_variant(st_handle h, int variant);
int st_num_variants(void);
/* Host string describing variant v ("TY=8,CG=16": band height, disparity
 * chunks of 8 per workgroup), "" if out of range. */
const char *st_variant_name(int v);

/* Build information (host string). */
const char *st_version(void);

#ifdef __cplusplus
}
#endif

#endif /* STEREO_MI355X_H */
