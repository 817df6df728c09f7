// Differentiable sub-pixel refinement: energy of a float disparity field and
// its hand-written gradient.  The paper refines continuous disparities with a
// ZNCC-coupled improved Laplacian scheme (Section II-C); this path instead
// descends the photometric energy
//   E(d) = sum_{p in Omega} (1 - Z_p(d)) + lambda * TV(d)
// where R_w(q) is the right row linearly interpolated at q_x - d(q) (clamped
// to [0, W-1]) and Z_p the ZNCC of the left window and the R_w window at p.
// With a = L - mean_L and b = R_w - mean_w over the window of p,
//   dZ_p/dR_w(q) = a_q / (|a||b|) - Z_p b_q / |b|^2,
// so dE/dR_w(q) = -[L(q) B(alpha) - B(mu_L alpha) - R_w(q) B(Z beta) + B(Z mu_w beta)]
// with alpha = 1/(|a||b|), beta = 1/|b|^2 and B(f)(q) the sum of f over the
// windows containing q (a box sum, windows being symmetric).  Everything is
// FP64: window sums of non-integer R_w cancel as badly as any variance.
#include "common.h"

namespace st {

// Per-pixel planes kept between the passes: the backward fields of Omega's
// pixels (0 elsewhere).
enum { RF_A1 = 0, RF_A2, RF_A3, RF_A4, RF_NPLANES };

// Both passes are fused box-sum kernels: a block of RT_T threads owns RT_T
// consecutive columns (RT_T - 2h of them outputs) and A.sy rows.  Each
// thread keeps the vertical window sums of its column in registers (the
// entering row added, the leaving row removed, every input computed where
// it is needed: R_w from d and the right image, or a plane read); per row
// the block stores them in LDS and every output thread adds the 2h + 1 of
// its window.  Two LDS buffers alternate between rows, so one barrier per
// row orders the stores of a row after the reads of the row before.
// Rows per block: 32, halved down to 1 while a launch has fewer than
// RT_MINB blocks (a 960x540 pair: 2 rows, 1080 blocks).  The seed of 2h rows
// per block is the price of the blocks that fill the chip: 68 blocks of 32
// rows took 0.309 ms per refinement step at 960x540, 1080 of 2 rows 0.071.
constexpr int RT_T = 256, RT_SY = 32, RT_HMAX = 7, RT_MINB = 1024;

// R_w(x, y): the right row interpolated at u = x - d(x, y) clamped to
// [0, W-1] (segment [floor(u), floor(u) + 1]: at an integer u the segment
// to the right), and its slope dR_w/du (0 where u is clamped).
__device__ __forceinline__ void warp_px(const RefineArgs &A, int x, int y, double &rw,
                                        double &slope) {
  const double dd = (double)A.d[(size_t)y * A.W + x];
  const double u0 = (double)x - dd;
  const double u = u0 < 0.0 ? 0.0 : (u0 > A.W - 1.0 ? A.W - 1.0 : u0);
  int i0 = (int)floor(u);
  if (i0 > A.W - 1) i0 = A.W - 1;
  const int i1 = i0 + 1 < A.W ? i0 + 1 : A.W - 1;
  const double t = u - i0;
  const uint8_t *rr = A.R + (size_t)y * A.pitch;
  const double r0 = rr[i0], r1 = rr[i1];
  rw = r0 * (1.0 - t) + r1 * t;
  slope = (u0 >= 0.0 && u0 <= A.W - 1.0) ? (r1 - r0) : 0.0;
}

// Anisotropic TV terms of pixel k: lambda |d(q+e) - d(q)| over the right and
// down neighbours (energy), and the subgradient with sign(0) = 0.
__device__ __forceinline__ double sgn(double v) { return v > 0.0 ? 1.0 : (v < 0.0 ? -1.0 : 0.0); }

// Block sum of one double per thread in a fixed order (deterministic).
__device__ __forceinline__ double block_sum(double v, double *red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int off = RT_T / 2; off > 0; off >>= 1) {
    if (t < off) red[t] += red[t + off];
    __syncthreads();
  }
  return red[0];
}

// Forward: the six window sums (valid count, R_w, R_w^2, L R_w, L, L^2),
// Omega, Z, the energy of the block's pixels (to one partial per block)
// and the backward fields a1..a4 = alpha, mu_L alpha, Z beta, Z mu_w beta.
__global__ __launch_bounds__(RT_T) void refine_fwd_kernel(RefineArgs A) {
  __shared__ double sv[2][6][RT_T];
  const int h = A.win / 2, W = A.W, H = A.H, nout = RT_T - 2 * h;
  const int xo = blockIdx.x * nout, y0 = blockIdx.y * A.sy;
  const int t = threadIdx.x, c = xo - h + t;
  const bool cin = c >= 0 && c < W;
  const size_t N = (size_t)W * H;
  const double n = (double)A.win * A.win;
  double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  auto add_row = [&](int r, double sg) {
    if (!cin || r < 0 || r >= H) return;
    double rw, sl;
    warp_px(A, c, r, rw, sl);
    const double l = A.L[(size_t)r * A.pitch + c];
    acc[0] += A.mask[(size_t)r * W + c] ? sg : 0.0;
    acc[1] += sg * rw;
    acc[2] += sg * (rw * rw);
    acc[3] += sg * (l * rw);
    acc[4] += sg * l;
    acc[5] += sg * (l * l);
  };
  for (int r = y0 - h; r < y0 + h; ++r) add_row(r, 1.0);
  const int y1 = min(y0 + A.sy, H);
  const bool out_col = t >= h && t < RT_T - h && c < W;
  double e = 0.0;
  for (int y = y0; y < y1; ++y) {  // the same rows for every thread
    add_row(y + h, 1.0);
    const int b = y & 1;
#pragma unroll
    for (int q = 0; q < 6; ++q) sv[b][q][t] = acc[q];
    add_row(y - h, -1.0);
    __syncthreads();
    if (out_col) {
      double sb[6];
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        double v = 0.0;
        for (int j = -h; j <= h; ++j) v += sv[b][q][t + j];
        sb[q] = v;
      }
      const size_t k = (size_t)y * W + c;
      double z = __builtin_nan(""), a1 = 0, a2 = 0, a3 = 0, a4 = 0;
      const bool inside = c >= h && c <= W - 1 - h && y >= h && y <= H - 1 - h;
      if (A.mask[k] && inside && sb[0] > n - 0.5) {
        const double sw = sb[1], sww = sb[2], slw = sb[3], sl = sb[4], sll = sb[5];
        const double saa = sll - sl * sl / n;
        if (saa > 0.0 && n * sll - sl * sl > 0.5) {
          const double sbb = sww - sw * sw / n;
          const double sab = slw - sl * sw / n;
          z = 0.0;
          if (sbb > 1e-6 * n) {  // numerically constant R_w window: Z = 0
            const double al = 1.0 / sqrt(saa * sbb);
            const double be = 1.0 / sbb;
            z = sab * al;
            a1 = al;
            a2 = (sl / n) * al;
            a3 = z * be;
            a4 = z * (sw / n) * be;
          }
          e += 1.0 - z;
        }
      }
      if (A.Z) A.Z[k] = (float)z;
      A.f[RF_A1 * N + k] = a1;
      A.f[RF_A2 * N + k] = a2;
      A.f[RF_A3 * N + k] = a3;
      A.f[RF_A4 * N + k] = a4;
      if (A.mask[k]) {
        const double dk = A.d[k];
        if (c + 1 < W && A.mask[k + 1]) e += A.lambda * fabs((double)A.d[k + 1] - dk);
        if (y + 1 < H && A.mask[k + W]) e += A.lambda * fabs((double)A.d[k + W] - dk);
      }
    }
  }
  __syncthreads();  // the last row's window reads are done before sv is reused
  const double tot = block_sum(e, &sv[0][0][0]);
  if (t == 0) A.partial[blockIdx.y * gridDim.x + blockIdx.x] = tot;
}

// Fixed-order sum of the block partials (deterministic).
__global__ __launch_bounds__(RT_T) void refine_sum_kernel(const double *partial, int n, double *E) {
  __shared__ double red[RT_T];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += RT_T) s += partial[i];
  const double tot = block_sum(s, red);
  if (threadIdx.x == 0) *E = tot;
}

// Backward: B(a1..a4), the sums of the fields over the windows that contain
// q, then dE/dd(q) = dE/dR_w(q) (-slope(q)) + lambda dTV/dd(q) with
// dE/dR_w(q) = -[L(q) B(a1) - B(a2) - R_w(q) B(a3) + B(a4)].
__global__ __launch_bounds__(RT_T) void refine_bwd_kernel(RefineArgs A) {
  __shared__ double sv[2][4][RT_T];
  const int h = A.win / 2, W = A.W, H = A.H, nout = RT_T - 2 * h;
  const int xo = blockIdx.x * nout, y0 = blockIdx.y * A.sy;
  const int t = threadIdx.x, c = xo - h + t;
  const bool cin = c >= 0 && c < W;
  const size_t N = (size_t)W * H;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  auto add_row = [&](int r, double sg) {
    if (!cin || r < 0 || r >= H) return;
    const size_t k = (size_t)r * W + c;
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] += sg * A.f[q * N + k];
  };
  for (int r = y0 - h; r < y0 + h; ++r) add_row(r, 1.0);
  const int y1 = min(y0 + A.sy, H);
  const bool out_col = t >= h && t < RT_T - h && c < W;
  for (int y = y0; y < y1; ++y) {
    add_row(y + h, 1.0);
    const int b = y & 1;
#pragma unroll
    for (int q = 0; q < 4; ++q) sv[b][q][t] = acc[q];
    add_row(y - h, -1.0);
    __syncthreads();
    if (out_col) {
      double bs[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        double v = 0.0;
        for (int j = -h; j <= h; ++j) v += sv[b][q][t + j];
        bs[q] = v;
      }
      const size_t k = (size_t)y * W + c;
      double rw, slope;
      warp_px(A, c, y, rw, slope);
      const double l = A.L[(size_t)y * A.pitch + c];
      const double gR = -(l * bs[0] - bs[1] - rw * bs[2] + bs[3]);
      double g = gR * (-slope);
      if (A.mask[k]) {
        const double dk = A.d[k];
        double tv = 0.0;
        if (c + 1 < W && A.mask[k + 1]) tv -= sgn((double)A.d[k + 1] - dk);
        if (y + 1 < H && A.mask[k + W]) tv -= sgn((double)A.d[k + W] - dk);
        if (c > 0 && A.mask[k - 1]) tv += sgn(dk - (double)A.d[k - 1]);
        if (y > 0 && A.mask[k - W]) tv += sgn(dk - (double)A.d[k - W]);
        g += A.lambda * tv;
      }
      A.grad[k] = (float)g;
    }
  }
}

__global__ void refine_step_kernel(float *d, const float *g, const uint8_t *mask, int N, float tau,
                                   float ms) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N || !mask[k]) return;
  float s = tau * g[k];
  s = s > ms ? ms : (s < -ms ? -ms : s);
  d[k] -= s;
}

// The launch's rows per block (A.sy) and grid.
static dim3 rgrid(RefineArgs &A) {
  const int gx = ceil_div(A.W, RT_T - 2 * (A.win / 2));
  A.sy = RT_SY;
  while (A.sy > 1 && (long long)gx * ceil_div(A.H, A.sy) < RT_MINB) A.sy /= 2;
  return dim3(gx, ceil_div(A.H, A.sy));
}

int refine_planes() { return RF_NPLANES; }
// partials of the forward pass: at most one block per row and column
// segment of the largest window
int refine_partials(int H, int W) { return ceil_div(W, RT_T - 2 * RT_HMAX) * H; }

hipError_t launch_refine_forward(const RefineArgs &A0, hipStream_t s) {
  RefineArgs A = A0;
  const dim3 g = rgrid(A);
  hipLaunchKernelGGL(refine_fwd_kernel, g, dim3(RT_T), 0, s, A);
  hipLaunchKernelGGL(refine_sum_kernel, dim3(1), dim3(RT_T), 0, s, A.partial, (int)(g.x * g.y), A.E);
  return hipGetLastError();
}

hipError_t launch_refine_backward(const RefineArgs &A0, hipStream_t s) {
  RefineArgs A = A0;
  const dim3 g = rgrid(A);
  hipLaunchKernelGGL(refine_fwd_kernel, g, dim3(RT_T), 0, s, A);
  hipLaunchKernelGGL(refine_bwd_kernel, g, dim3(RT_T), 0, s, A);
  return hipGetLastError();
}

hipError_t launch_refine_step(float *d, const float *g, const uint8_t *mask, int N, float tau,
                              float ms, hipStream_t s) {
  hipLaunchKernelGGL(refine_step_kernel, dim3(ceil_div(N, 256)), dim3(256), 0, s, d, g, mask, N,
                     tau, ms);
  return hipGetLastError();
}

}  // namespace st
