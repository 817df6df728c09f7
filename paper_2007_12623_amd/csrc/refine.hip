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

enum {
  RF_RW = 0, RF_SLOPE, RF_V, RF_W, RF_WW, RF_LW, RF_L, RF_LL,   // inputs of the box sums
  RF_BV, RF_BW, RF_BWW, RF_BLW, RF_BL, RF_BLL,                  // their box sums
  RF_TMP, RF_A1, RF_A2, RF_A3, RF_A4, RF_B1, RF_B2, RF_B3, RF_B4,
  RF_NPLANES
};

__global__ void refine_warp_kernel(RefineArgs A) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= A.W) return;
  const size_t N = (size_t)A.W * A.H, k = (size_t)y * A.W + x;
  const double dd = (double)A.d[k];
  const double u0 = (double)x - dd;
  double u = u0 < 0.0 ? 0.0 : (u0 > A.W - 1.0 ? A.W - 1.0 : u0);
  int i0 = (int)floor(u);
  if (i0 > A.W - 1) i0 = A.W - 1;
  const int i1 = i0 + 1 < A.W ? i0 + 1 : A.W - 1;
  const double t = u - i0;
  const uint8_t *rr = A.R + (size_t)y * A.pitch;
  const double r0 = rr[i0], r1 = rr[i1];
  const double rw = r0 * (1.0 - t) + r1 * t;
  const double l = A.L[(size_t)y * A.pitch + x];
  A.f[RF_RW * N + k] = rw;
  A.f[RF_SLOPE * N + k] = (u0 >= 0.0 && u0 <= A.W - 1.0) ? (r1 - r0) : 0.0;
  A.f[RF_V * N + k] = A.mask[k] ? 1.0 : 0.0;
  A.f[RF_W * N + k] = rw;
  A.f[RF_WW * N + k] = rw * rw;
  A.f[RF_LW * N + k] = l * rw;
  A.f[RF_L * N + k] = l;
  A.f[RF_LL * N + k] = l * l;
}

__global__ void rbox_v_kernel(const double *__restrict__ in, double *out, int H, int W, int R,
                              int seg) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y0 = blockIdx.y * seg;
  if (x >= W || y0 >= H) return;
  double s = 0.0;
  for (int v = y0 - R; v <= y0 + R; ++v)
    if (v >= 0 && v < H) s += in[(size_t)v * W + x];
  const int y1 = min(y0 + seg, H);
  for (int y = y0; y < y1; ++y) {
    out[(size_t)y * W + x] = s;
    const int a = y + R + 1, b = y - R;
    if (a < H) s += in[(size_t)a * W + x];
    if (b >= 0) s -= in[(size_t)b * W + x];
  }
}

__global__ void rbox_h_kernel(const double *__restrict__ in, double *out, int H, int W, int R,
                              int seg) {
  const int y = blockIdx.x * blockDim.x + threadIdx.x;
  const int x0 = blockIdx.y * seg;
  if (y >= H || x0 >= W) return;
  const double *row = in + (size_t)y * W;
  double s = 0.0;
  for (int u = x0 - R; u <= x0 + R; ++u)
    if (u >= 0 && u < W) s += row[u];
  const int x1 = min(x0 + seg, W);
  for (int x = x0; x < x1; ++x) {
    out[(size_t)y * W + x] = s;
    const int a = x + R + 1, b = x - R;
    if (a < W) s += row[a];
    if (b >= 0) s -= row[b];
  }
}

// Omega, Z, the energy terms and the backward fields A1..A4.
__global__ __launch_bounds__(256) void refine_z_kernel(RefineArgs A) {
  __shared__ double red[256];
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  const size_t N = (size_t)A.W * A.H;
  double e = 0.0;
  if (x < A.W) {
    const size_t k = (size_t)y * A.W + x;
    const int h = A.win / 2;
    const double n = (double)A.win * A.win;
    const double *f = A.f;
    double z = __builtin_nan(""), a1 = 0, a2 = 0, a3 = 0, a4 = 0;
    const bool inside = x >= h && x <= A.W - 1 - h && y >= h && y <= A.H - 1 - h;
    if (A.mask[k] && inside && f[RF_BV * N + k] > n - 0.5) {
      const double sl = f[RF_BL * N + k], sll = f[RF_BLL * N + k];
      const double sw = f[RF_BW * N + k], sww = f[RF_BWW * N + k], slw = f[RF_BLW * N + k];
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
      if (x + 1 < A.W && A.mask[k + 1]) e += A.lambda * fabs((double)A.d[k + 1] - dk);
      if (y + 1 < A.H && A.mask[k + A.W]) e += A.lambda * fabs((double)A.d[k + A.W] - dk);
    }
  }
  red[threadIdx.x] = e;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) A.partial[blockIdx.y * gridDim.x + blockIdx.x] = red[0];
}

// Fixed-order sum of the block partials (deterministic).
__global__ __launch_bounds__(256) void refine_sum_kernel(const double *partial, int n, double *E) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += partial[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *E = red[0];
}

__device__ __forceinline__ double sgn(double v) { return v > 0.0 ? 1.0 : (v < 0.0 ? -1.0 : 0.0); }

__global__ void refine_grad_kernel(RefineArgs A) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= A.W) return;
  const size_t N = (size_t)A.W * A.H, k = (size_t)y * A.W + x;
  const double *f = A.f;
  const double l = f[RF_L * N + k], rw = f[RF_RW * N + k];
  const double gR = -(l * f[RF_B1 * N + k] - f[RF_B2 * N + k] - rw * f[RF_B3 * N + k] +
                      f[RF_B4 * N + k]);
  double g = gR * (-f[RF_SLOPE * N + k]);
  if (A.mask[k]) {
    const double dk = A.d[k];
    double tv = 0.0;
    if (x + 1 < A.W && A.mask[k + 1]) tv -= sgn((double)A.d[k + 1] - dk);
    if (y + 1 < A.H && A.mask[k + A.W]) tv -= sgn((double)A.d[k + A.W] - dk);
    if (x > 0 && A.mask[k - 1]) tv += sgn(dk - (double)A.d[k - 1]);
    if (y > 0 && A.mask[k - A.W]) tv += sgn(dk - (double)A.d[k - A.W]);
    g += A.lambda * tv;
  }
  A.grad[k] = (float)g;
}

__global__ void refine_step_kernel(float *d, const float *g, const uint8_t *mask, int N, float tau,
                                   float ms) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N || !mask[k]) return;
  float s = tau * g[k];
  s = s > ms ? ms : (s < -ms ? -ms : s);
  d[k] -= s;
}

static void rbox(const RefineArgs &A, int in, int out, hipStream_t s) {
  const size_t N = (size_t)A.W * A.H;
  const int R = A.win / 2, seg = 32;
  hipLaunchKernelGGL(rbox_v_kernel, dim3(ceil_div(A.W, 64), ceil_div(A.H, seg)), dim3(64), 0, s,
                     A.f + in * N, A.f + RF_TMP * N, A.H, A.W, R, seg);
  hipLaunchKernelGGL(rbox_h_kernel, dim3(ceil_div(A.H, 64), ceil_div(A.W, seg)), dim3(64), 0, s,
                     A.f + RF_TMP * N, A.f + out * N, A.H, A.W, R, seg);
}

int refine_planes() { return RF_NPLANES; }
int refine_partials(int H, int W) { return ceil_div(W, 256) * H; }

static void refine_common(const RefineArgs &A, hipStream_t s) {
  const dim3 g(ceil_div(A.W, 256), A.H);
  hipLaunchKernelGGL(refine_warp_kernel, g, dim3(256), 0, s, A);
  for (int p = 0; p < 6; ++p) rbox(A, RF_V + p, RF_BV + p, s);
  hipLaunchKernelGGL(refine_z_kernel, g, dim3(256), 0, s, A);
}

hipError_t launch_refine_forward(const RefineArgs &A, hipStream_t s) {
  refine_common(A, s);
  hipLaunchKernelGGL(refine_sum_kernel, dim3(1), dim3(256), 0, s, A.partial,
                     refine_partials(A.H, A.W), A.E);
  return hipGetLastError();
}

hipError_t launch_refine_backward(const RefineArgs &A, hipStream_t s) {
  refine_common(A, s);
  for (int p = 0; p < 4; ++p) rbox(A, RF_A1 + p, RF_B1 + p, s);
  hipLaunchKernelGGL(refine_grad_kernel, dim3(ceil_div(A.W, 256), A.H), dim3(256), 0, s, A);
  return hipGetLastError();
}

hipError_t launch_refine_step(float *d, const float *g, const uint8_t *mask, int N, float tau,
                              float ms, hipStream_t s) {
  hipLaunchKernelGGL(refine_step_kernel, dim3(ceil_div(N, 256)), dim3(256), 0, s, d, g, mask, N,
                     tau, ms);
  return hipGetLastError();
}

}  // namespace st
