// Device code of the rigid registration (the preliminary step of Section I:
// the displacement maps from the reference state to each gate): the residual
// of the warped reference against the gate's image, written into the padded
// layout that the motion-gradient kernel reads. The warp, the reductions and
// the motion gradient are the library's own kernels.
#pragma once

#include "mcr_kernels.h"

namespace mcr {

// rP = wP - target on the image (the zero border of rP is left as it is).
// grid (ceil(n/16), ceil(n/16)), block (16, 16)
template <typename T>
__global__ __launch_bounds__(256) void k_residual_padded(int n, int pitch, const T* __restrict__ wP,
                                                         const T* __restrict__ target, T* __restrict__ rP) {
  const int c = blockIdx.x * 16 + threadIdx.x;
  const int r = blockIdx.y * 16 + threadIdx.y;
  if (c < n && r < n) {
    const long q = (long)(r + kPad) * pitch + c + kPad;
    rP[q] = wP[q] - target[(long)r * n + c];
  }
}

// Affine displacement field u(p) = A (p - c) + t of one gate, written into its
// padded field planes (plane_stride apart): x = column - c, y = row - c,
// c = (n - 1) / 2, each component evaluated as (A_r0 x + A_r1 y) + t_r in
// double without contraction, then rounded to float (the library's field
// precision). grid (ceil(n/16), ceil(n/16)), block (16, 16)
__global__ __launch_bounds__(256) void k_affine_field(int n, int pitch, long plane_stride, double a00, double a01,
                                                      double a10, double a11, double tx, double ty,
                                                      float* __restrict__ fP) {
#pragma clang fp contract(off)
  const int c = blockIdx.x * 16 + threadIdx.x;
  const int r = blockIdx.y * 16 + threadIdx.y;
  if (c < n && r < n) {
    const double hc = 0.5 * (n - 1);
    const double x = c - hc, y = r - hc;
    const double ux = (a00 * x + a01 * y) + tx;
    const double uy = (a10 * x + a11 * y) + ty;
    const long q = (long)(r + kPad) * pitch + c + kPad;
    fP[q] = (float)ux;
    fP[plane_stride + q] = (float)uy;
  }
}

// The six moments of the field gradient planes G = (G_x, G_y) [2][n][n] that
// give the affine parameters' gradient: sum G_x x, sum G_x y, sum G_y x,
// sum G_y y, sum G_x, sum G_y (x, y centred as above). Block partials
// [kRedBlocks][6], then a fixed-order sum: deterministic.
template <typename T>
__global__ __launch_bounds__(256) void k_affine_moments(int n, const T* __restrict__ gf, double* __restrict__ partial) {
  __shared__ double sh[4];
  double a[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const double hc = 0.5 * (n - 1);
  const long n2 = (long)n * n;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n2; i += (long)kRedBlocks * 256) {
    const double x = double(i % n) - hc, y = double(i / n) - hc;
    const double gx = double(gf[i]), gy = double(gf[n2 + i]);
    a[0] = __builtin_fma(gx, x, a[0]);
    a[1] = __builtin_fma(gx, y, a[1]);
    a[2] = __builtin_fma(gy, x, a[2]);
    a[3] = __builtin_fma(gy, y, a[3]);
    a[4] += gx;
    a[5] += gy;
  }
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    const double s = block_sum(a[m], sh);
    if (threadIdx.x == 0) partial[(long)blockIdx.x * 6 + m] = s;
    __syncthreads();  // sh is reused by the next sum
  }
}

// out[m] = sum over the kRedBlocks partials of moment m, in block order.
__global__ __launch_bounds__(256) void k_affine_moments_final(const double* __restrict__ partial,
                                                              double* __restrict__ out) {
  __shared__ double sh[4];
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < kRedBlocks; b += 256) acc += partial[(long)b * 6 + m];
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) out[m] = s;
    __syncthreads();
  }
}

// Dense displacement-field registration: the iterate u [2][n*n] (FP64) and
// its float32 rounding in the gate's padded field planes (plane_stride
// apart), which the warp and the motion gradient read.
//   k_field_load:  u = f (the caller's float32 field), planes = f
//   k_field_trial: u_new = u - alpha g, planes = float(u_new)
// grid (ceil(n/16), ceil(n/16)), block (16, 16)
__global__ __launch_bounds__(256) void k_field_load(int n, int pitch, long plane_stride, const float* __restrict__ f,
                                                    double* __restrict__ u, float* __restrict__ fP) {
  const int c = blockIdx.x * 16 + threadIdx.x;
  const int r = blockIdx.y * 16 + threadIdx.y;
  if (c >= n || r >= n) return;
  const long n2 = (long)n * n, q = (long)r * n + c, o = (long)(r + kPad) * pitch + c + kPad;
  for (int pl = 0; pl < 2; ++pl) {
    const float v = f[pl * n2 + q];
    u[pl * n2 + q] = double(v);
    fP[pl * plane_stride + o] = v;
  }
}

__global__ __launch_bounds__(256) void k_field_trial(int n, int pitch, long plane_stride,
                                                     const double* __restrict__ u, const double* __restrict__ g,
                                                     double alpha, double* __restrict__ u_new,
                                                     float* __restrict__ fP) {
#pragma clang fp contract(off)
  const int c = blockIdx.x * 16 + threadIdx.x;
  const int r = blockIdx.y * 16 + threadIdx.y;
  if (c >= n || r >= n) return;
  const long n2 = (long)n * n, q = (long)r * n + c, o = (long)(r + kPad) * pitch + c + kPad;
  for (int pl = 0; pl < 2; ++pl) {
    const double step = alpha * g[pl * n2 + q];
    const double v = u[pl * n2 + q] - step;
    u_new[pl * n2 + q] = v;
    fP[pl * plane_stride + o] = float(v);
  }
}

// Gradient of the regularised misfit from the data part gd (the motion
// gradient planes, handle dtype): g = gd + lam L u, (L u)(p) the sum of
// u(p) - u(q) over the image neighbours q of p, u the float32 field planes;
// partial[block] = the block's share of R(u), the squared differences of
// horizontally and vertically adjacent pixels (both components). Grid-stride
// over the pixels: grid kRedBlocks, block 256.
template <typename T>
__global__ __launch_bounds__(256) void k_field_reg_grad(int n, int pitch, long plane_stride,
                                                        const float* __restrict__ fP, const T* __restrict__ gd,
                                                        double lam, double* __restrict__ g,
                                                        double* __restrict__ partial) {
  __shared__ double sh[4];
  const long n2 = (long)n * n;
  const long origin = (long)kPad * pitch + kPad;
  double acc = 0.0;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n2; i += (long)kRedBlocks * 256) {
    const int r = (int)(i / n), c = (int)(i % n);
    for (int pl = 0; pl < 2; ++pl) {
      const float* u = fP + pl * plane_stride + origin + (long)r * pitch + c;
      const double v = double(u[0]);
      double L = 0.0;
      if (c + 1 < n) {
        const double d = double(u[1]) - v;
        L -= d;
        acc = __builtin_fma(d, d, acc);
      }
      if (c > 0) L += v - double(u[-1]);
      if (r + 1 < n) {
        const double d = double(u[pitch]) - v;
        L -= d;
        acc = __builtin_fma(d, d, acc);
      }
      if (r > 0) L += v - double(u[-pitch]);
      g[pl * n2 + i] = double(gd[pl * n2 + i]) + lam * L;
    }
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// partial[block] = the block's share of sum (a1 - a0)(b1 - b0) (FP64), for the
// Barzilai-Borwein step lengths. Grid-stride: grid kRedBlocks, block 256.
__global__ __launch_bounds__(256) void k_dot_diff(long count, const double* __restrict__ a1,
                                                  const double* __restrict__ a0, const double* __restrict__ b1,
                                                  const double* __restrict__ b0, double* __restrict__ partial) {
  __shared__ double sh[4];
  double acc = 0.0;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < count; i += (long)kRedBlocks * 256)
    acc = __builtin_fma(a1[i] - a0[i], b1[i] - b0[i], acc);
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// One pass of the separable Gaussian of the scale-space schedule: out[p] =
// sum_k w[k + R] in[p + k e], e along the row (AXIS 1) or the column (AXIS 0),
// zero outside the image, accumulated in FP64 in the order of k.
// grid (ceil(n/16), ceil(n/16)), block (16, 16)
template <typename T, int AXIS>
__global__ __launch_bounds__(256) void k_blur(int n, int R, const double* __restrict__ w, const T* __restrict__ in,
                                              T* __restrict__ out) {
  const int c = blockIdx.x * 16 + threadIdx.x;
  const int r = blockIdx.y * 16 + threadIdx.y;
  if (c >= n || r >= n) return;
  double acc = 0.0;
  for (int k = -R; k <= R; ++k) {
    const int rr = AXIS == 0 ? r + k : r, cc = AXIS == 1 ? c + k : c;
    if ((unsigned)rr < (unsigned)n && (unsigned)cc < (unsigned)n) acc += w[k + R] * double(in[(long)rr * n + cc]);
  }
  out[(long)r * n + c] = T(acc);
}

}  // namespace mcr
