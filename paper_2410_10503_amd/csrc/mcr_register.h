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

}  // namespace mcr
