// Reverse pass of one SPDHG iteration (Algorithm 1), for differentiation
// through unrolled iterations. With c_x = 1/(1 + 2 tau alpha),
// c_y = 1/(1 + sigma N/2), the forward iteration on gate i is
//   x1 = c_x (x - tau zbar);  s = A D_i x1;  y1 = c_y (y + sigma (s - d));
//   dy = y1 - y;  b = A^T dy;  dz = D_i^T b;  z1 = z + dz;  zbar1 = z1 + (theta/p) dz
// and, given the adjoints (gx, gy, gz, gzbar) of its outputs, its reverse is
//   gdz = gz + (1 + theta/p) gzbar;  gz += gzbar
//   gb = D_i gdz;          motion += d/dtheta <b, D_i(theta) gdz>
//   gdy = A gb;  G = gy + gdy;  gy = c_y G - gdy;  gs = c_y sigma G
//   gw = A^T gs;  gx1 = gx + D_i^T gw;   motion += d/dtheta <gw, D_i(theta) x1>
//   gx = c_x gx1;  gzbar = -tau c_x gx1
// The elementwise steps are below; the operators are the forward kernels.
#pragma once

#include "mcr_kernels.h"

namespace mcr {

template <typename T>
__global__ __launch_bounds__(256) void k_bwd_z(long count, T* __restrict__ gz, const T* __restrict__ gzb,
                                               T* __restrict__ gdz, T coef1) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  const T a = gz[i], b = gzb[i];
  gdz[i] = fmaT(coef1, b, a);
  gz[i] = a + b;
}

template <typename T>
__global__ __launch_bounds__(256) void k_bwd_dual(long count, T* __restrict__ gy, T* __restrict__ gdy_gs, T cy,
                                                  T sigma) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  const T gdy = gdy_gs[i];
  const T G = gy[i] + gdy;
  gy[i] = cy * G - gdy;
  gdy_gs[i] = cy * sigma * G;
}

template <typename T>
__global__ __launch_bounds__(256) void k_bwd_x(long count, T* __restrict__ gx, T* __restrict__ gzb, T cx,
                                               T tau) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  const T g1 = gx[i];
  gx[i] = cx * g1;
  gzb[i] = -tau * cx * g1;
}

// d/d(motion of gate) <h, D(theta) v>: the bilinear interpolant's gradient
// at the sample position (floor branch at grid lines) times the position's
// derivative. h: padded image (interior read), v: unpadded image.
//   rigid: three sums (phi, t_x, t_y) per block into partial[block][3] (FP64)
//   field: gfield[0][p] += h gx, gfield[1][p] += h gy
// grid (ceil(n/16), ceil(n/16)), block (16, 16)
template <typename T>
__global__ __launch_bounds__(256) void k_motion_grad(Geo<T> g, const GateMotion<T>* __restrict__ gm, int gate,
                                                     const float* __restrict__ field, long field_stride,
                                                     long plane_stride, const T* __restrict__ hP,
                                                     const T* __restrict__ v, double* __restrict__ partial,
                                                     T* __restrict__ gfield) {
  __shared__ double sh[3][4];
  const int c = blockIdx.x * 16 + threadIdx.x;
  const int r = blockIdx.y * 16 + threadIdx.y;
  const int n = g.n, pitch = g.pitch;
  const GateMotion<T> M = gm[gate];
  const long origin = (long)kPad * pitch + kPad;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  if (c < n && r < n) {
    const float* ux = field + gate * field_stride + origin;
    const float* uy = ux + plane_stride;
    const Tap<T> tp = motion_tap(M, ux, uy, pitch, g.hc, r, c);
    auto at = [&](int rr, int cc) -> T {
      return ((unsigned)rr < (unsigned)n && (unsigned)cc < (unsigned)n) ? v[(long)rr * n + cc] : T(0);
    };
    const T v00 = at(tp.r0, tp.c0), v01 = at(tp.r0, tp.c0 + 1);
    const T v10 = at(tp.r0 + 1, tp.c0), v11 = at(tp.r0 + 1, tp.c0 + 1);
    const T gx = (T(1) - tp.fy) * (v01 - v00) + tp.fy * (v11 - v10);
    const T gy = (T(1) - tp.fx) * (v10 - v00) + tp.fx * (v11 - v01);
    const T hv = hP[origin + (long)r * pitch + c];
    if (M.kind == 1) {
      const T xc = T(c) - g.hc, yc = T(r) - g.hc;
      const T cs = M.cm1 + T(1);
      const T dpx = -M.sn * xc - cs * yc;  // d(px)/d(phi)
      const T dpy = cs * xc - M.sn * yc;   // d(py)/d(phi)
      a0 = double(hv) * (double(gx) * double(dpx) + double(gy) * double(dpy));
      a1 = double(hv) * double(gx);
      a2 = double(hv) * double(gy);
    } else if (M.kind == 2) {
      const long q = (long)r * n + c;
      gfield[q] += hv * gx;
      gfield[(long)n * n + q] += hv * gy;
    }
  }
  if (M.kind != 1) return;
  const int tid = threadIdx.y * 16 + threadIdx.x;
  double vals[3] = {a0, a1, a2};
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    double x = vals[m];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if ((tid & 63) == 0) sh[m][tid >> 6] = x;
  }
  __syncthreads();
  if (tid < 3) {
    const double s = sh[tid][0] + sh[tid][1] + sh[tid][2] + sh[tid][3];
    partial[(long)(blockIdx.y * gridDim.x + blockIdx.x) * 3 + tid] = s;
  }
}

// Adds the block partials (fixed order) to grad[0..2].
__global__ __launch_bounds__(256) void k_motion_grad_final(const double* __restrict__ partial, int blocks,
                                                           double* __restrict__ grad) {
  __shared__ double sh[3][4];
  double a[3] = {0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < blocks; b += 256) {
#pragma unroll
    for (int m = 0; m < 3; ++m) a[m] += partial[(long)b * 3 + m];
  }
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    double x = a[m];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if ((threadIdx.x & 63) == 0) sh[m][threadIdx.x >> 6] = x;
  }
  __syncthreads();
  if (threadIdx.x < 3) grad[threadIdx.x] += sh[threadIdx.x][0] + sh[threadIdx.x][1] + sh[threadIdx.x][2] + sh[threadIdx.x][3];
}

}  // namespace mcr
