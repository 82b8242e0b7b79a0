// Device code of libmcr: the hot path of motion-compensated SPDHG/PDHG on
// gfx950. Every kernel is templated on the scalar type T (float for the bulk
// path, double for the FP64 diagnostics); all are gathers, so every output
// element is written by exactly one thread (no atomics on the hot path, bitwise
// reproducible).
//
// Layouts in HBM
//   image         [n][n] row-major (caller arrays)
//   padded image  [n+2P][n+2P] with a zero border of P = 4 pixels (handle
//                 workspaces): lets the projector and the transposed warp read
//                 neighbours of edge pixels without bounds checks
//   sinogram      [n_angles][n_det] row-major, detector fastest
//   field         padded [2][n+2P][n+2P] float (u_x plane, u_y plane)
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcr {

constexpr int kPad = 4;          // zero border of padded images and fields
constexpr int kMaxRadius = 3;    // largest gather window radius of D^T
constexpr int kLineBlock = 16;   // block length of the two-level float sums

// Per-angle constants of the Joseph projector, built in FP64 on the host.
// Along the stepping line at offset u from the centre, ray t crosses the
// interpolation axis at  cf = t * a + (u * beta + hc)  (index coordinates).
template <typename T>
struct AngleT {
  T a;      // 1/cos (row stepping) or 1/sin (column stepping)
  T beta;   // -sin/cos or -cos/sin
  T ia;     // 1/a
  T ds;     // |a|: length of the ray per line
  int rows; // 1: lines are image rows, interpolation along columns
  int pad_;
};

// Per-angle constants of the float32 projector pair in 32.32 fixed point
// (exact integer arithmetic, about 1e-7 px over the whole image):
//   crossing of ray j with line L, along the interpolation axis:
//     CF(j, L) = C0 + j A + L B          (A = 1/cos or 1/sin, B = beta)
//   detector coordinate of the point at position s on line L (pixel units):
//     U(s, L)  = U0 + s P + L Q          (P = 1/A, Q = -beta/A)
// Ray j puts weight max(0, 1 - |CF/2^32 - s|) on pixel s of line L; seen from
// the pixel this is max(0, 1 - |a| |j - U/2^32|), non-zero for the two bins
// around U/2^32 only.
struct AngleFx {
  long long C0, A, B;
  long long U0, P, Q;
  long long RS;   // U step to the next column of an image row: P when lines are rows, else Q
  float a, beta;  // float copies for the loop bounds
  float absa;     // |a|
  float oma;      // 1 - |a|
  float ds;       // length of the ray per line
  int rows;       // 1: lines are image rows
  float na32;     // -|a| 2^-32 and |a| 2^-32: hat weights from the raw fraction
  float pa32;
};

constexpr float kFix = 2.3283064365386963e-10f;  // 2^-32

// Motion of one gate. The rigid map is stored as a displacement from the
// pixel itself, phi(p) = p + delta(p) with, for xc = c - hc, yc = r - hc,
//   delta_x = (cos - 1) xc - sin yc + t_x,   delta_y = sin xc + (cos - 1) yc + t_y,
// so that the fractional part of the sample position keeps the precision of
// the (small) displacement instead of that of the (large) absolute position.
template <typename T>
struct GateMotion {
  int kind;    // 0 identity, 1 rigid, 2 field
  int radius;  // gather window radius of the transposed warp
  T cm1, sn, tx, ty;      // cos - 1, sin, translation (rigid)
  T i00, i01, i10, i11;   // inverse rotation (window centres only)
  T bx, by;               // hc + t (window centres only)
};

// Angles a launch covers: [ka, kb) and [kc, kd) (the second range may be
// empty). An angle subset of the gates x angle-subsets sampling is one or two
// such ranges (a contiguous range, or a range and its partner range a
// quarter turn away).
struct AngleRanges {
  int ka, kb, kc, kd;
  __host__ __device__ int count() const { return (kb - ka) + (kd - kc); }
  // the v-th angle of the launch, v in [0, count())
  __host__ __device__ int at(int v) const { return v < kb - ka ? ka + v : kc + (v - (kb - ka)); }
  // angles from the v-th one to the end of its range
  __host__ __device__ int run(int v) const { return v < kb - ka ? kb - ka - v : count() - v; }
};

// Per-gate scalars of one call of Algorithm 1.
template <typename T>
struct GateScalars {
  T sigma;  // sigma_i
  T cy;     // 1 / (1 + sigma_i N / 2)
  T coef;   // theta / p_i
  T pad_;
};

// Device pointers of one gate for the fused dual step.
template <typename T>
struct GatePtrs {
  T* y;
  const T* d;
};

template <typename T>
struct Geo {
  int n, na, nd, pitch;
  T hc;  // (n-1)/2
  T jc;  // (n_det-1)/2
};

// Batched launches: block z works on slot z, which belongs to image `slice`
// and gate `gate` (an index into the handle's flat gate tables); do_x asks the
// update to fuse the next step (i) of that slice.
struct SlotInfo {
  int slice;
  int gate;
  int do_x;
  int pad_;
};

__device__ __forceinline__ int slot_gate(const SlotInfo* slots, int gate0) {
  return slots ? slots[blockIdx.z].gate : gate0 + (int)blockIdx.z;
}

__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Bilinear tap of output pixel (r, c) under the gate's motion: the sample
// position is (c0 + fx, r0 + fy) with integer (c0, r0) and fx, fy in [0, 1).
// The forward warp, the transposed warp and the window check all call this,
// so their weights are the same floating-point numbers.
template <typename T>
struct Tap {
  int c0, r0;
  T fx, fy;
};

// The bilinear tap of the sample taken for pixel (r, c) at displacement (dx, dy).
template <typename T>
__device__ __forceinline__ Tap<T> tap_from_displacement(T dx, T dy, int r, int c) {
  const T fdx = floor(dx), fdy = floor(dy);
  Tap<T> t;
  t.fx = dx - fdx;
  t.fy = dy - fdy;
  // far-away samples only need to stay far away; clamp keeps the int cast finite
  t.c0 = c + (int)fmax(fmin(fdx, T(16384)), T(-16384));
  t.r0 = r + (int)fmax(fmin(fdy, T(16384)), T(-16384));
  return t;
}

template <typename T>
__device__ __forceinline__ Tap<T> motion_tap(const GateMotion<T>& M, const float* __restrict__ ux,
                                             const float* __restrict__ uy, int pitch, T hc, int r,
                                             int c) {
  T dx = T(0), dy = T(0);
  if (M.kind == 1) {
    const T xc = T(c) - hc, yc = T(r) - hc;
    dx = fmaT(M.cm1, xc, fmaT(-M.sn, yc, M.tx));
    dy = fmaT(M.sn, xc, fmaT(M.cm1, yc, M.ty));
  } else if (M.kind == 2) {
    const long o = (long)r * pitch + c;
    dx = T(ux[o]);
    dy = T(uy[o]);
  }
  return tap_from_displacement<T>(dx, dy, r, c);
}

// Centre of the gather window of output pixel (qr, qc) for the transposed
// warp: the rounded inverse image of q (rigid: analytic inverse; field: the
// set-up table), clamped to [-1, n] so that every candidate of a window of
// radius <= kMaxRadius lies inside the zero border.
template <typename T>
__device__ __forceinline__ void window_centre(const GateMotion<T>& M, const short2* __restrict__ centres,
                                              int gate, int n, T hc, int qr, int qc, int& cr, int& cc) {
  if (M.kind == 1) {
    const T dx = T(qc) - M.bx, dy = T(qr) - M.by;
    cc = (int)rint(fmaT(M.i00, dx, fmaT(M.i01, dy, hc)));
    cr = (int)rint(fmaT(M.i10, dx, fmaT(M.i11, dy, hc)));
    cc = min(max(cc, -1), n);
    cr = min(max(cr, -1), n);
  } else {
    const short2 cen = centres[(long)gate * n * n + (long)qr * n + qc];
    cc = cen.x;
    cr = cen.y;
  }
}

// Epilogue of the projection kernels for ray idx of gate slot z:
//   MODE 0: out = A_i x
//   MODE 1: Algorithm 1 (ii): y' = (y + sigma (A_i x - d)) / (1 + sigma N/2),
//           y <- y', out = y' - y
//   MODE 2: the same dy without writing y (recomputation in the reverse pass)
template <typename T, int MODE>
__device__ __forceinline__ void project_epilogue(T s, long idx, T* __restrict__ out, int gate,
                                                 const GateScalars<T>* __restrict__ gs,
                                                 const GatePtrs<T>* __restrict__ gp) {
  if (MODE == 0) {
    out[idx] = s;
  } else {
    const GateScalars<T> S = gs[gate];
    const GatePtrs<T> P = gp[gate];
    const T yv = P.y[idx];
    const T yn = (yv + S.sigma * (s - P.d[idx])) * S.cy;
    if (MODE == 1) P.y[idx] = yn;
    out[idx] = yn - yv;
  }
}

// ---------------------------------------------------------------------------
// a1: forward warp  w = D_i x  (bilinear pull-back, zero outside the image).
// One thread per output pixel, 32x32 tiles (1024 threads, so that a 512^2
// image fills every SIMD with 4 waves); the tile is also written transposed
// (through LDS) so that the projector reads column-stepping angles with unit
// stride. With wQ, nq = 3 extra planes P_m[q] = w[R^m q] (m = 1..3,
// R (r, c) -> (c, n - 1 - r)) or nq = 7, adding Q_m[q] = w[T R^m q]
// (m = 0..3, T (r, c) -> (c, r)), q_plane apart: pixel s of w goes to
// R^-m s and R^-m T s.
// grid (ceil(n/32), ceil(n/32), G), block (32, 32)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(1024) void k_warp_fwd(Geo<T> g, const GateMotion<T>* __restrict__ gm,
                                                  int gate0, const float* __restrict__ field,
                                                  long field_stride, long plane_stride,
                                                  const T* __restrict__ x, long x_stride,
                                                  T* __restrict__ wP, T* __restrict__ wTP,
                                                  long w_stride, const SlotInfo* __restrict__ slots,
                                                  T* __restrict__ wQ, long q_stride, long q_plane, int nq) {
  __shared__ T tile[32][33];
  const int gate = slot_gate(slots, gate0);
  const int slice = slots ? slots[blockIdx.z].slice : (int)blockIdx.z;
  const GateMotion<T> M = gm[gate];
  const int n = g.n, pitch = g.pitch;
  const long origin = (long)kPad * pitch + kPad;
  const float* ux = field + gate * field_stride + origin;
  const float* uy = ux + plane_stride;
  const T* src = x + slice * x_stride;
  T* dst = wP + blockIdx.z * w_stride + origin;
  T* dstT = wTP ? wTP + blockIdx.z * w_stride + origin : nullptr;
  const int c = blockIdx.x * 32 + threadIdx.x;
  {
    const int r = blockIdx.y * 32 + threadIdx.y;
    T v = T(0);
    if (r < n && c < n) {
      if (M.kind == 0) {
        v = src[(long)r * n + c];
      } else {
        const Tap<T> tp = motion_tap(M, ux, uy, pitch, g.hc, r, c);
        const T fx = tp.fx, fy = tp.fy;
        const int c0 = tp.c0, r0 = tp.r0;
        const T w00 = (T(1) - fx) * (T(1) - fy), w01 = fx * (T(1) - fy);
        const T w10 = (T(1) - fx) * fy, w11 = fx * fy;
        const bool cin0 = (unsigned)c0 < (unsigned)n, cin1 = (unsigned)(c0 + 1) < (unsigned)n;
        const bool rin0 = (unsigned)r0 < (unsigned)n, rin1 = (unsigned)(r0 + 1) < (unsigned)n;
        // the four loads are unconditional (indices clamped into the image) so
        // that they are in flight together; taps outside the image weigh 0
        const long ra = (long)min(max(r0, 0), n - 1) * n, rb = (long)min(max(r0 + 1, 0), n - 1) * n;
        const int ca = min(max(c0, 0), n - 1), cb = min(max(c0 + 1, 0), n - 1);
        const T v00 = src[ra + ca], v01 = src[ra + cb], v10 = src[rb + ca], v11 = src[rb + cb];
        T acc = T(0);
        acc = fmaT((rin0 && cin0) ? w00 : T(0), v00, acc);
        acc = fmaT((rin0 && cin1) ? w01 : T(0), v01, acc);
        acc = fmaT((rin1 && cin0) ? w10 : T(0), v10, acc);
        acc = fmaT((rin1 && cin1) ? w11 : T(0), v11, acc);
        v = acc;
      }
      dst[(long)r * pitch + c] = v;
      // quarter-turn planes P_m[q] = w[R^m q], R (r, c) -> (c, n - 1 - r):
      // P_2 takes w(r, c) at (n - 1 - r, n - 1 - c); Q_1 at (n - 1 - r, c),
      // Q_3 at (r, n - 1 - c)
      if (wQ) {
        T* q = wQ + blockIdx.z * q_stride + origin;
        q[q_plane + (long)(n - 1 - r) * pitch + (n - 1 - c)] = v;
        if (nq == 7) {
          q[4 * q_plane + (long)(n - 1 - r) * pitch + c] = v;
          q[6 * q_plane + (long)r * pitch + (n - 1 - c)] = v;
        }
      }
    }
    tile[threadIdx.y][threadIdx.x] = v;
  }
  __syncthreads();
  // transposed store: thread (tx, ty) writes column blockIdx.x*32 + ty, rows along tx
  const int cc = blockIdx.x * 32 + threadIdx.y;
  const int rr = blockIdx.y * 32 + threadIdx.x;
  if (cc < n && rr < n) {
    const T v = tile[threadIdx.x][threadIdx.y];  // w(rr, cc)
    if (wTP) dstT[(long)cc * pitch + rr] = v;
    if (wQ) {  // P_1 takes it at (n - 1 - cc, rr), P_3 at (cc, n - 1 - rr)
      T* q = wQ + blockIdx.z * q_stride + origin;
      q[(long)(n - 1 - cc) * pitch + rr] = v;
      q[2 * q_plane + (long)cc * pitch + (n - 1 - rr)] = v;
      if (nq == 7) {  // Q_0 at (cc, rr), Q_2 at (n - 1 - cc, n - 1 - rr)
        q[3 * q_plane + (long)cc * pitch + rr] = v;
        q[5 * q_plane + (long)(n - 1 - cc) * pitch + (n - 1 - rr)] = v;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// a2 (+ a3): Joseph forward projection of the padded image, one thread per
// ray; the lanes of a wave are adjacent detector bins of one angle, so each
// line's two taps are read along a contiguous run of the (row-major or
// transposed) padded image. Mode 0 writes the sinogram; mode 1 fuses the
// dual step of Algorithm 1 (ii):
//   y' = (y + sigma (A_i x - d)) / (1 + sigma N / 2),  dy = y' - y
// grid (ceil(n_det/256), angles, G), block 256; angle k0 + blockIdx.y
// ---------------------------------------------------------------------------
template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_joseph_fwd(Geo<T> g, const AngleT<T>* __restrict__ ang,
                                                    const T* __restrict__ wP,
                                                    const T* __restrict__ wTP, long w_stride,
                                                    T* __restrict__ out, long out_stride,
                                                    int gate0, const GateScalars<T>* __restrict__ gs,
                                                    const GatePtrs<T>* __restrict__ gp,
                                                    const SlotInfo* __restrict__ slots, int k0) {
  __shared__ int s_lo, s_hi;
  const int k = k0 + blockIdx.y;
  const int j = blockIdx.x * 256 + threadIdx.x;
  const AngleT<T> A = ang[k];
  const int n = g.n, pitch = g.pitch;
  const bool live = j < g.nd;
  const T t = T(j) - g.jc;
  if (threadIdx.x == 0) {
    s_lo = n;
    s_hi = -1;
  }
  __syncthreads();
  if (live) {
    // lines where the crossing lies in (-1, n): cf(u) = t a + hc + u beta
    const float ta = float(t) * float(A.a) + float(g.hc);
    const float bt = float(A.beta);
    int lo = 0, hi = n - 1;
    if (fabsf(bt) < 1e-12f) {
      if (!(ta > -1.0f && ta < float(n))) {
        lo = n;
        hi = -1;
      }
    } else {
      const float u1 = (-1.0f - ta) / bt, u2 = (float(n) - ta) / bt;
      // clamp before the integer conversion (nearly axis-parallel rays give huge values)
      const float l1 = fminf(fmaxf(fminf(u1, u2) + float(g.hc), -4.0f), float(n + 4));
      const float l2 = fminf(fmaxf(fmaxf(u1, u2) + float(g.hc), -4.0f), float(n + 4));
      lo = max(0, (int)floorf(l1) - 2);
      hi = min(n - 1, (int)ceilf(l2) + 2);
    }
    if (lo <= hi) {
      atomicMin(&s_lo, lo);
      atomicMax(&s_hi, hi);
    }
  }
  __syncthreads();
  const int lo = s_lo, hi = s_hi;
  const T* img = (A.rows ? wP : wTP) + blockIdx.z * w_stride + (long)kPad * pitch + kPad;
  // two-level sum (blocks of kLineBlock lines) keeps the float32 rounding of
  // long ray sums close to that of a single block
  T acc = T(0);
  for (int L0 = lo; L0 <= hi; L0 += kLineBlock) {
    const int L1 = min(L0 + kLineBlock, hi + 1);
    T blk = T(0);
    for (int L = L0; L < L1; ++L) {
      const T gl = fmaT(T(L) - g.hc, A.beta, g.hc);
      T cf = fmaT(t, A.a, gl);
      cf = fmin(fmax(cf, T(-1)), T(n));
      const T c0 = floor(cf);
      const T f = cf - c0;
      const T* p = img + (long)L * pitch + (int)c0;
      blk += (T(1) - f) * p[0] + f * p[1];
    }
    acc += blk;
  }
  if (!live) return;
  const T s = A.ds * acc;
  const long idx = (long)k * g.nd + j;
  project_epilogue<T, MODE>(s, idx, out + blockIdx.z * out_stride, slot_gate(slots, gate0), gs, gp);
}

// ---------------------------------------------------------------------------
// a4: exact-transpose Joseph backprojection, one thread per pixel. For each
// angle the pixel receives from the (at most 2) rays whose line crossing lies
// within one pixel of it; the three candidates around the nearest bin are
// weighted with the same crossing the forward kernel computes, so the matrix
// entries are the forward's. Output into the interior of a padded image (or
// an unpadded image when `padded` is 0).
// grid (ceil(n/16), ceil(n/16), G), block (16, 16)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_joseph_adj(Geo<T> g, const AngleT<T>* __restrict__ ang,
                                                    const T* __restrict__ sino, long sino_stride,
                                                    T* __restrict__ out, long out_stride,
                                                    int padded, AngleRanges ar) {
  const int c = blockIdx.x * 16 + threadIdx.x;
  const int r = blockIdx.y * 16 + threadIdx.y;
  if (c >= g.n || r >= g.n) return;
  const T* s = sino + blockIdx.z * sino_stride;
  const T xc = T(c) - g.hc, yr = T(r) - g.hc;
  const T fc = T(c), fr = T(r);
  const int nd = g.nd;
  T acc = T(0), blk = T(0);
  for (int part = 0; part < 2; ++part)
  for (int k = part ? ar.kc : ar.ka; k < (part ? ar.kd : ar.kb); ++k) {
    if ((k & (kLineBlock - 1)) == 0) {  // two-level sum over angles
      acc += blk;
      blk = T(0);
    }
    const AngleT<T> A = ang[k];
    const T uline = A.rows ? yr : xc;
    const T pos = A.rows ? fc : fr;
    const T gl = fmaT(uline, A.beta, g.hc);
    const T u = fmaT(pos - gl, A.ia, g.jc);
    const int m = (int)rint(u);
    const T* srow = s + (long)k * nd;
    T part = T(0);
#pragma unroll
    for (int dj = -1; dj <= 1; ++dj) {
      const int j = m + dj;
      const T t = T(j) - g.jc;
      const T cf = fmaT(t, A.a, gl);
      const T w = fmax(T(0), T(1) - fabs(cf - pos));
      const bool ok = (unsigned)j < (unsigned)nd;
      const T v = srow[ok ? j : 0];
      part = fmaT(ok ? w : T(0), v, part);
    }
    blk = fmaT(A.ds, part, blk);
  }
  acc += blk;
  if (padded)
    out[blockIdx.z * out_stride + (long)(r + kPad) * g.pitch + (c + kPad)] = acc;
  else
    out[blockIdx.z * out_stride + (long)r * g.n + c] = acc;
}

// ---------------------------------------------------------------------------
// a2 (+ a3), float32: Joseph forward projection with fixed-point crossings.
// One thread per ray; the lanes of a wave are adjacent bins of one angle and
// walk the lines together, so the two taps of each line are read along a
// contiguous run of the padded image (its transpose for column stepping).
// Modes as in k_joseph_fwd.  grid (ceil(n_det/256), angles, G), block 256; angle k0 + blockIdx.y
// ---------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(256) void k_joseph_fwd_fx(Geo<float> g, const AngleFx* __restrict__ ang,
                                                       const float* __restrict__ wP,
                                                       const float* __restrict__ wTP, long w_stride,
                                                       float* __restrict__ out, long out_stride, int gate0,
                                                       const GateScalars<float>* __restrict__ gs,
                                                       const GatePtrs<float>* __restrict__ gp,
                                                       const SlotInfo* __restrict__ slots, int k0) {
  __shared__ int s_lo, s_hi;
  const int k = k0 + blockIdx.y;
  const int j = blockIdx.x * 256 + threadIdx.x;
  const AngleFx A = ang[k];
  const int n = g.n, pitch = g.pitch;
  const bool live = j < g.nd;
  if (threadIdx.x == 0) {
    s_lo = n;
    s_hi = -1;
  }
  __syncthreads();
  if (live) {
    // lines where the crossing lies in (-1, n): cf(L) = ta + hc + (L - hc) beta
    const float ta = (float(j) - g.jc) * A.a + g.hc;
    int lo = 0, hi = n - 1;
    if (fabsf(A.beta) < 1e-12f) {
      if (!(ta > -1.0f && ta < float(n))) {
        lo = n;
        hi = -1;
      }
    } else {
      const float u1 = (-1.0f - ta) / A.beta, u2 = (float(n) - ta) / A.beta;
      const float l1 = fminf(fmaxf(fminf(u1, u2) + g.hc, -4.0f), float(n + 4));
      const float l2 = fminf(fmaxf(fmaxf(u1, u2) + g.hc, -4.0f), float(n + 4));
      lo = max(0, (int)floorf(l1) - 2);
      hi = min(n - 1, (int)ceilf(l2) + 2);
    }
    if (lo <= hi) {
      atomicMin(&s_lo, lo);
      atomicMax(&s_hi, hi);
    }
  }
  __syncthreads();
  const int lo = s_lo, hi = s_hi;
  // wave-uniform start of the padded row (column -kPad), taps addressed by a
  // 32-bit byte offset: the loads use the scalar-base + vector-offset form
  const char* row = (const char*)((A.rows ? wP : wTP) + blockIdx.z * w_stride + (long)(kPad + lo) * pitch);
  const unsigned rowb = (unsigned)pitch * 4u;
  // the crossing is carried 2 columns to the right, so that one unsigned min
  // maps every tap left of column -1 or right of column n to the zero column n
  long long cf = A.C0 + (long long)j * A.A + (long long)lo * A.B + (2LL << 32);
  const unsigned cmax = (unsigned)(n + 2);
  float acc = 0.0f;
  int L0 = lo;
  // full blocks of kLineBlock lines: every tap of the block is loaded before
  // the first is used, so a wave keeps kLineBlock loads in flight. The sample
  // p0 + f (p1 - p0) is accumulated as sum p0 + 2^-32 sum F (p1 - p0) with
  // F = 2^32 f the raw fraction.
  for (; L0 + kLineBlock - 1 <= hi; L0 += kLineBlock) {
    float p0[kLineBlock], p1[kLineBlock], f[kLineBlock];
#pragma unroll
    for (int i = 0; i < kLineBlock; ++i) {
      const unsigned cc = min((unsigned)(cf >> 32), cmax);  // column + 2
      const unsigned off = (cc + (unsigned)(kPad - 2)) * 4u + (unsigned)i * rowb;
      f[i] = float((unsigned)cf);
      p0[i] = *(const float*)(row + off);
      p1[i] = *(const float*)(row + off + 4);
      cf += A.B;
    }
    float b0 = 0.0f, b1 = 0.0f;
#pragma unroll
    for (int i = 0; i < kLineBlock; ++i) {
      b0 += p0[i];
      b1 = fmaf(f[i], p1[i] - p0[i], b1);
    }
    acc += fmaf(b1, kFix, b0);
    row += (long)kLineBlock * rowb;
  }
  {
    float b0 = 0.0f, b1 = 0.0f;
    for (int L = L0; L <= hi; ++L) {
      const unsigned cc = min((unsigned)(cf >> 32), cmax);
      const unsigned off = (cc + (unsigned)(kPad - 2)) * 4u;
      const float f = float((unsigned)cf);
      const float p0 = *(const float*)(row + off), p1 = *(const float*)(row + off + 4);
      b0 += p0;
      b1 = fmaf(f, p1 - p0, b1);
      cf += A.B;
      row += rowb;
    }
    acc += fmaf(b1, kFix, b0);
  }
  if (!live) return;
  const float s = A.ds * acc;
  const long idx = (long)k * g.nd + j;
  project_epilogue<float, MODE>(s, idx, out + blockIdx.z * out_stride, slot_gate(slots, gate0), gs, gp);
}

// ---------------------------------------------------------------------------
// a4, float32: transpose of k_joseph_fwd_fx, one thread per pixel. For each
// angle the pixel's detector coordinate U (fixed point) gives the two bins
// j0 = floor(U), j0 + 1 and their weights 1 - |a| d and 1 - |a| (1 - d),
// d = frac(U): the hat weights of the forward seen from the pixel.
// grid (ceil(n/16), ceil(n/16), G), block (16, 16)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_joseph_adj_fx(Geo<float> g, const AngleFx* __restrict__ ang,
                                                       const float* __restrict__ sino, long sino_stride,
                                                       float* __restrict__ out, long out_stride, int padded,
                                                       AngleRanges ar) {
  const int c = blockIdx.x * 16 + threadIdx.x;
  const int r = blockIdx.y * 16 + threadIdx.y;
  if (c >= g.n || r >= g.n) return;
  const float* s = sino + blockIdx.z * sino_stride;
  const int nd = g.nd;
  float acc = 0.0f, blk = 0.0f;
  for (int part = 0; part < 2; ++part)
  for (int k = part ? ar.kc : ar.ka; k < (part ? ar.kd : ar.kb); ++k) {
    if ((k & (kLineBlock - 1)) == 0) {
      acc += blk;
      blk = 0.0f;
    }
    const AngleFx A = ang[k];
    const int line = A.rows ? r : c;
    const int pos = A.rows ? c : r;
    const long long u = A.U0 + (long long)pos * A.P + (long long)line * A.Q;
    const int j0 = (int)(u >> 32);
    const float d = float((unsigned)u) * kFix;
    const float w0 = fmaxf(0.0f, fmaf(-A.absa, d, 1.0f));
    const float w1 = fmaxf(0.0f, fmaf(A.absa, d, A.oma));
    const float* srow = s + (long)k * nd;
    const bool ok0 = (unsigned)j0 < (unsigned)nd, ok1 = (unsigned)(j0 + 1) < (unsigned)nd;
    const float y0 = srow[ok0 ? j0 : 0], y1 = srow[ok1 ? j0 + 1 : 0];
    const float part = fmaf(ok1 ? w1 : 0.0f, y1, (ok0 ? w0 : 0.0f) * y0);
    blk = fmaf(A.ds, part, blk);
  }
  acc += blk;
  if (padded)
    out[blockIdx.z * out_stride + (long)(r + kPad) * g.pitch + (c + kPad)] = acc;
  else
    out[blockIdx.z * out_stride + (long)r * g.n + c] = acc;
}

// ---------------------------------------------------------------------------
// a5 (+ a6): transposed warp as a gather, summed over G gates, fused with the
// dual-image updates of Algorithm 1 (iii) and the next primal step (i).
// Output pixel q receives from the pixels p of a (2R+1)^2 window around the
// inverse image of q; each candidate's weight on q is recomputed with the
// forward warp's arithmetic (motion_tap and the same products), so the
// result is the exact transpose. Candidates in the zero border of the padded
// input contribute zero.
//   mode 0: out = sum_g D_g^T b_g                       (plain adjoint)
//   mode 1: out += sum_g D_g^T b_g                      (accumulate)
//   mode 2: z += dz; zbar = z + sum_g coef_g dz_g; optionally x = (x - tau zbar) cx
// grid (ceil(n/32), ceil(n/8)), block (32, 8)
// ---------------------------------------------------------------------------
template <typename T>
struct UpdateArgs {
  T* x;
  T* z;
  T* zbar;
  T tau, cx;
  int do_x;
};

// With a slot table (batched SPDHG) block z handles slot z alone (G = 1): its
// gate, its slice's x, z, zbar (slice_stride apart), that slice's (tau, c_x)
// from slice_tc and the slot's do_x.
template <typename T, int MODE, int R>
__global__ __launch_bounds__(256) void k_twarp(Geo<T> g, const GateMotion<T>* __restrict__ gm,
                                               int gate0, int G,
                                               const GateScalars<T>* __restrict__ gs,
                                               const float* __restrict__ field, long field_stride,
                                               long plane_stride, const short2* __restrict__ centres,
                                               const T* __restrict__ bP, long b_stride,
                                               T* __restrict__ out, UpdateArgs<T> ua,
                                               const SlotInfo* __restrict__ slots, long slice_stride,
                                               const T* __restrict__ slice_tc) {
  // 32 x 8 tiles: each row of a tile is one 128-byte line of the images
  const int qc = blockIdx.x * 32 + threadIdx.x;
  const int qr = blockIdx.y * 8 + threadIdx.y;
  const int n = g.n, pitch = g.pitch;
  if (qc >= n || qr >= n) return;
  const long origin = (long)kPad * pitch + kPad;
  int slot0 = 0;
  if (slots) {
    const SlotInfo si = slots[blockIdx.z];
    slot0 = (int)blockIdx.z;
    gate0 = si.gate;
    G = 1;
    const long off = (long)si.slice * slice_stride;
    ua.x += off;
    ua.z += off;
    ua.zbar += off;
    ua.tau = slice_tc[2 * si.slice];
    ua.cx = slice_tc[2 * si.slice + 1];
    ua.do_x = si.do_x;
  }
  const long q = (long)qr * n + qc;
  // the update's inputs are loaded before the gathers, so that their latency
  // overlaps them (and x is not reloaded after the stores of z and z-bar)
  T z0 = T(0), x0 = T(0);
  if (MODE == 2) {
    z0 = ua.z[q];
    if (ua.do_x) x0 = ua.x[q];
  }
  T dz = T(0), dzb = T(0);
  for (int gi = 0; gi < G; ++gi) {
    const int gate = gate0 + gi;
    const GateMotion<T> M = gm[gate];
    const T* b = bP + (slot0 + gi) * b_stride + origin;
    T part = T(0);
    if (M.kind == 0) {
      part = b[(long)qr * pitch + qc];
    } else {
      // every load of the window is issued before any is used: the values of
      // b, and for a field the displacements, of the (2R+1)^2 candidates
      constexpr int K = (2 * R + 1) * (2 * R + 1);
      int cr, cc;
      window_centre(M, centres, gate, n, g.hc, qr, qc, cr, cc);
      const long o0 = (long)cr * pitch + cc;
      T bv[K], dxv[K], dyv[K];
#pragma unroll
      for (int t = 0; t < K; ++t) bv[t] = b[o0 + (long)(t / (2 * R + 1) - R) * pitch + (t % (2 * R + 1) - R)];
      if (M.kind == 2) {
        const float* ux = field + gate * field_stride + origin;
        const float* uy = ux + plane_stride;
#pragma unroll
        for (int t = 0; t < K; ++t) {
          const long o = o0 + (long)(t / (2 * R + 1) - R) * pitch + (t % (2 * R + 1) - R);
          dxv[t] = T(ux[o]);
          dyv[t] = T(uy[o]);
        }
      } else {
#pragma unroll
        for (int t = 0; t < K; ++t) {
          const T xc = T(cc + t % (2 * R + 1) - R) - g.hc, yc = T(cr + t / (2 * R + 1) - R) - g.hc;
          dxv[t] = fmaT(M.cm1, xc, fmaT(-M.sn, yc, M.tx));
          dyv[t] = fmaT(M.sn, xc, fmaT(M.cm1, yc, M.ty));
        }
      }
#pragma unroll
      for (int t = 0; t < K; ++t) {
        const Tap<T> tp = tap_from_displacement<T>(dxv[t], dyv[t], cr + t / (2 * R + 1) - R, cc + t % (2 * R + 1) - R);
        const T wx = (qc == tp.c0) ? (T(1) - tp.fx) : ((qc == tp.c0 + 1) ? tp.fx : T(0));
        const T wy = (qr == tp.r0) ? (T(1) - tp.fy) : ((qr == tp.r0 + 1) ? tp.fy : T(0));
        part = fmaT(wx * wy, bv[t], part);
      }
    }
    dz += part;
    if (MODE == 2) dzb = fmaT(gs[gate].coef, part, dzb);
  }
  if (MODE == 0) {
    out[q] = dz;
  } else if (MODE == 1) {
    out[q] += dz;
  } else {
    const T z = z0 + dz;
    const T zb = z + dzb;
    ua.z[q] = z;
    ua.zbar[q] = zb;
    if (ua.do_x) ua.x[q] = (x0 - ua.tau * zb) * ua.cx;
  }
}

// Algorithm 1 step (i) on its own: x = (x - tau zbar) cx.
template <typename T>
__global__ __launch_bounds__(256) void k_xstep(long count, T* __restrict__ x,
                                               const T* __restrict__ zbar, T tau, T cx) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i < count) x[i] = (x[i] - tau * zbar[i]) * cx;
}

// Step (i) for every slice of a batch: x = (x - tau zbar) c_x with the
// slice's (tau, c_x). grid (ceil(n*n/256), slices)
template <typename T>
__global__ __launch_bounds__(256) void k_xstep_batch(long count, T* __restrict__ x, const T* __restrict__ zbar,
                                                     const T* __restrict__ slice_tc) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  const long o = (long)blockIdx.y * count + i;
  const T tau = slice_tc[2 * blockIdx.y], cx = slice_tc[2 * blockIdx.y + 1];
  x[o] = (x[o] - tau * zbar[o]) * cx;
}

// Copy an unpadded image into the interior of a padded one (converting type).
template <typename Ts, typename Td>
__global__ __launch_bounds__(256) void k_to_padded(int n, int pitch, const Ts* __restrict__ src,
                                                   Td* __restrict__ dst) {
  const int c = blockIdx.x * 16 + threadIdx.x;
  const int r = blockIdx.y * 16 + threadIdx.y;
  if (c < n && r < n) dst[(long)(r + kPad) * pitch + c + kPad] = Td(src[(long)r * n + c]);
}

template <typename Ts, typename Td>
__global__ __launch_bounds__(256) void k_convert(long count, const Ts* __restrict__ src,
                                                 Td* __restrict__ dst) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i < count) dst[i] = Td(src[i]);
}

template <typename T>
__global__ __launch_bounds__(256) void k_scale(long count, T* __restrict__ v, double s) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i < count) v[i] = T(double(v[i]) * s);
}

// ---------------------------------------------------------------------------
// FP64 reductions, deterministic: a fixed grid of kRedBlocks blocks, each
// folding a fixed strided subset, then one block folding the partials in
// order. op 0: sum a^2; op 1: sum a b; op 2: sum (a - b)^2.
// ---------------------------------------------------------------------------
constexpr int kRedBlocks = 512;

__device__ __forceinline__ double block_sum(double v, double* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w];
  }
  return s;
}

template <typename Ta, typename Tb, int OP>
__global__ __launch_bounds__(256) void k_reduce_partial(long count, const Ta* __restrict__ a,
                                                        const Tb* __restrict__ b,
                                                        double* __restrict__ partial) {
  __shared__ double sh[4];
  double acc = 0.0;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < count; i += (long)kRedBlocks * 256) {
    const double va = double(a[i]);
    if (OP == 0) acc = __builtin_fma(va, va, acc);
    if (OP == 1) acc = __builtin_fma(va, double(b[i]), acc);
    if (OP == 2) {
      const double dd = va - double(b[i]);
      acc = __builtin_fma(dd, dd, acc);
    }
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Sums kRedBlocks partials in a fixed order into out[slot].
__global__ __launch_bounds__(256) void k_reduce_final(const double* __restrict__ partial,
                                                      double* __restrict__ out, int slot) {
  __shared__ double sh[4];
  double acc = 0.0;
  for (int i = threadIdx.x; i < kRedBlocks; i += 256) acc += partial[i];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) out[slot] = s;
}

// ---------------------------------------------------------------------------
// Set-up of the transposed warp for displacement fields: the centre of each
// output pixel's gather window (an estimate of phi^{-1}(q) by fixed-point
// iteration on the bilinearly interpolated field), then a verification that
// every nonzero forward weight falls inside its window (the largest Chebyshev
// distance found is returned through `need`).
// ---------------------------------------------------------------------------
__device__ __forceinline__ float field_at(const float* __restrict__ u, int n, int pitch, float x,
                                          float y) {
  x = fminf(fmaxf(x, 0.0f), float(n - 1));
  y = fminf(fmaxf(y, 0.0f), float(n - 1));
  const int c0 = min((int)x, n - 2 < 0 ? 0 : n - 2), r0 = min((int)y, n - 2 < 0 ? 0 : n - 2);
  const float fx = x - c0, fy = y - r0;
  const int c1 = min(c0 + 1, n - 1), r1 = min(r0 + 1, n - 1);
  const float v00 = u[(long)r0 * pitch + c0], v01 = u[(long)r0 * pitch + c1];
  const float v10 = u[(long)r1 * pitch + c0], v11 = u[(long)r1 * pitch + c1];
  return (1 - fy) * ((1 - fx) * v00 + fx * v01) + fy * ((1 - fx) * v10 + fx * v11);
}

__global__ __launch_bounds__(256) void k_field_centres(int n, int pitch, const float* __restrict__ fieldP,
                                                       long plane_stride, short2* __restrict__ centres) {
  const int qc = blockIdx.x * 16 + threadIdx.x;
  const int qr = blockIdx.y * 16 + threadIdx.y;
  if (qc >= n || qr >= n) return;
  const long origin = (long)kPad * pitch + kPad;
  const float* ux = fieldP + origin;
  const float* uy = ux + plane_stride;
  float vx = float(qc) - ux[(long)qr * pitch + qc];
  float vy = float(qr) - uy[(long)qr * pitch + qc];
  for (int it = 0; it < 12; ++it) {
    const float nx = float(qc) - field_at(ux, n, pitch, vx, vy);
    const float ny = float(qr) - field_at(uy, n, pitch, vx, vy);
    vx = nx;
    vy = ny;
  }
  int cc = (int)rintf(fminf(fmaxf(vx, -1.0f), float(n)));
  int cr = (int)rintf(fminf(fmaxf(vy, -1.0f), float(n)));
  centres[(long)qr * n + qc] = make_short2((short)cc, (short)cr);
}

template <typename T>
__global__ __launch_bounds__(256) void k_window_check(Geo<T> g, const GateMotion<T>* __restrict__ gm,
                                                      int gate, const float* __restrict__ field,
                                                      long field_stride, long plane_stride,
                                                      const short2* __restrict__ centres,
                                                      int* __restrict__ need) {
  const int c = blockIdx.x * 16 + threadIdx.x;
  const int r = blockIdx.y * 16 + threadIdx.y;
  const int n = g.n, pitch = g.pitch;
  if (c >= n || r >= n) return;
  const GateMotion<T> M = gm[gate];
  if (M.kind == 0) return;
  const long origin = (long)kPad * pitch + kPad;
  const float* ux = field + gate * field_stride + origin;
  const float* uy = ux + plane_stride;
  const Tap<T> tp = motion_tap(M, ux, uy, pitch, g.hc, r, c);
  const T fx = tp.fx, fy = tp.fy;
  const int c0 = tp.c0, r0 = tp.r0;
  int worst = 0;
  for (int a = 0; a < 2; ++a) {
    for (int bb = 0; bb < 2; ++bb) {
      const int qr = r0 + a, qc = c0 + bb;
      if ((unsigned)qr >= (unsigned)n || (unsigned)qc >= (unsigned)n) continue;
      const T wx = bb ? fx : T(1) - fx;
      const T wy = a ? fy : T(1) - fy;
      if (wx * wy == T(0)) continue;
      int cr, cc;
      window_centre(M, centres, gate, n, g.hc, qr, qc, cr, cc);
      worst = max(worst, max(abs(c - cc), abs(r - cr)));
    }
  }
  if (worst > 0) atomicMax(need, worst);
}

}  // namespace mcr
