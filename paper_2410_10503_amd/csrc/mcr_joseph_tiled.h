// LDS-tiled float32 Joseph projector pair (gfx950). Same fixed-point geometry
// as k_joseph_fwd_fx / k_joseph_adj_fx (AngleFx), different work split:
//
//  forward  - a block owns consecutive angles of one stepping type times a
//             tile of detector bins and walks the lines in bands. Each band of
//             the padded image is staged once in LDS as a window that follows
//             the rays' slope (k_joseph_fwd_lds / _sched: integer shear per
//             line; k_joseph_fwd_shear: per-line shift from the chunk's mean
//             fixed-point slope, host-scheduled pieces) and read by all the
//             block's rays; the LDS index of a tap is the integer part of the
//             ray's fixed-point crossing, so a sample costs a 64-bit add, one
//             conversion, one LDS read and two FMAs.
//  adjoint  - a block owns a 32-row x 8*PX-column pixel tile and a share of
//             the angles (S shares in total). Chunks of KC angles of the
//             sinogram are staged in LDS (bin window per angle, pre-scaled by
//             the ray length per line), and each thread accumulates PX pixels
//             along a row from the two bins around each pixel's fixed-point
//             detector coordinate.
#pragma once

#include "mcr_kernels.h"

namespace mcr {

constexpr int kFwdMaxBand = 32;

// grid (ceil(n_det/JD), n_chunks, G), block KA*JD (= 256)
template <int KA, int JD, int WL, int MODE>
__global__ __launch_bounds__(256) void k_joseph_fwd_lds(Geo<float> g, const AngleFx* __restrict__ ang,
                                                        const int2* __restrict__ chunks,
                                                        const float* __restrict__ wP,
                                                        const float* __restrict__ wTP, long w_stride,
                                                        float* __restrict__ out, long out_stride, int gate0,
                                                        const GateScalars<float>* __restrict__ gs,
                                                        const GatePtrs<float>* __restrict__ gp,
                                                        const SlotInfo* __restrict__ slots) {
  static_assert(KA * JD == 256, "one ray per thread");
  __shared__ float st[kFwdMaxBand * WL];
  __shared__ int s_lo, s_hi;
  __shared__ int s_min[6], s_max[6];
  __shared__ int s_S0, s_BL, s_W;
  const int tid = threadIdx.x;
  const int2 ch = chunks[blockIdx.y];
  const int kk = tid / JD, jj = tid % JD;
  const int j_first = blockIdx.x * JD;
  const int j_last = min(j_first + JD - 1, g.nd - 1);
  const int j = j_first + jj;
  const bool live = kk < ch.y && j < g.nd;
  const int k = ch.x + min(kk, ch.y - 1);
  const AngleFx A = ang[k];
  const int n = g.n, pitch = g.pitch;
  const int rows = ang[ch.x].rows;
  const int m = (int)rintf(ang[ch.x + (ch.y >> 1)].beta);  // integer shear of the window
  if (tid == 0) {
    s_lo = n;
    s_hi = -1;
  }
  if (tid < 6) {
    s_min[tid] = 0x7fffffff;
    s_max[tid] = -0x7fffffff;
  }
  __syncthreads();
  if (live) {
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
  const float* img = (rows ? wP : wTP) + blockIdx.z * w_stride + (long)kPad * pitch + kPad;
  const long long cfj = A.C0 + (long long)j * A.A;            // crossing at line 0
  const long long step = A.B + ((long long)(WL - m) << 32);   // next line, next LDS row
  float acc = 0.0f;
  for (int L0 = lo; L0 <= hi; L0 += s_BL) {
    // window of the band: for band lengths 32, 16, ..., 1 the extreme sheared
    // columns over the corner rays (first/last bin of each angle, first/last line)
    if (tid < 2 * KA) {
      const int a = tid >> 1;
      if (a < ch.y) {
        const AngleFx C = ang[ch.x + a];
        const long long c0 = C.C0 + (long long)((tid & 1) ? j_last : j_first) * C.A + (long long)L0 * C.B;
        const int v0 = (int)(c0 >> 32);
        for (int b = 0, bl = kFwdMaxBand; b < 6; ++b, bl >>= 1) {
          const int v1 = (int)((c0 + (long long)(bl - 1) * C.B) >> 32) - (bl - 1) * m;
          atomicMin(&s_min[b], min(v0, v1));
          atomicMax(&s_max[b], max(v0, v1));
        }
      }
    }
    __syncthreads();
    if (tid == 0) {
      int b = 0, bl = kFwdMaxBand;
      while (b < 5 && s_max[b] - s_min[b] + 3 > WL) {
        ++b;
        bl >>= 1;
      }
      s_BL = min(bl, hi - L0 + 1);
      s_S0 = s_min[b] - 1;
      s_W = s_max[b] - s_min[b] + 3;
    }
    __syncthreads();
    const int BL = s_BL, S0 = s_S0, W = s_W;
    if (tid < 6) {
      s_min[tid] = 0x7fffffff;
      s_max[tid] = -0x7fffffff;
    }
    // stage the sheared window (zero outside the image)
    for (int i = tid; i < BL * WL; i += 256) {
      const int l = i / WL, q = i % WL;
      if (q < W) {
        const int c = S0 + l * m + q;
        st[i] = ((unsigned)c < (unsigned)n) ? img[(long)(L0 + l) * pitch + c] : 0.0f;
      }
    }
    __syncthreads();
    if (live) {
      long long cf = cfj + (long long)L0 * A.B - ((long long)S0 << 32);
      float b0 = 0.0f, b1 = 0.0f;
      for (int l = 0; l < BL; ++l) {
        const int idx = (int)(cf >> 32);
        const float fl = float((unsigned)cf);
        const float p0 = st[idx], p1 = st[idx + 1];
        b0 += p0;
        b1 = fmaf(fl, p1 - p0, b1);
        cf += step;
      }
      acc += fmaf(b1, kFix, b0);
    }
    __syncthreads();
  }
  if (!live) return;
  const float s = A.ds * acc;
  const long idx = (long)k * g.nd + j;
  project_epilogue<float, MODE>(s, idx, out + blockIdx.z * out_stride, slot_gate(slots, gate0), gs, gp);
}

// Scheduled variant of the tiled forward: the line bands of every block, with
// their sheared LDS windows, are computed on the host (exact integer
// arithmetic on the same AngleFx constants); the kernel only streams them. The
// next band is loaded into registers while the current one is computed.
//   chunk  : (first angle, angle count, shear m, -)
//   blocks : per (chunk, detector tile): (first band, band count)
//   bands  : (first line L0, lines BL, window start S0, window width W); every
//            tap of every ray of the block lies in window columns [1, W - 2]
// grid (ceil(n_det/JD), n_chunks, G), block 256
template <int KA, int JD, int WL, int MODE>
__global__ __launch_bounds__(256) void k_joseph_fwd_sched(Geo<float> g, const AngleFx* __restrict__ ang,
                                                          const int4* __restrict__ chunks,
                                                          const int2* __restrict__ blocks,
                                                          const int4* __restrict__ bands,
                                                          const float* __restrict__ wP,
                                                          const float* __restrict__ wTP, long w_stride,
                                                          float* __restrict__ out, long out_stride, int gate0,
                                                          const GateScalars<float>* __restrict__ gs,
                                                          const GatePtrs<float>* __restrict__ gp,
                                                          const SlotInfo* __restrict__ slots) {
  static_assert(KA * JD == 256, "one ray per thread");
  constexpr int kPer = kFwdMaxBand * WL / 256;
  __shared__ float st[kFwdMaxBand * WL];
  const int tid = threadIdx.x;
  const int4 ch = chunks[blockIdx.y];
  const int2 bb = blocks[blockIdx.y * gridDim.x + blockIdx.x];
  const int kk = tid / JD, jj = tid % JD;
  const int j = blockIdx.x * JD + jj;
  const bool live = kk < ch.y && j < g.nd;
  const int k = ch.x + min(kk, ch.y - 1);
  const AngleFx A = ang[k];
  const int n = g.n, pitch = g.pitch, m = ch.z;
  const float* img = (ang[ch.x].rows ? wP : wTP) + blockIdx.z * w_stride + (long)kPad * pitch + kPad;
  const long long cfj = A.C0 + (long long)j * A.A;
  const long long step = A.B + ((long long)(WL - m) << 32);
  float pre[kPer];
  auto fetch = [&](const int4 bd) {
#pragma unroll
    for (int e = 0; e < kPer; ++e) {
      const int i = tid + e * 256;
      const int l = i / WL, q = i % WL;
      float v = 0.0f;
      if (l < bd.y && q < bd.w) {
        const int c = bd.z + l * m + q;
        if ((unsigned)c < (unsigned)n) v = img[(long)(bd.x + l) * pitch + c];
      }
      pre[e] = v;
    }
  };
  if (bb.y > 0) fetch(bands[bb.x]);
  float acc = 0.0f;
  for (int b = 0; b < bb.y; ++b) {
    const int4 bd = bands[bb.x + b];
#pragma unroll
    for (int e = 0; e < kPer; ++e) st[tid + e * 256] = pre[e];
    __syncthreads();
    if (b + 1 < bb.y) fetch(bands[bb.x + b + 1]);
    if (live) {
      long long cf = cfj + (long long)bd.x * A.B - ((long long)bd.z << 32);
      float b0 = 0.0f, b1 = 0.0f;
      for (int l = 0; l < bd.y; ++l) {
        const float* q = st + (int)(cf >> 32);
        const float fl = float((unsigned)cf);
        const float p0 = q[0];
        b0 += p0;
        b1 = fmaf(fl, q[1] - p0, b1);
        cf += step;
      }
      acc += fmaf(b1, kFix, b0);
    }
    __syncthreads();
  }
  if (!live) return;
  const float s = A.ds * acc;
  const long idx = (long)k * g.nd + j;
  project_epilogue<float, MODE>(s, idx, out + blockIdx.z * out_stride, slot_gate(slots, gate0), gs, gp);
}

// Line-sheared scheduled forward. A block owns up to 16 consecutive angles of
// one stepping type times 32 detector bins; thread (kk, jj) computes the rays
// of angles kk and kk + 8 at bin jj, so every staged value serves two rays
// per thread. Band lines are staged one per wave (64 columns each) with a
// per-line shift o_l = floor(l Bm / 2^32), Bm the fixed-point slope of the
// chunk's middle angle: the window follows the mean ray direction, so its
// width is set by the spread of the block's rays on one line (about 50
// columns at 720 angles). The LDS line pitch is a power of two >= 64 chosen
// per band (wide windows get fewer lines), at most kShCap entries. Each staged entry holds
// the pixel and its difference to the next column, (x[c], x[c+1] - x[c]), so
// a tap is one 8-byte LDS read and two FMAs. The ray position is carried as
// two 32-bit words (window column, fraction) of the 32.32 crossing; the LDS
// address is the column word shifted plus a block-uniform line offset.
// Staged columns are clamped into the zero halo of the padded image, so no
// per-lane bounds test is needed.
// The bands of a (chunk, detector tile) unit are split into pieces of about
// kShPieceLines lines, one block each, so that blocks carry similar work. A
// unit of P > 1 pieces writes P partial sums per ray, which
// k_joseph_fwd_shear_finish adds in piece order before the epilogue.
//   chunks : (first angle, angle count, low and high words of Bm)
//   pieces : per block: (first band, band count, unit, piece index)
//   units  : (chunk, detector tile, pieces P, offset of the unit's P x 512
//            partial sums in part)
//   bands  : (first line L0, lines BL, window start S0, log2 pitch lp); the
//            taps of every ray of the block on band line l lie in window
//            columns [1, 2^lp - 2] after the shift o_l, BL 2^lp <= kShCap
// grid (pieces, 1, G), block 256; piece piece0 + blockIdx.x
constexpr int kShCap = 2048;  // staged entries per band
constexpr int kShPieceLines = 128;  // target lines per block
constexpr int kShBL = 32;     // lines per band at most
constexpr int kShKA = 16;  // angles per chunk at most
constexpr int kShJD = 32;  // detector bins per block

template <int MODE>
__global__ __launch_bounds__(256) void k_joseph_fwd_shear(Geo<float> g, const AngleFx* __restrict__ ang,
                                                          const int4* __restrict__ chunks,
                                                          const int4* __restrict__ pieces,
                                                          const int4* __restrict__ units,
                                                          const int4* __restrict__ bands,
                                                          const float* __restrict__ wP,
                                                          const float* __restrict__ wTP, long w_stride,
                                                          float* __restrict__ out, long out_stride, int gate0,
                                                          const GateScalars<float>* __restrict__ gs,
                                                          const GatePtrs<float>* __restrict__ gp,
                                                          const SlotInfo* __restrict__ slots,
                                                          float* __restrict__ part, long part_stride, int piece0) {
  constexpr int kPer = kShCap / 256;  // staged entries per thread
  __shared__ float2 st[kShCap];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int4 pc = pieces[piece0 + blockIdx.x];
  const int4 un = units[pc.z];
  const int4 ch = chunks[un.x];
  const long long Bm = (long long)(((unsigned long long)(unsigned)ch.w << 32) | (unsigned)ch.z);
  const int2 bb = make_int2(pc.x, pc.y);
  const int kk = tid >> 5;
  const int j = un.y * kShJD + (tid & 31);
  const int jc = min(j, g.nd - 1);
  const AngleFx& A0 = ang[ch.x + min(kk, ch.y - 1)];
  const AngleFx& A1 = ang[ch.x + min(kk + 8, ch.y - 1)];
  // per-line steps of the crossings
  const unsigned long long S0 = (unsigned long long)A0.B;
  const unsigned long long S1 = (unsigned long long)A1.B;
  const unsigned s0lo = (unsigned)S0, s0hi = (unsigned)(S0 >> 32);
  const unsigned s1lo = (unsigned)S1, s1hi = (unsigned)(S1 >> 32);
  const long long c0j = A0.C0 + (long long)jc * A0.A;
  const long long c1j = A1.C0 + (long long)jc * A1.A;
  const int n = g.n, pitch = g.pitch;
  const float* img = (ang[ch.x].rows ? wP : wTP) + blockIdx.z * w_stride + (long)kPad * pitch + kPad;
  float pre[kPer], prd[kPer];
  // entry i = l * pitch + q of a band; a wave's 64 entries share one line
  auto fetch = [&](const int4 bd) {
#pragma unroll
    for (int e = 0; e < kPer; ++e) {
      const int ib = 256 * e + 64 * wv;
      const int l = ib >> bd.w;
      float v = 0.0f, v1 = 0.0f;
      if (l < bd.y) {
        const int o = (int)(((long long)l * Bm) >> 32);
        // column + kPad, clamped into the padded row [0, n + 2 kPad - 1]; its
        // right neighbour is read unclamped: past the row's right halo it is
        // the next padded row's left halo (or a bottom padding row), zero too
        const float* row = img - kPad + (long)(bd.x + l) * pitch;
        const unsigned i =
            (unsigned)min(max(bd.z + o + (ib & ((1 << bd.w) - 1)) + lane + kPad, 0), n + 2 * kPad - 1);
        const float* q = row + i;
        v = q[0];
        v1 = q[1];
      }
      pre[e] = v;
      prd[e] = v1 - v;
    }
  };
  // crossings of both rays on the piece's first line, relative to the first
  // band's window; the bands of a piece are consecutive lines, so at a band
  // change only the window start moves
  unsigned lo0 = 0, hi0 = 0, lo1 = 0, hi1 = 0;
  int s_prev = 0;
  if (bb.y > 0) {
    const int4 bd = bands[bb.x];
    fetch(bd);
    const unsigned long long p0 = (unsigned long long)(c0j + (long long)bd.x * A0.B - ((long long)bd.z << 32));
    const unsigned long long p1 = (unsigned long long)(c1j + (long long)bd.x * A1.B - ((long long)bd.z << 32));
    lo0 = (unsigned)p0;
    hi0 = (unsigned)(p0 >> 32);
    lo1 = (unsigned)p1;
    hi1 = (unsigned)(p1 >> 32);
    s_prev = bd.z;
  }
  float acc0 = 0.0f, acc1 = 0.0f;
  for (int b = 0; b < bb.y; ++b) {
    const int4 bd = bands[bb.x + b];
#pragma unroll
    for (int e = 0; e < kPer; ++e) st[256 * e + tid] = make_float2(pre[e], prd[e]);
    __syncthreads();
    if (b + 1 < bb.y) fetch(bands[bb.x + b + 1]);
    hi0 += (unsigned)(s_prev - bd.z);
    hi1 += (unsigned)(s_prev - bd.z);
    s_prev = bd.z;
    long long om = 0;
    float a0 = 0.0f, f0 = 0.0f, a1 = 0.0f, f1 = 0.0f;
    const char* base = (const char*)st;
    // the tap pair of both rays on the current line; so = 8 (l pitch - o_l)
    // >= 0 is the byte offset of line l's window (uniform)
    auto tap = [&](int so, float2& x0, float& w0, float2& x1, float& w1) {
      x0 = *(const float2*)(base + ((hi0 << 3) + (unsigned)so));
      x1 = *(const float2*)(base + ((hi1 << 3) + (unsigned)so));
      w0 = float(lo0);
      w1 = float(lo1);
      unsigned c0, c1;
      lo0 = __builtin_addc(lo0, s0lo, 0u, &c0);
      hi0 = __builtin_addc(hi0, s0hi, c0, &c0);
      lo1 = __builtin_addc(lo1, s1lo, 0u, &c1);
      hi1 = __builtin_addc(hi1, s1hi, c1, &c1);
    };
    int l = 0;
    for (; l + 4 <= bd.y; l += 4) {
      float2 x0[4], x1[4];
      float w0[4], w1[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int so = 8 * (((l + t) << bd.w) - (int)(om >> 32));
        om += Bm;
        tap(so, x0[t], w0[t], x1[t], w1[t]);
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        a0 += x0[t].x;
        f0 = fmaf(w0[t], x0[t].y, f0);
        a1 += x1[t].x;
        f1 = fmaf(w1[t], x1[t].y, f1);
      }
    }
    for (; l < bd.y; ++l) {
      float2 x0, x1;
      float w0, w1;
      const int so = 8 * ((l << bd.w) - (int)(om >> 32));
      om += Bm;
      tap(so, x0, w0, x1, w1);
      a0 += x0.x;
      f0 = fmaf(w0, x0.y, f0);
      a1 += x1.x;
      f1 = fmaf(w1, x1.y, f1);
    }
    acc0 += fmaf(f0, kFix, a0);
    acc1 += fmaf(f1, kFix, a1);
    __syncthreads();
  }
  if (un.z > 1) {  // partial sums; k_joseph_fwd_shear_finish adds them
    float* pu = part + blockIdx.z * part_stride + un.w + pc.w * 512;
    pu[tid] = acc0;
    pu[256 + tid] = acc1;
    return;
  }
  if (j >= g.nd) return;
  const int gate = slot_gate(slots, gate0);
  float* o = out + blockIdx.z * out_stride;
  if (kk < ch.y) project_epilogue<float, MODE>(A0.ds * acc0, (long)(ch.x + kk) * g.nd + j, o, gate, gs, gp);
  if (kk + 8 < ch.y)
    project_epilogue<float, MODE>(A1.ds * acc1, (long)(ch.x + kk + 8) * g.nd + j, o, gate, gs, gp);
}

// Sum of the partial sums of the multi-piece units in piece order, then the
// projection epilogue. grid (count, 1, G), block 256; multi lists the units
// with P > 1, this launch handles entries multi0 .. multi0 + count - 1.
template <int MODE>
__global__ __launch_bounds__(256) void k_joseph_fwd_shear_finish(Geo<float> g, const AngleFx* __restrict__ ang,
                                                                 const int4* __restrict__ chunks,
                                                                 const int4* __restrict__ units,
                                                                 const int* __restrict__ multi,
                                                                 const float* __restrict__ part, long part_stride,
                                                                 float* __restrict__ out, long out_stride, int gate0,
                                                                 const GateScalars<float>* __restrict__ gs,
                                                                 const GatePtrs<float>* __restrict__ gp,
                                                                 const SlotInfo* __restrict__ slots, int multi0) {
  const int tid = threadIdx.x;
  const int4 un = units[multi[multi0 + blockIdx.x]];
  const int4 ch = chunks[un.x];
  const int kk = tid >> 5;
  const int j = un.y * kShJD + (tid & 31);
  if (j >= g.nd) return;
  const float* pu = part + blockIdx.z * part_stride + un.w;
  float acc0 = 0.0f, acc1 = 0.0f;
  // loads of up to 8 pieces in flight, then their sum in piece order
  for (int q0 = 0; q0 < un.z; q0 += 8) {
    float a[8], b[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const bool in = q0 + q < un.z;
      a[q] = in ? pu[(q0 + q) * 512 + tid] : 0.0f;
      b[q] = in ? pu[(q0 + q) * 512 + 256 + tid] : 0.0f;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      acc0 += a[q];
      acc1 += b[q];
    }
  }
  const int gate = slot_gate(slots, gate0);
  float* o = out + blockIdx.z * out_stride;
  if (kk < ch.y)
    project_epilogue<float, MODE>(ang[ch.x + kk].ds * acc0, (long)(ch.x + kk) * g.nd + j, o, gate, gs, gp);
  if (kk + 8 < ch.y)
    project_epilogue<float, MODE>(ang[ch.x + kk + 8].ds * acc1, (long)(ch.x + kk + 8) * g.nd + j, o, gate, gs, gp);
}

// Byte offset 16 col + so of a staged entry, as one v_lshl_add_u32: written
// out because the compiler otherwise folds the high word of a 64-bit
// position and the shift into an align-bit and a mask (two instructions).
// so is a scalar operand: the same for the whole wave (the line's offset in
// the band, which depends on the band and the line counter only).
__device__ __forceinline__ unsigned lds_col_offset(unsigned col, int so) {
  unsigned r;
  asm("v_lshl_add_u32 %0, %1, 4, %2" : "=v"(r) : "v"(col), "s"(so));
  return r;
}

// 64-bit add as one v_lshl_add_u64: written out so that the compiler keeps
// one position per ray instead of splitting it into several induction
// variables of the unrolled line loop.
__device__ __forceinline__ void add_u64(unsigned long long& a, unsigned long long b) {
  asm("v_lshl_add_u64 %0, %0, 0, %1" : "+v"(a) : "v"(b));
}

// Quarter-turn forward. For a row-stepping (primary) angle k, with k2 = k +
// n_angles/2 (k < n_angles/2) or k - n_angles/2 (then reversed), the Joseph
// rays of angle k through the quarter turns of the image give the other
// rays: with the planes P_m[q] = x[R^m q], R (r, c) -> (c, n - 1 - r),
//   ray j of P_0 -> ray (k, j)          ray j of P_2 -> ray (k, n_det - 1 - j)
//   ray j of P_1 -> ray (k2, j)         ray j of P_3 -> ray (k2, n_det - 1 - j)
// (k2's bins reversed when k >= n_angles/2). So each staged entry holds the
// four planes' values at one pixel (a float4) and one crossing, one
// conversion and one pair of weights serve four rays; the bins run over
// [0, ceil(n_det/2)) only. The work split is the line-sheared one of
// k_joseph_fwd_shear (same schedule format, kQuCap entries per band, the
// piece list ordered so that block i, which runs on XCD i mod 8, gets pieces
// from the i mod 8-th eighth of the image rows; entries with unit -1 are
// padding); a tap
// reads the entries at the crossing's column and the next one and
// interpolates. Multi-piece units write 2 NP partial sums per thread (planes
// x two rays), added by k_joseph_fwd_quad_finish.
//
// NP = 8 (n_angles a multiple of 4) adds the transposed image's quarter
// turns, Q_m[q] = x[T R^m q] with T (r, c) -> (c, r): the ray (k, j) of the
// transposed image is the ray (n_angles/2 - k, j) of the image (the line
// x cos t + y sin t = u through transposed points is the line at pi/2 - t),
// for k <= n_angles/2, and (3 n_angles/2 - k, n_det - 1 - j) above. The
// primary angles are then k = 0 .. n_angles/4 (0 to 45 degrees) and one
// crossing serves eight rays; at k = 0 and k = n_angles/4 the transposes
// repeat planes 0-3 and are not written. A staged entry is two float4 (the
// second half of the LDS array holds planes 4-7).
// grid (pieces, 1, G), block 256; piece piece0 + blockIdx.x. wQ holds the
// planes P_1, P_2, P_3 (and for NP = 8 Q_0 .. Q_3) plane_stride apart for
// each slot, wP is P_0.
constexpr int kQuCap = 1024;       // staged entries per band
constexpr int kQuPieceLines = 48;  // target lines per block
constexpr int kOcPieceLines = 32;  // the same for NP = 8

// Sinogram index of the output of plane m for the ray (k, j), or -1 where
// it repeats another plane's (the centre bin of an odd detector is its own
// reversal, written once; the transposes at k = 0 and k = n_angles/4).
__device__ __forceinline__ long quad_index(int m, int k, int j, int na, int nd) {
  const int H = na >> 1;
  const int k2 = k < H ? k + H : k - H;
  const int jr = nd - 1 - j;
  const bool rev = k >= H;
  if (m == 0) return (long)k * nd + j;
  if (m == 1) return (long)k2 * nd + (rev ? jr : j);
  if (jr == j) return -1;
  return m == 2 ? (long)k * nd + jr : (long)k2 * nd + (rev ? j : jr);
}

__device__ __forceinline__ long oct_index(int m, int k, int j, int na, int nd) {
  if (m < 4) return quad_index(m, k, j, na, nd);
  if (k == 0 || 4 * k == na) return -1;
  const long t = quad_index(m - 4, k, j, na, nd);
  if (t < 0) return -1;
  const int kt = (int)(t / nd), jt = (int)(t - (long)kt * nd);
  const int H = na >> 1;
  return kt <= H ? (long)(H - kt) * nd + jt : (long)(na + H - kt) * nd + (nd - 1 - jt);
}

template <int MODE, int NP>
__device__ __forceinline__ void quad_epilogue(const float (&v)[NP], int k, int j, int na, int nd, float* o, int gate,
                                              const GateScalars<float>* gs, const GatePtrs<float>* gp) {
#pragma unroll
  for (int m = 0; m < NP; ++m) {
    const long idx = oct_index(m, k, j, na, nd);
    if (idx >= 0) project_epilogue<float, MODE>(v[m], idx, o, gate, gs, gp);
  }
}

// Thread -> (angle slot kk of 8, bin of 32) of k_joseph_fwd_quad: wave w
// holds bins 8w .. 8w + 7 of all 8 slots, one slot per octet of lanes. A
// 16-byte LDS read is served 16 lanes per cycle; with 8 neighbouring bins of
// close angles in every cycle, the entries read lie within a few consecutive
// ones, and the LDS conflict counters of gfx950 show no bank conflicts for
// this layout (layouts with 16 or 32 bins of one angle per wave have 2-3
// conflict cycles per read).
__device__ __forceinline__ int quad_bin(int tid) { return (tid & 7) | ((tid >> 6) << 3); }
__device__ __forceinline__ int quad_slot(int tid) { return (tid >> 3) & 7; }

template <int MODE, int NP>
__global__ __launch_bounds__(256) void k_joseph_fwd_quad(Geo<float> g, const AngleFx* __restrict__ ang,
                                                         const int4* __restrict__ chunks,
                                                         const int4* __restrict__ pieces,
                                                         const int4* __restrict__ units,
                                                         const int4* __restrict__ bands,
                                                         const float* __restrict__ wP,
                                                         const float* __restrict__ wQ, long w_stride,
                                                         long q_stride, long plane_stride,
                                                         float* __restrict__ out, long out_stride, int gate0,
                                                         const GateScalars<float>* __restrict__ gs,
                                                         const GatePtrs<float>* __restrict__ gp,
                                                         const SlotInfo* __restrict__ slots,
                                                         float* __restrict__ part, long part_stride, int piece0) {
  static_assert(NP == 4 || NP == 8, "four or eight planes");
  constexpr int kH = NP / 4;          // float4 halves per staged entry
  constexpr int kPer = kQuCap / 256;  // staged entries per thread
  constexpr int kUnroll = NP == 4 ? 2 : 1;
  __shared__ float4 st[kQuCap * kH];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int4 pc = pieces[piece0 + blockIdx.x];
  if (pc.z < 0) return;  // padding entry of the XCD-ordered piece list
  const int4 un = units[pc.z];
  const int4 ch = chunks[un.x];
  const long long Bm = (long long)(((unsigned long long)(unsigned)ch.w << 32) | (unsigned)ch.z);
  const int2 bb = make_int2(pc.x, pc.y);
  const int kk = quad_slot(tid);
  const int nb = (g.nd + 1) >> 1;
  const int j = un.y * kShJD + quad_bin(tid);
  const int jc = min(j, nb - 1);
  const AngleFx& A0 = ang[ch.x + min(kk, ch.y - 1)];
  const AngleFx& A1 = ang[ch.x + min(kk + 8, ch.y - 1)];
  const unsigned long long S0 = (unsigned long long)A0.B;
  const unsigned long long S1 = (unsigned long long)A1.B;
  const long long c0j = A0.C0 + (long long)jc * A0.A;
  const long long c1j = A1.C0 + (long long)jc * A1.A;
  const int n = g.n, pitch = g.pitch;
  // plane bases (uniform) and 32-bit byte offsets from them (the host keeps
  // a padded plane under 2^31 bytes)
  const char* pl[NP];
  pl[0] = (const char*)(wP + blockIdx.z * w_stride);
#pragma unroll
  for (int m = 1; m < NP; ++m) pl[m] = (const char*)(wQ + blockIdx.z * q_stride + (m - 1) * plane_stride);
  auto ld = [&](int m, unsigned off) { return *(const float*)(pl[m] + off); };
  // staged entries of lines beyond a band's last are never read: they keep
  // whatever an earlier band left (zero at first)
  float4 pre[kPer * kH];
#pragma unroll
  for (int e = 0; e < kPer * kH; ++e) pre[e] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  // entry i = l * pitch + q of a band; a wave's 64 entries share one line
  auto fetch = [&](const int4 bd) {
#pragma unroll
    for (int e = 0; e < kPer; ++e) {
      const int ib = 256 * e + 64 * wv;
      const int l = ib >> bd.w;
      if (l < bd.y) {
        const int o = (int)(((long long)l * Bm) >> 32);
        // column clamped into the padded row [-kPad, n + kPad - 1] (zero halo)
        const int c = min(max(bd.z + o + (ib & ((1 << bd.w) - 1)) + lane, -kPad), n + kPad - 1);
        const unsigned off = 4u * (unsigned)((bd.x + l + kPad) * pitch + c + kPad);
#pragma unroll
        for (int h = 0; h < kH; ++h)
          pre[e * kH + h] = make_float4(ld(4 * h, off), ld(4 * h + 1, off), ld(4 * h + 2, off), ld(4 * h + 3, off));
      }
    }
  };
  // the two rays' 32.32 crossings relative to the band's window start: one
  // 64-bit add per line (v_lshl_add_u64), the high word the window column,
  // the low word the fraction
  unsigned long long p0 = 0, p1 = 0;
  int s_prev = 0;
  if (bb.y > 0) {
    const int4 bd = bands[bb.x];
    fetch(bd);
    p0 = (unsigned long long)(c0j + (long long)bd.x * A0.B - ((long long)bd.z << 32));
    p1 = (unsigned long long)(c1j + (long long)bd.x * A1.B - ((long long)bd.z << 32));
    s_prev = bd.z;
  }
  float acc0[NP], acc1[NP];
#pragma unroll
  for (int m = 0; m < NP; ++m) acc0[m] = acc1[m] = 0.0f;
  for (int b = 0; b < bb.y; ++b) {
    const int4 bd = bands[bb.x + b];
#pragma unroll
    for (int e = 0; e < kPer; ++e)
#pragma unroll
      for (int h = 0; h < kH; ++h) st[h * kQuCap + 256 * e + tid] = pre[e * kH + h];
    __syncthreads();
    if (b + 1 < bb.y) fetch(bands[bb.x + b + 1]);
    p0 += (unsigned long long)(long long)(s_prev - bd.z) << 32;
    p1 += (unsigned long long)(long long)(s_prev - bd.z) << 32;
    s_prev = bd.z;
    long long om = 0;
    float b0[NP], b1[NP];
#pragma unroll
    for (int m = 0; m < NP; ++m) b0[m] = b1[m] = 0.0f;
    const char* base = (const char*)st;
    // the taps of both rays on line l: the entries at the crossing's column
    // and the next one (each half of the entry); so = 16 (l pitch - o_l) is
    // the byte offset of line l's window (uniform)
    auto tap = [&](int so, float4 (&x0)[kH], float4 (&y0)[kH], float& f0, float4 (&x1)[kH], float4 (&y1)[kH],
                   float& f1) {
      const char* q0 = base + lds_col_offset((unsigned)(p0 >> 32), so);
      const char* q1 = base + lds_col_offset((unsigned)(p1 >> 32), so);
#pragma unroll
      for (int h = 0; h < kH; ++h) {
        x0[h] = *(const float4*)(q0 + 16 * kQuCap * h);
        y0[h] = *(const float4*)(q0 + 16 * kQuCap * h + 16);
        x1[h] = *(const float4*)(q1 + 16 * kQuCap * h);
        y1[h] = *(const float4*)(q1 + 16 * kQuCap * h + 16);
      }
      f0 = float((unsigned)p0);
      f1 = float((unsigned)p1);
      add_u64(p0, S0);
      add_u64(p1, S1);
    };
    // tap weights times 2^32: w1 = f, w0 = 2^32 - f (one rounding, the
    // rounding of 1 - f 2^-32 scaled by 2^32), so that every sum is 2^32
    // times the sum of the unscaled weights, exactly; kFix undoes the scale
    auto mix = [&](const float4 (&x)[kH], const float4 (&y)[kH], float f, float (&a)[NP]) {
      const float w1 = f, w0 = fmaf(f, -1.0f, 4294967296.0f);
#pragma unroll
      for (int h = 0; h < kH; ++h) {
        a[4 * h + 0] = fmaf(w1, y[h].x, fmaf(w0, x[h].x, a[4 * h + 0]));
        a[4 * h + 1] = fmaf(w1, y[h].y, fmaf(w0, x[h].y, a[4 * h + 1]));
        a[4 * h + 2] = fmaf(w1, y[h].z, fmaf(w0, x[h].z, a[4 * h + 2]));
        a[4 * h + 3] = fmaf(w1, y[h].w, fmaf(w0, x[h].w, a[4 * h + 3]));
      }
    };
    int l = 0;
    for (; l + kUnroll <= bd.y; l += kUnroll) {
      float4 x0[kUnroll][kH], y0[kUnroll][kH], x1[kUnroll][kH], y1[kUnroll][kH];
      float f0[kUnroll], f1[kUnroll];
#pragma unroll
      for (int t = 0; t < kUnroll; ++t) {
        const int so = 16 * (((l + t) << bd.w) - (int)(om >> 32));
        om += Bm;
        tap(so, x0[t], y0[t], f0[t], x1[t], y1[t], f1[t]);
      }
#pragma unroll
      for (int t = 0; t < kUnroll; ++t) {
        mix(x0[t], y0[t], f0[t], b0);
        mix(x1[t], y1[t], f1[t], b1);
      }
    }
    if (kUnroll > 1 && l < bd.y) {
      float4 x0[kH], y0[kH], x1[kH], y1[kH];
      float f0, f1;
      const int so = 16 * ((l << bd.w) - (int)(om >> 32));
      om += Bm;
      tap(so, x0, y0, f0, x1, y1, f1);
      mix(x0, y0, f0, b0);
      mix(x1, y1, f1, b1);
    }
#pragma unroll
    for (int m = 0; m < NP; ++m) {
      acc0[m] += b0[m];
      acc1[m] += b1[m];
    }
    __syncthreads();
  }
#pragma unroll
  for (int m = 0; m < NP; ++m) {
    acc0[m] *= kFix;
    acc1[m] *= kFix;
  }
  if (un.z > 1) {  // partial sums; k_joseph_fwd_quad_finish adds them
    float* pu = part + blockIdx.z * part_stride + un.w + pc.w * (NP * 512);
#pragma unroll
    for (int m = 0; m < NP; ++m) {
      pu[m * 512 + tid] = acc0[m];
      pu[m * 512 + 256 + tid] = acc1[m];
    }
    return;
  }
  if (j >= nb) return;
  const int gate = slot_gate(slots, gate0);
  float* o = out + blockIdx.z * out_stride;
  if (kk < ch.y) {
    float v[NP];
#pragma unroll
    for (int m = 0; m < NP; ++m) v[m] = A0.ds * acc0[m];
    quad_epilogue<MODE, NP>(v, ch.x + kk, j, g.na, g.nd, o, gate, gs, gp);
  }
  if (kk + 8 < ch.y) {
    float v[NP];
#pragma unroll
    for (int m = 0; m < NP; ++m) v[m] = A1.ds * acc1[m];
    quad_epilogue<MODE, NP>(v, ch.x + kk + 8, j, g.na, g.nd, o, gate, gs, gp);
  }
}

// Sum of the partial sums of the multi-piece units of k_joseph_fwd_quad in
// piece order, then the outputs; block y handles plane y (NP times the
// blocks of one launch per unit, for latency). grid (count, NP, G), block 256.
template <int MODE, int NP>
__global__ __launch_bounds__(256) void k_joseph_fwd_quad_finish(Geo<float> g, const AngleFx* __restrict__ ang,
                                                                const int4* __restrict__ chunks,
                                                                const int4* __restrict__ units,
                                                                const int* __restrict__ multi,
                                                                const float* __restrict__ part, long part_stride,
                                                                float* __restrict__ out, long out_stride, int gate0,
                                                                const GateScalars<float>* __restrict__ gs,
                                                                const GatePtrs<float>* __restrict__ gp,
                                                                const SlotInfo* __restrict__ slots, int multi0) {
  const int tid = threadIdx.x;
  const int4 un = units[multi[multi0 + blockIdx.x]];
  const int4 ch = chunks[un.x];
  const int kk = quad_slot(tid);
  const int nb = (g.nd + 1) >> 1;
  const int j = un.y * kShJD + quad_bin(tid);
  if (j >= nb) return;
  const int m = blockIdx.y;
  const float* pu = part + blockIdx.z * part_stride + un.w + m * 512;
  float a0 = 0.0f, a1 = 0.0f;
  // loads of up to 8 pieces in flight, then their sum in piece order
  for (int q0 = 0; q0 < un.z; q0 += 8) {
    float va[8], vb[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const bool in = q0 + q < un.z;
      va[q] = in ? pu[(q0 + q) * (NP * 512) + tid] : 0.0f;
      vb[q] = in ? pu[(q0 + q) * (NP * 512) + 256 + tid] : 0.0f;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      a0 += va[q];
      a1 += vb[q];
    }
  }
  const int gate = slot_gate(slots, gate0);
  float* o = out + blockIdx.z * out_stride;
  if (kk < ch.y) {
    const long idx = oct_index(m, ch.x + kk, j, g.na, g.nd);
    if (idx >= 0) project_epilogue<float, MODE>(ang[ch.x + kk].ds * a0, idx, o, gate, gs, gp);
  }
  if (kk + 8 < ch.y) {
    const long idx = oct_index(m, ch.x + kk + 8, j, g.na, g.nd);
    if (idx >= 0) project_epilogue<float, MODE>(ang[ch.x + kk + 8].ds * a1, idx, o, gate, gs, gp);
  }
}

constexpr int kAdjKC = 32;  // angles per staged chunk

// Bins staged per angle: a 32 x 8PX pixel tile projects onto at most
// sqrt(32^2 + (8PX)^2) bins (< 46 for PX = 4, < 71 for PX = 8), plus the
// window margins.
template <int PX>
constexpr int adj_window() {
  return PX == 8 ? 80 : 64;
}

// grid (ceil(n/(8*PX)), ceil(n/32), G*S), block 256; the angles of `ar`. With S > 1 block z
// handles angle share z % S of gate slot z / S and writes an unpadded partial
// image to out + (z % S) * part_stride + (z / S) * out_stride (summed later).
template <int PX>
__global__ __launch_bounds__(256) void k_joseph_adj_lds(Geo<float> g, const AngleFx* __restrict__ ang,
                                                        const float* __restrict__ sino, long sino_stride,
                                                        float* __restrict__ out, long out_stride,
                                                        int padded, int S, long part_stride, AngleRanges ar) {
  constexpr int kAdjW = adj_window<PX>();
  constexpr int kAdjUnroll = PX >= 8 ? 1 : 2;  // angles per unrolled step (registers)
  __shared__ float sy[kAdjKC * kAdjW];
  __shared__ long long s_row[kAdjKC][32];  // detector coordinate of row offset ty (incl. window base)
  __shared__ long long s_col[kAdjKC][8];   // ... plus column offset tx*PX
  __shared__ long long s_step[kAdjKC];     // to the next pixel of the row
  __shared__ float4 s_w[kAdjKC];           // hat-weight constants (na32, pa32, oma)
  __shared__ int s_jb[2][kAdjKC];
  __shared__ float s_ds[2][kAdjKC];
  const int tid = threadIdx.x;
  const int tx = tid & 7, ty = tid >> 3;
  // consecutive workgroups go to the 8 XCDs in turn: making the share the
  // fastest-varying index keeps each share (angle range) on one XCD's L2
  // when S is 8 (or a divisor of it)
  const int L = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  const int share = L % S, rest = L / S;
  const int tiles = gridDim.x * gridDim.y, tile = rest % tiles, slot = rest / tiles;
  const int R0 = (tile / gridDim.x) * 32, C0 = (tile % gridDim.x) * (8 * PX);
  // the share's angles: launch angles [vbeg, vend) in the order of `ar`,
  // staged in chunks of consecutive angles that end where a range ends
  const int V = ar.count();
  const int vbeg = (int)((long)V * share / S), vend = (int)((long)V * (share + 1) / S);
  auto chunk = [&](int v, int& k0, int& kcn) {
    k0 = ar.at(v);
    kcn = min(min(kAdjKC, vend - v), ar.run(v));
  };
  const float* s = sino + slot * sino_stride;
  const int nd = g.nd;
  float acc[PX], blk[PX];
#pragma unroll
  for (int p = 0; p < PX; ++p) acc[p] = blk[p] = 0.0f;
  constexpr int kPer = kAdjKC * kAdjW / 256;  // staged values per thread
  // bin window of the chunk starting at angle k0, for angle k0 + tid
  auto window = [&](int k0, int kcn, int& jb, float& ds) {
    if (tid < kcn) {
      const AngleFx A = ang[k0 + tid];
      const int pmin = A.rows ? C0 : R0, lmin = A.rows ? R0 : C0;
      const int pext = A.rows ? 8 * PX - 1 : 31, lext = A.rows ? 31 : 8 * PX - 1;
      const long long u00 = A.U0 + (long long)pmin * A.P + (long long)lmin * A.Q;
      const long long up = (long long)pext * A.P, ul = (long long)lext * A.Q;
      const long long umin = min(min(u00, u00 + up), min(u00 + ul, u00 + up + ul));
      jb = (int)(umin >> 32) - 1;
      ds = A.ds;
    }
  };
  // loads of a chunk into registers (bins scaled later, zero off the detector)
  float pre[kPer];
  auto fetch = [&](int k0, int kcn, const int* jbs) {
#pragma unroll
    for (int e = 0; e < kPer; ++e) {
      const int i = tid + e * 256;
      const int kc = i / kAdjW, q = i % kAdjW;
      float v = 0.0f;
      if (kc < kcn) {
        const int jj = jbs[kc] + q;
        if ((unsigned)jj < (unsigned)nd) v = s[(long)(k0 + kc) * nd + jj];
      }
      pre[e] = v;
    }
  };
  // bin windows of two chunks (double buffered: the next chunk's loads are in
  // flight while the current chunk is computed)
  int jb = 0;
  float ds = 0.0f;
  int k0 = 0, kcn = 0;
  if (vbeg < vend) chunk(vbeg, k0, kcn);
  window(k0, kcn, jb, ds);
  if (tid < kAdjKC) {
    s_jb[0][tid] = jb;
    s_ds[0][tid] = ds;
  }
  __syncthreads();
  if (vbeg < vend) fetch(k0, kcn, s_jb[0]);
  int cur = 0;
  for (int v0 = vbeg; v0 < vend; v0 += kcn, cur ^= 1) {
    chunk(v0, k0, kcn);
    const int v1 = v0 + kcn;
    int k1 = 0, kcn1 = 0;
    if (v1 < vend) chunk(v1, k1, kcn1);
    // stage the fetched bins, pre-scaled by the ray length per line
#pragma unroll
    for (int e = 0; e < kPer; ++e) {
      const int i = tid + e * 256;
      const int kc = i / kAdjW;
      sy[i] = kc < kcn ? pre[e] * s_ds[cur][kc] : 0.0f;
    }
    // per-angle coordinate tables: rows (32) and column groups (8)
    for (int i = tid; i < kcn * 40; i += 256) {
      const int kc = i / 40, e = i % 40;
      const AngleFx A = ang[k0 + kc];
      const long long sc = A.rows ? A.P : A.Q;  // along a row (column step)
      const long long sr = A.rows ? A.Q : A.P;  // along a column (row step)
      if (e < 32) {
        const int pmin = A.rows ? C0 : R0, lmin = A.rows ? R0 : C0;
        const long long base = A.U0 + (long long)pmin * A.P + (long long)lmin * A.Q -
                               ((long long)s_jb[cur][kc] << 32) + ((long long)(kc * kAdjW) << 32);
        s_row[kc][e] = base + (long long)e * sr;
      } else {
        s_col[kc][e - 32] = (long long)((e - 32) * PX) * sc;
        if (e == 32) {
          s_step[kc] = sc;
          s_w[kc] = make_float4(A.na32, A.pa32, A.oma, 0.0f);
        }
      }
    }
    if (v1 < vend) {
      window(k1, kcn1, jb, ds);
      if (tid < kAdjKC) {
        s_jb[cur ^ 1][tid] = jb;
        s_ds[cur ^ 1][tid] = ds;
      }
    }
    __syncthreads();
    if (v1 < vend) fetch(k1, kcn1, s_jb[cur ^ 1]);
#pragma unroll kAdjUnroll
    for (int kc = 0; kc < kcn; ++kc) {
      const float4 wc = s_w[kc];
      const float na32 = wc.x, pa32 = wc.y, oma = wc.z;
      const long long st = s_step[kc];
      long long u = s_row[kc][ty] + s_col[kc][tx];
      // the bin pairs of all PX pixels are read before any is used
      float y0[PX], y1[PX], fl[PX];
#pragma unroll
      for (int p = 0; p < PX; ++p) {
        const float* q = sy + (int)(u >> 32);
        fl[p] = float((unsigned)u);
        y0[p] = q[0];
        y1[p] = q[1];
        u += st;
      }
#pragma unroll
      for (int p = 0; p < PX; ++p) {
        // hat weights 1 - |a| d and 1 - |a| (1 - d), clamped at 0 (neither
        // exceeds 1, so a clamp to [0, 1] is the same)
        const float w0 = __builtin_amdgcn_fmed3f(fmaf(na32, fl[p], 1.0f), 0.0f, 1.0f);
        const float w1 = __builtin_amdgcn_fmed3f(fmaf(pa32, fl[p], oma), 0.0f, 1.0f);
        blk[p] = fmaf(w1, y1[p], fmaf(w0, y0[p], blk[p]));
      }
    }
#pragma unroll
    for (int p = 0; p < PX; ++p) {
      acc[p] += blk[p];
      blk[p] = 0.0f;
    }
    __syncthreads();
  }
  const int r = R0 + ty;
  if (r >= g.n) return;
#pragma unroll
  for (int p = 0; p < PX; ++p) {
    const int c = C0 + tx * PX + p;
    if (c >= g.n) continue;
    if (S > 1)
      out[share * part_stride + slot * out_stride + (long)r * g.n + c] = acc[p];
    else if (padded)
      out[slot * out_stride + (long)(r + kPad) * g.pitch + (c + kPad)] = acc[p];
    else
      out[slot * out_stride + (long)r * g.n + c] = acc[p];
  }
}

// Quarter-turn backprojection. With x = c - hc, y = r - hc and an even number
// of angles spread over [0, pi), angle k + na/2 is angle k turned by pi/2, and
// the quarter turn of the image R: (r, c) -> (c, n - 1 - r) keeps the detector
// coordinate: U(R p, theta + pi/2) = U(p, theta). A half turn of the angle
// (theta + pi, outside [0, pi)) is angle theta with the detector reversed,
// U -> (n_det - 1) - U. The hat weights depend on |a| only, which is the same
// for angle k and angle k +- na/2. So for a pixel p of the top-left quadrant
// (n even) and any angle k, one detector coordinate and one pair of weights
// serve four (pixel, angle) pairs:
//   p      at k                                (bins as they are)
//   R p    at k + na/2, or k - na/2 reversed
//   R^2 p  at k, reversed
//   R^3 p  at k + na/2 reversed, or k - na/2
// and the four quadrants' pixels get every angle exactly once. The four rows
// of angle k's chunk entry are staged interleaved (one float4 per bin), the
// reversed ones read backwards from the mirrored window, so that the bin index
// and the weights are shared. Per four pairs: a 64-bit add, one conversion,
// two clamped FMAs for the weights, two 16-byte LDS reads and eight FMAs.
//
// A block owns a TY x TX*PX tile of the quadrant; a thread accumulates PX
// pixels of a row TX columns apart (columns C0 + tx + TX p), so that the TX
// lanes of a row read neighbouring 16-byte entries (distinct LDS banks)
// rather than entries PX bins apart.
// grid (ceil(n/2/(TX*PX)), ceil(n/2/TY), G*S), block TX*TY; all angles.
// S > 1: partial images as in k_joseph_adj_lds.
constexpr int kQuadKC = 16;  // angles per staged chunk

// Bins staged per angle for a TY x TX*PX tile: its pixels project onto at most
// sqrt((TY - 1)^2 + (TX PX - 1)^2) bins, and the window needs 3 more (the
// bin below the lowest, the second bin of the highest, rounding); rounded up
// to a multiple of 16.
template <int PX, int TX, int TY>
constexpr int quad_window() {
  int span = 0;
  while (span * span < (TY - 1) * (TY - 1) + (TX * PX - 1) * (TX * PX - 1)) ++span;
  return (span + 3 + 15) / 16 * 16;
}

template <int PX, int TX, int TY>
__global__ __launch_bounds__(TX * TY) __attribute__((amdgpu_waves_per_eu(PX <= 4 ? 4 : 1))) void k_joseph_adj_quad(Geo<float> g, const AngleFx* __restrict__ ang,
                                                             const float* __restrict__ sino, long sino_stride,
                                                             float* __restrict__ out, long out_stride, int padded,
                                                             int S, long part_stride, AngleRanges ar) {
  constexpr int NT = TX * TY;
  constexpr int kW = quad_window<PX, TX, TY>();
  constexpr int KC = kQuadKC;
  constexpr int kPer = (KC * kW + NT - 1) / NT;  // staged entries per thread
  __shared__ float4 sy[KC * kW];
  __shared__ long long s_row[KC][TY];
  __shared__ long long s_col[KC][TX];
  // per angle of a chunk (double-buffered: the next chunk's are written
  // while the current chunk is computed): bin window start, ray length per
  // line, the tile corner's window coordinate, its steps along a column and
  // a row
  __shared__ int s_jb[2][KC];
  __shared__ float s_ds[2][KC];
  __shared__ long long s_base[2][KC], s_sr[2][KC], s_sc[2][KC];
  // byte offsets in the slot's sinogram of the four staged rows at the
  // window's first bin (rows k and k' = k +- na/2, forwards and backwards;
  // entry q of the window is at offset + q times the row's step) and the
  // step of row k' (+4 forwards, -4 backwards)
  __shared__ int4 s_fo[2][KC];
  __shared__ int s_fs[2][KC];
  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = tid / TX;
  const int L = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  // workgroup-uniform (held in scalar registers)
  const int share = __builtin_amdgcn_readfirstlane(L % S), rest = __builtin_amdgcn_readfirstlane(L / S);
  const int tiles = gridDim.x * gridDim.y;
  const int tile = __builtin_amdgcn_readfirstlane(rest % tiles), slot = __builtin_amdgcn_readfirstlane(rest / tiles);
  const int R0 = (tile / gridDim.x) * TY, C0 = (tile % gridDim.x) * (TX * PX);
  const int na = g.na, H = na >> 1, nd = g.nd;
  // the share's angles: launch angles [vbeg, vend) in the order of `ar`
  // (all angles, or an angle subset closed under k <-> k +- n_angles/2),
  // staged in chunks of consecutive angles that end where a range ends
  const int V = ar.count();
  const int vbeg = (int)((long)V * share / S), vend = (int)((long)V * (share + 1) / S);
  auto chunk = [&](int v, int& k0, int& kcn) {
    k0 = ar.at(v);
    kcn = min(min(KC, vend - v), ar.run(v));
  };
  const float* s = sino + slot * sino_stride;
  float acc[4][PX], blk[4][PX];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int p = 0; p < PX; ++p) acc[m][p] = blk[m][p] = 0.0f;
  // one thread per angle of the chunk: the window and the table constants
  auto window = [&](int k0, int kcn, int buf) {
    if (tid < kcn) {
      const AngleFx A = ang[k0 + tid];
      const int pmin = A.rows ? C0 : R0, lmin = A.rows ? R0 : C0;
      const int pext = A.rows ? TX * PX - 1 : TY - 1, lext = A.rows ? TY - 1 : TX * PX - 1;
      const long long u00 = A.U0 + (long long)pmin * A.P + (long long)lmin * A.Q;
      const long long up = (long long)pext * A.P, ul = (long long)lext * A.Q;
      const long long umin = min(min(u00, u00 + up), min(u00 + ul, u00 + up + ul));
      const int jb = (int)(umin >> 32) - 1;
      const long long sc = A.rows ? A.P : A.Q;  // along a row (column step)
      const long long sr = A.rows ? A.Q : A.P;  // along a column (row step)
      s_jb[buf][tid] = jb;
      s_ds[buf][tid] = A.ds;
      // the tile corner's coordinate in the chunk's staged window (angle
      // tid's bins start at entry tid kW)
      s_base[buf][tid] = u00 - ((long long)jb << 32) + ((long long)(tid * kW) << 32);
      s_sr[buf][tid] = sr;
      s_sc[buf][tid] = sc;
      // x: k forwards, z: k backwards (bin nd - 1 - j), and for k < na/2
      // y: k' forwards, w: k' backwards, else the other way round
      const int k = k0 + tid, k2 = k < H ? k + H : k - H;
      const int fa = 4 * (k * nd + jb), ra = 4 * (k * nd + nd - 1 - jb);
      const int fb = 4 * (k2 * nd + jb), rb = 4 * (k2 * nd + nd - 1 - jb);
      s_fo[buf][tid] = k < H ? make_int4(fa, ra, fb, rb) : make_int4(fa, ra, rb, fb);
      s_fs[buf][tid] = k < H ? 4 : -4;
    }
  };
  // the four rows of a chunk's entries: angle k forwards and backwards, angle
  // k +- na/2 forwards and backwards (zero off the detector); the offsets
  // are 32-bit (the host keeps 4 n_angles n_det below 2^31) from the slot's
  // base, so each load takes one multiply-add
  float4 pre[kPer];
  const char* sb = (const char*)s;
  auto ld = [&](int off) { return *(const float*)(sb + (unsigned)off); };
  auto fetch = [&](int kcn, int buf) {
#pragma unroll
    for (int e = 0; e < kPer; ++e) {
      const int i = tid + e * NT;
      const int kc = i / kW, q = i % kW;
      float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      // the window start is read for every entry (kc < KC unless KC kW is
      // not a multiple of NT: then clamped into the array)
      const int kcr = KC * kW % NT == 0 ? kc : min(kc, KC - 1);
      const bool in = (kc < kcn) & ((unsigned)(s_jb[buf][kcr] + q) < (unsigned)nd);
      if (in) {
        const int4 o = s_fo[buf][kc];
        const int sq = __mul24(s_fs[buf][kc], q);
        v.x = ld(o.x + 4 * q);
        v.z = ld(o.y - 4 * q);
        v.y = ld(o.z + sq);
        v.w = ld(o.w - sq);
      }
      pre[e] = v;
    }
  };
  int k0 = 0, kcn = 0;
  if (vbeg < vend) chunk(vbeg, k0, kcn);
  window(k0, kcn, 0);
  __syncthreads();
  if (vbeg < vend) fetch(kcn, 0);
  int cur = 0;
  for (int v0 = vbeg; v0 < vend; v0 += kcn, cur ^= 1) {
    chunk(v0, k0, kcn);
    const int v1 = v0 + kcn;
    int k1 = 0, kcn1 = 0;
    if (v1 < vend) chunk(v1, k1, kcn1);
#pragma unroll
    for (int e = 0; e < kPer; ++e) {
      const int i = tid + e * NT;
      if (KC * kW % NT == 0 || i < KC * kW) {
        const int kc = i / kW;
        const float sc = kc < kcn ? s_ds[cur][kc] : 0.0f;
        sy[i] = make_float4(pre[e].x * sc, pre[e].y * sc, pre[e].z * sc, pre[e].w * sc);
      }
    }
    // the row table (entry i = kc TY + e) and the column table (i = kc TX
    // + e), each a fixed set of entries per thread; the thread index is made
    // opaque so that the entries' (kc, e) are recomputed per chunk rather
    // than held in registers across the loop
    int tq = tid;
    asm volatile("" : "+v"(tq));
#pragma unroll
    for (int it = 0; it < (KC * TY + NT - 1) / NT; ++it) {
      const int i = tq + it * NT;
      const int kc = i / TY, e = i % TY;
      if (kc < kcn) s_row[kc][e] = s_base[cur][kc] + s_sr[cur][kc] * e;
    }
#pragma unroll
    for (int it = 0; it < (KC * TX + NT - 1) / NT; ++it) {
      const int i = tq + it * NT;
      const int kc = i / TX, e = i % TX;
      if (kc < kcn) s_col[kc][e] = s_sc[cur][kc] * e;
    }
    if (v1 < vend) window(k1, kcn1, cur ^ 1);
    __syncthreads();
    if (v1 < vend) fetch(kcn1, cur ^ 1);
#pragma unroll 2
    for (int kc = 0; kc < kcn; ++kc) {
      // the angle's constants through scalar loads (uniform address)
      const AngleFx& A = ang[k0 + kc];
      const float na32 = A.na32, pa32 = A.pa32, oma = A.oma;
      const long long st = TX * A.RS;
      long long u = s_row[kc][ty] + s_col[kc][tx];
      float4 y0[PX], y1[PX];
      float fl[PX];
#pragma unroll
      for (int p = 0; p < PX; ++p) {
        const float4* q = sy + (int)(u >> 32);
        fl[p] = float((unsigned)u);
        y0[p] = q[0];
        y1[p] = q[1];
        u += st;
      }
#pragma unroll
      for (int p = 0; p < PX; ++p) {
        const float w0 = __builtin_amdgcn_fmed3f(fmaf(na32, fl[p], 1.0f), 0.0f, 1.0f);
        const float w1 = __builtin_amdgcn_fmed3f(fmaf(pa32, fl[p], oma), 0.0f, 1.0f);
        blk[0][p] = fmaf(w1, y1[p].x, fmaf(w0, y0[p].x, blk[0][p]));
        blk[1][p] = fmaf(w1, y1[p].y, fmaf(w0, y0[p].y, blk[1][p]));
        blk[2][p] = fmaf(w1, y1[p].z, fmaf(w0, y0[p].z, blk[2][p]));
        blk[3][p] = fmaf(w1, y1[p].w, fmaf(w0, y0[p].w, blk[3][p]));
      }
    }
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int p = 0; p < PX; ++p) {
        acc[m][p] += blk[m][p];
        blk[m][p] = 0.0f;
      }
    __syncthreads();
  }
  const int n = g.n, h = n >> 1;
  const int r = R0 + ty;
  if (r >= h) return;
#pragma unroll
  for (int p = 0; p < PX; ++p) {
    const int c = C0 + tx + TX * p;
    if (c >= h) continue;
    // p, R p, R^2 p, R^3 p
    const int rr[4] = {r, c, n - 1 - r, n - 1 - c};
    const int cc[4] = {c, n - 1 - r, n - 1 - c, r};
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      if (S > 1)
        out[share * part_stride + slot * out_stride + (long)rr[m] * n + cc[m]] = acc[m][p];
      else if (padded)
        out[slot * out_stride + (long)(rr[m] + kPad) * g.pitch + (cc[m] + kPad)] = acc[m][p];
      else
        out[slot * out_stride + (long)rr[m] * n + cc[m]] = acc[m][p];
    }
  }
}

// Sum of S partial images (fixed order) into the padded or unpadded output,
// four pixels of a row per thread (n a multiple of 4: every row and the
// padded rows start 16-byte aligned). grid (ceil(n/64), ceil(n/16), G),
// block (16, 16).
__global__ __launch_bounds__(256) void k_sum_parts4(int n, int pitch, int S, const float* __restrict__ parts,
                                                    long part_stride, long slot_stride, float* __restrict__ out,
                                                    long out_stride, int padded) {
  const int c = (blockIdx.x * 16 + threadIdx.x) * 4;
  const int r = blockIdx.y * 16 + threadIdx.y;
  if (c >= n || r >= n) return;
  const long q = (long)r * n + c;
  const float* src = parts + blockIdx.z * slot_stride;
  float4 a[16];
#pragma unroll
  for (int s = 0; s < 16; ++s)
    a[s] = s < S ? *(const float4*)(src + s * part_stride + q) : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    v.x += a[s].x;
    v.y += a[s].y;
    v.z += a[s].z;
    v.w += a[s].w;
  }
  float* o = padded ? out + blockIdx.z * out_stride + (long)(r + kPad) * pitch + c + kPad
                    : out + blockIdx.z * out_stride + q;
  *(float4*)o = v;
}

// Sum of S partial images (fixed order) into the padded or unpadded output.
// grid (ceil(n/16), ceil(n/16), G), block (16, 16)
__global__ __launch_bounds__(256) void k_sum_parts(int n, int pitch, int S, const float* __restrict__ parts,
                                                   long part_stride, long slot_stride, float* __restrict__ out,
                                                   long out_stride, int padded) {
  const int c = blockIdx.x * 16 + threadIdx.x;
  const int r = blockIdx.y * 16 + threadIdx.y;
  if (c >= n || r >= n) return;
  const long q = (long)r * n + c;
  const float* src = parts + blockIdx.z * slot_stride;
  // all S loads in flight together (S <= 16), then the sum in share order
  float a[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) a[s] = s < S ? src[s * part_stride + q] : 0.0f;
  float v = 0.0f;
#pragma unroll
  for (int s = 0; s < 16; ++s) v += a[s];
  if (padded)
    out[blockIdx.z * out_stride + (long)(r + kPad) * pitch + c + kPad] = v;
  else
    out[blockIdx.z * out_stride + q] = v;
}

}  // namespace mcr
