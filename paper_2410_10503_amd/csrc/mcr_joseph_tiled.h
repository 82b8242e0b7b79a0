// LDS-tiled float32 Joseph projector pair (gfx950). Same fixed-point geometry
// as k_joseph_fwd_fx / k_joseph_adj_fx (AngleFx), different work split:
//
//  forward  - a block owns KA consecutive angles of one stepping type times JD
//             detector bins and walks the lines in bands. Each band of the
//             padded image is staged once in LDS as a sheared window (window
//             start moves by an integer slope m per line) and read by all
//             KA x JD rays; the LDS index of a tap is the integer part of the
//             ray's fixed-point crossing, so a sample costs one 64-bit add, one
//             conversion, one paired LDS read and two FMAs.
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

constexpr int kAdjKC = 32;  // angles per staged chunk
constexpr int kAdjW = 64;   // bins staged per angle

// grid (ceil(n/(8*PX)), ceil(n/32), G*S), block 256. With S > 1 block z
// handles angle share z % S of gate slot z / S and writes an unpadded partial
// image to out + (z % S) * part_stride + (z / S) * out_stride (summed later).
template <int PX>
__global__ __launch_bounds__(256) void k_joseph_adj_lds(Geo<float> g, const AngleFx* __restrict__ ang,
                                                        const float* __restrict__ sino, long sino_stride,
                                                        float* __restrict__ out, long out_stride,
                                                        int padded, int S, long part_stride) {
  __shared__ float sy[kAdjKC * kAdjW];
  __shared__ long long s_row[kAdjKC][32];  // detector coordinate of row offset ty (incl. window base)
  __shared__ long long s_col[kAdjKC][8];   // ... plus column offset tx*PX
  __shared__ long long s_step[kAdjKC];     // to the next pixel of the row
  __shared__ float4 s_w[kAdjKC];           // hat-weight constants (na32, pa32, oma)
  __shared__ int s_jb[2][kAdjKC];
  __shared__ float s_ds[2][kAdjKC];
  const int tid = threadIdx.x;
  const int tx = tid & 7, ty = tid >> 3;
  const int R0 = blockIdx.y * 32, C0 = blockIdx.x * (8 * PX);
  const int share = blockIdx.z % S, slot = blockIdx.z / S;
  const int kbeg = (int)((long)g.na * share / S), kend = (int)((long)g.na * (share + 1) / S);
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
  window(kbeg, min(kAdjKC, kend - kbeg), jb, ds);
  if (tid < kAdjKC) {
    s_jb[0][tid] = jb;
    s_ds[0][tid] = ds;
  }
  __syncthreads();
  if (kbeg < kend) fetch(kbeg, min(kAdjKC, kend - kbeg), s_jb[0]);
  int cur = 0;
  for (int k0 = kbeg; k0 < kend; k0 += kAdjKC, cur ^= 1) {
    const int kcn = min(kAdjKC, kend - k0);
    const int k1 = k0 + kAdjKC;
    const int kcn1 = min(kAdjKC, kend - k1);
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
    if (k1 < kend) {
      window(k1, kcn1, jb, ds);
      if (tid < kAdjKC) {
        s_jb[cur ^ 1][tid] = jb;
        s_ds[cur ^ 1][tid] = ds;
      }
    }
    __syncthreads();
    if (k1 < kend) fetch(k1, kcn1, s_jb[cur ^ 1]);
#pragma unroll 2
    for (int kc = 0; kc < kcn; ++kc) {
      const float4 wc = s_w[kc];
      const float na32 = wc.x, pa32 = wc.y, oma = wc.z;
      const long long st = s_step[kc];
      long long u = s_row[kc][ty] + s_col[kc][tx];
#pragma unroll
      for (int p = 0; p < PX; ++p) {
        const float* q = sy + (int)(u >> 32);
        const float fl = float((unsigned)u);
        // hat weights 1 - |a| d and 1 - |a| (1 - d), clamped at 0
        const float w0 = fmaxf(0.0f, fmaf(na32, fl, 1.0f));
        const float w1 = fmaxf(0.0f, fmaf(pa32, fl, oma));
        blk[p] = fmaf(w1, q[1], fmaf(w0, q[0], blk[p]));
        u += st;
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
  float v = 0.0f;
  for (int s = 0; s < S; ++s) v += src[s * part_stride + q];
  if (padded)
    out[blockIdx.z * out_stride + (long)(r + kPad) * pitch + c + kPad] = v;
  else
    out[blockIdx.z * out_stride + q] = v;
}

}  // namespace mcr
