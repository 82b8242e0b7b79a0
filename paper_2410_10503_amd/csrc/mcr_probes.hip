// Roofline probes of the GPU (libmcr_probes.so, include/mcr_probes.h): the
// on-chip read rates that bound the gather kernels of libmcr (LDS reads of
// 16-byte entries, L2-resident 16-byte global reads) and the streaming copy
// rate that bounds its elementwise kernels. Measurement only; the
// reconstruction never calls these.
#include "mcr_probes.h"

#include <hip/hip_runtime.h>

namespace {

// Every lane reads 16-byte entries of a 16 KB LDS array at conflict-free
// addresses (consecutive lanes, consecutive entries), four reads per step.
// The array does not change, so an empty asm statement with a memory clobber
// ends every step: it keeps the compiler from reusing loaded values across
// steps (each step's reads are issued again). The values are folded with
// three-input XORs (two VALU instructions per read), well under the LDS
// rate, so the LDS bounds the kernel.
__global__ __launch_bounds__(256) void k_probe_lds(int iters, unsigned* __restrict__ out) {
  __shared__ uint4 buf[1024];
  const int tid = threadIdx.x;
#pragma unroll
  for (int e = 0; e < 4; ++e) buf[tid + 256 * e] = make_uint4(tid, e, tid ^ e, blockIdx.x);
  __syncthreads();
  unsigned a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  for (int i = 0; i < iters; ++i) {
    const int base = (tid + (i & 3) * 64) & 255;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const uint4 v = buf[base + 256 * e];
      if (e & 1) {
        a0 = a0 ^ v.x ^ v.y;
        a1 = a1 ^ v.z ^ v.w;
      } else {
        a2 = a2 ^ v.x ^ v.y;
        a3 = a3 ^ v.z ^ v.w;
      }
    }
    __asm__ volatile("" ::: "memory");
  }
  out[blockIdx.x * 256 + tid] = a0 ^ a1 ^ a2 ^ a3;
}

// Every block walks the whole buffer (a few MiB, resident in the L2 of each
// XCD after the first pass) with 16-byte loads, starting at a block-dependent
// offset; the per-CU working set far exceeds the L1, so the reads are served
// by the L2.
__global__ __launch_bounds__(256) void k_probe_l2(const uint4* __restrict__ buf, long count, int passes,
                                                  unsigned* __restrict__ out) {
  const int tid = threadIdx.x;
  long i = ((long)blockIdx.x * 4096 + tid) % count;
  unsigned a0 = 0, a1 = 0;
  const long steps = passes * (count / 256);
  for (long s = 0; s < steps; s += 4) {
    uint4 v[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      long j = i + 256L * e;
      if (j >= count) j -= count;
      v[e] = buf[j];
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      a0 = a0 ^ v[e].x ^ v[e].y;
      a1 = a1 ^ v[e].z ^ v[e].w;
    }
    i += 1024;
    if (i >= count) i -= count;
  }
  out[blockIdx.x * 256 + tid] = a0 ^ a1;
}

// Every lane of every wave reads the 16-byte entry pattern[lane] (< 64) of a
// 512-entry LDS array, shifted each step by a multiple of 64 entries (which
// keeps each entry's banks). With a pattern that puts two lanes on different
// entries of the same banks, the read takes longer exactly when the LDS
// serves those two lanes in the same cycle: the pattern's read rate against
// a conflict-free one tells which lanes share a cycle.
__global__ __launch_bounds__(256) void k_probe_lds_pattern(const int* __restrict__ pattern, int iters,
                                                           unsigned* __restrict__ out) {
  __shared__ uint4 buf[512];
  const int tid = threadIdx.x;
  buf[tid] = make_uint4(tid, blockIdx.x, 1u, 2u);
  buf[tid + 256] = make_uint4(tid, blockIdx.x, 3u, 4u);
  __syncthreads();
  const int e = pattern[tid & 63];
  unsigned a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  for (int i = 0; i < iters; ++i) {
    // four independent reads per step, so that the LDS bounds the loop
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint4 v = buf[e + 64 * ((4 * i + k) & 7)];
      if (k & 1) {
        a0 = a0 ^ v.x ^ v.y;
        a1 = a1 ^ v.z ^ v.w;
      } else {
        a2 = a2 ^ v.x ^ v.y;
        a3 = a3 ^ v.z ^ v.w;
      }
    }
    __asm__ volatile("" ::: "memory");
  }
  out[blockIdx.x * 256 + tid] = a0 ^ a1 ^ a2 ^ a3;
}

// Four 16-byte loads in flight per thread, then the four stores.
__global__ __launch_bounds__(256) void k_probe_copy(const float4* __restrict__ a, float4* __restrict__ b, long n4) {
  const long i0 = (long)blockIdx.x * 1024 + threadIdx.x;
  float4 v[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const long i = i0 + 256L * e;
    v[e] = i < n4 ? a[i] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const long i = i0 + 256L * e;
    if (i < n4) b[i] = v[e];
  }
}

int timed(hipEvent_t e0, hipEvent_t e1, float* ms) {
  if (hipEventSynchronize(e1) != hipSuccess) return 1;
  return hipEventElapsedTime(ms, e0, e1) != hipSuccess;
}

}  // namespace

extern "C" {

int mcr_probe_lds_read(int blocks, int iters, double* bytes_per_s) {
  if (blocks < 1 || iters < 1 || !bytes_per_s) return 1;
  unsigned* out = nullptr;
  if (hipMalloc(&out, sizeof(unsigned) * 256 * (size_t)blocks) != hipSuccess) return 2;
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  hipLaunchKernelGGL(k_probe_lds, dim3(blocks), dim3(256), 0, nullptr, iters, out);  // warm-up
  (void)hipEventRecord(e0, nullptr);
  hipLaunchKernelGGL(k_probe_lds, dim3(blocks), dim3(256), 0, nullptr, iters, out);
  (void)hipEventRecord(e1, nullptr);
  float ms = 0.0f;
  const int err = timed(e0, e1, &ms) || hipGetLastError() != hipSuccess;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(out);
  if (err || ms <= 0.0f) return 3;
  *bytes_per_s = 16.0 * 4.0 * 256.0 * (double)blocks * (double)iters / (ms * 1e-3);
  return 0;
}

int mcr_probe_lds_pattern(const int* pattern, int blocks, int iters, double* bytes_per_s) {
  if (!pattern || blocks < 1 || iters < 1 || !bytes_per_s) return 1;
  for (int t = 0; t < 64; ++t)
    if (pattern[t] < 0 || pattern[t] >= 64) return 1;
  int* pat = nullptr;
  unsigned* out = nullptr;
  if (hipMalloc(&pat, sizeof(int) * 64) != hipSuccess) return 2;
  if (hipMalloc(&out, sizeof(unsigned) * 256 * (size_t)blocks) != hipSuccess) {
    (void)hipFree(pat);
    return 2;
  }
  int err = hipMemcpy(pat, pattern, sizeof(int) * 64, hipMemcpyHostToDevice) != hipSuccess;
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  float ms = 0.0f;
  if (!err) {
    hipLaunchKernelGGL(k_probe_lds_pattern, dim3(blocks), dim3(256), 0, nullptr, pat, iters, out);  // warm-up
    (void)hipEventRecord(e0, nullptr);
    hipLaunchKernelGGL(k_probe_lds_pattern, dim3(blocks), dim3(256), 0, nullptr, pat, iters, out);
    (void)hipEventRecord(e1, nullptr);
    err = timed(e0, e1, &ms) || hipGetLastError() != hipSuccess;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(pat);
  (void)hipFree(out);
  if (err || ms <= 0.0f) return 3;
  *bytes_per_s = 16.0 * 4.0 * 256.0 * (double)blocks * (double)iters / (ms * 1e-3);
  return 0;
}

int mcr_probe_l2_read(long long buffer_bytes, int blocks, int passes, double* bytes_per_s) {
  if (buffer_bytes < 16 * 1024 || blocks < 1 || passes < 1 || !bytes_per_s) return 1;
  const long count = (long)(buffer_bytes / 16) / 1024 * 1024;
  uint4* buf = nullptr;
  unsigned* out = nullptr;
  if (hipMalloc(&buf, 16 * (size_t)count) != hipSuccess) return 2;
  if (hipMalloc(&out, sizeof(unsigned) * 256 * (size_t)blocks) != hipSuccess) {
    (void)hipFree(buf);
    return 2;
  }
  (void)hipMemset(buf, 1, 16 * (size_t)count);
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  hipLaunchKernelGGL(k_probe_l2, dim3(blocks), dim3(256), 0, nullptr, (const uint4*)buf, count, 1, out);
  (void)hipEventRecord(e0, nullptr);
  hipLaunchKernelGGL(k_probe_l2, dim3(blocks), dim3(256), 0, nullptr, (const uint4*)buf, count, passes, out);
  (void)hipEventRecord(e1, nullptr);
  float ms = 0.0f;
  const int err = timed(e0, e1, &ms) || hipGetLastError() != hipSuccess;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(buf);
  (void)hipFree(out);
  if (err || ms <= 0.0f) return 3;
  const double steps = (double)passes * (double)(count / 256);
  const double per_block = 16.0 * 256.0 * 4.0 * (double)((long)(steps + 3) / 4);
  *bytes_per_s = per_block * (double)blocks / (ms * 1e-3);
  return 0;
}

int mcr_probe_copy(long long bytes, int reps, double* bytes_per_s) {
  if (bytes < 1024 * 1024 || reps < 1 || !bytes_per_s) return 1;
  const long n4 = (long)(bytes / 16);
  float4 *a = nullptr, *b = nullptr;
  if (hipMalloc(&a, 16 * (size_t)n4) != hipSuccess) return 2;
  if (hipMalloc(&b, 16 * (size_t)n4) != hipSuccess) {
    (void)hipFree(a);
    return 2;
  }
  (void)hipMemset(a, 0, 16 * (size_t)n4);
  const dim3 grid((unsigned)((n4 + 1023) / 1024));
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  hipLaunchKernelGGL(k_probe_copy, grid, dim3(256), 0, nullptr, (const float4*)a, b, n4);
  (void)hipEventRecord(e0, nullptr);
  for (int r = 0; r < reps; ++r) hipLaunchKernelGGL(k_probe_copy, grid, dim3(256), 0, nullptr, (const float4*)a, b, n4);
  (void)hipEventRecord(e1, nullptr);
  float ms = 0.0f;
  const int err = timed(e0, e1, &ms) || hipGetLastError() != hipSuccess;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(a);
  (void)hipFree(b);
  if (err || ms <= 0.0f) return 3;
  *bytes_per_s = 2.0 * 16.0 * (double)n4 * reps / (ms * 1e-3);
  return 0;
}

}  // extern "C"
