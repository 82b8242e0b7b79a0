/*
 * mcr_probes.h - roofline probes of libmcr_probes.so (measurement only).
 *
 * The gather kernels of libmcr (the Joseph projection and backprojection,
 * Section II-A's ray transform and its transpose) are bound by on-chip read
 * rates rather than by HBM; these probes measure the rates their roofline
 * figures are quoted against, on the GPU they run on. Each call allocates
 * its own device buffers (freed before it returns), runs one warm-up launch
 * and one timed launch (or reps launches) on the null stream of the current
 * device, timed with HIP events, and synchronises. Return value: 0 on
 * success, 1 for an invalid argument, 2 when a device allocation fails, 3
 * when the HIP runtime reports an error. Results are bytes per second.
 */
#ifndef MCR_PROBES_H
#define MCR_PROBES_H

#ifdef __cplusplus
extern "C" {
#endif

/* LDS reads: `blocks` workgroups of 256 threads, each thread reading
 * 4 * iters 16-byte entries of a 16 KB LDS array at conflict-free addresses
 * (the access the quarter-turn kernels make). bytes_per_s: bytes read from
 * LDS per second over the whole GPU.                                          */
int mcr_probe_lds_read(int blocks, int iters, double* bytes_per_s);

/* LDS lane grouping: `blocks` workgroups of 256 threads; lane t of every
 * wave reads the 16-byte entry pattern[t] (64 host ints, each in [0, 64);
 * the call copies them) of an LDS array, 4 * iters times, each time shifted
 * by a multiple of 64 entries. bytes_per_s: bytes read from LDS per second over
 * the whole GPU; a pattern whose lanes on the same banks at different
 * entries are served in one cycle reads slower than a conflict-free one.    */
int mcr_probe_lds_pattern(const int* pattern, int blocks, int iters, double* bytes_per_s);

/* L2-resident global reads: `blocks` workgroups of 256 threads each walk a
 * buffer of buffer_bytes (rounded down to 16 KB; a few MiB fits every XCD's
 * L2) `passes` times with 16-byte loads. bytes_per_s: bytes loaded per
 * second over the whole GPU.                                                  */
int mcr_probe_l2_read(long long buffer_bytes, int blocks, int passes, double* bytes_per_s);

/* Device copy of `bytes` (at least 1 MiB) with 16-byte loads and stores,
 * reps times. bytes_per_s: bytes read plus bytes written per second.         */
int mcr_probe_copy(long long bytes, int reps, double* bytes_per_s);

#ifdef __cplusplus
}
#endif

#endif /* MCR_PROBES_H */
