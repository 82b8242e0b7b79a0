/*
 * mcr.h - motion-compensated SPDHG / PDHG reconstruction on AMD Instinct
 * MI355X (gfx950). C ABI of libmcr.so.
 *
 * Problem (Section II-A of Delplancke, Thielemans, Ehrhardt, "Accelerated
 * Convergent Motion Compensated Image Reconstruction"): gated data
 * d_i = A_i x + noise with A_i = A D_i, where D_i: X -> X is the displacement
 * operator of gate i and A: X -> Y the ray transform; the reconstruction
 * minimises alpha |x|^2 + sum_i |A_i x - d_i|^2 / N with Algorithm 1 (SPDHG,
 * and PDHG as its special case p_i = 1, every gate every iteration).
 *
 * Discretisation used by every entry point (the paper names the operators,
 * not their discretisation):
 *   image   x: [n][n] row-major, pixel (r, c) centred at
 *              (c - (n-1)/2, r - (n-1)/2) in unit pixels;
 *   sinogram : [n_angles][n_det] row-major (angle-major, detector fastest),
 *              angle k at k*pi/n_angles, bin j centred at j - (n_det-1)/2;
 *   A        : Joseph ray transform - each ray steps along image rows when
 *              4k <= n_angles or 4k >= 3*n_angles, along columns otherwise,
 *              interpolating linearly between the two nearest pixels of each
 *              line (zero outside the image) and weighting the line sum by
 *              1/|cos| (rows) or 1/|sin| (columns);
 *   D_i      : bilinear pull-back (D x)(p) = x~(phi_i(p)), zero outside the
 *              image; rigid phi(p) = R(phi)(p - c) + c + t about the image
 *              centre c, or phi(p) = p + u(p) for a displacement field u;
 *   A^T, D^T : the exact transposes of the same weights (gather kernels, no
 *              atomics, deterministic).
 *
 * Conventions common to every call:
 *   - Array arguments typed void* / const void* are DEVICE pointers to
 *     contiguous arrays of the handle's dtype (float for MCR_F32, double for
 *     MCR_F64) unless stated otherwise. They stay owned by the caller; the
 *     library never frees them and never keeps them after the call returns.
 *   - Arrays of pointers (mcr_state.y, d) and arrays of per-gate scalars
 *     (sigma, p, gate_seq) are HOST arrays.
 *   - All work is queued on the handle's HIP stream and is asynchronous,
 *     except the calls that return a host scalar (norms, objective, gap),
 *     which synchronise the stream before returning.
 *   - Every argument is validated before any device work is queued; a call
 *     that returns a status other than MCR_OK has queued nothing (except
 *     MCR_ERR_HIP, which reports a failure of the HIP runtime itself).
 *     mcr_last_error() then returns a message for the calling thread.
 *   - A handle must not be used from two host threads at once.
 */
#ifndef MCR_H
#define MCR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MCR_OK = 0,
  MCR_ERR_ARG = 1,        /* invalid argument (size, index, null pointer, step size, ...) */
  MCR_ERR_HIP = 2,        /* the HIP runtime reported an error                            */
  MCR_ERR_NOMEM = 3,      /* a device or pinned host allocation failed                    */
  MCR_ERR_NONFINITE = 4,  /* a scalar result is NaN or infinite                           */
  MCR_ERR_STATE = 5       /* the handle cannot do this (e.g. motion too irregular)        */
} mcr_status;

typedef enum { MCR_F32 = 0, MCR_F64 = 1 } mcr_dtype;

typedef enum {
  MCR_MOTION_IDENTITY = 0,  /* D_i = I                                                     */
  MCR_MOTION_RIGID = 1,     /* rigid[0] = rotation phi [rad], rigid[1..2] = (t_x, t_y) [px] */
  MCR_MOTION_FIELD = 2      /* field: device float [2][n][n], plane 0 = u_x (along columns),
                               plane 1 = u_y (along rows), in pixels                         */
} mcr_motion_kind;

typedef struct {
  int32_t n;         /* image is n x n, 1 <= n <= 4096                         */
  int32_t n_angles;  /* angles k*pi/n_angles, k = 0..n_angles-1, 1..16384     */
  int32_t n_det;     /* unit-spaced centred detector bins, 1..16384           */
} mcr_geometry;

typedef struct {
  int32_t kind;        /* mcr_motion_kind                                        */
  double rigid[3];     /* MCR_MOTION_RIGID: (phi, t_x, t_y); ignored otherwise    */
  const float* field;  /* MCR_MOTION_FIELD: device [2][n][n] float32; the handle
                          copies it, so it may be freed after the call            */
} mcr_motion;

typedef struct mcr_handle mcr_handle;

/* State of Algorithm 1 (its initialisation is x = z = z-bar = 0, y = 0). All
 * device arrays of the handle's dtype: x, z, zbar [n][n]; y is a HOST array
 * of N device pointers, y[i] of shape [n_angles][n_det]. Updated in place.   */
typedef struct {
  void* x;
  void* z;
  void* zbar;
  void* const* y;
} mcr_state;

/* ---------------------------------------------------------------------------
 * Handle: geometry, the N gates' motion, device workspaces, a HIP stream.
 * `stream` is a hipStream_t (NULL = the null stream). The handle copies the
 * motion (fields included). dtype selects the precision of the operators and
 * of the state; the scalar diagnostics (norms, objective, gap) are always
 * computed in FP64 on the device. Fails with MCR_ERR_STATE if a displacement
 * field folds so strongly that the transposed warp's gather window (at most
 * 7 x 7 pixels around the inverse image of each pixel) cannot cover it.
 * ------------------------------------------------------------------------- */
mcr_status mcr_create(const mcr_geometry* geom, int32_t n_gates, const mcr_motion* motion,
                      mcr_dtype dtype, void* stream, mcr_handle** out);
mcr_status mcr_destroy(mcr_handle* h);
mcr_status mcr_set_stream(mcr_handle* h, void* stream);
/* Replace the motion of one gate (synchronises the handle's stream first).
 * MCR_ERR_STATE if a field folds too strongly for the transposed warp's
 * gather window; the gate is then reset to the identity.                      */
mcr_status mcr_set_motion(mcr_handle* h, int32_t gate, const mcr_motion* motion);
/* Replace the rigid parameters of every gate at once (host [N][3] doubles:
 * phi, t_x, t_y); all gates must be rigid. Asynchronous: the update is queued
 * on the handle's stream (no synchronisation, no window check: a 3 x 3 gather
 * window covers any rotation).                                                */
mcr_status mcr_set_rigid_params(mcr_handle* h, const double* params);
/* Sizes and settings of a handle (any pointer may be NULL). */
mcr_status mcr_get_info(const mcr_handle* h, mcr_geometry* geom, int32_t* n_gates,
                        mcr_dtype* dtype, int32_t* window_radius);

/* ---------------------------------------------------------------------------
 * Operators (Section II-A; A_i^* as used in Algorithm 1 step (iii)).
 * x, img: [n][n]; sino: [n_angles][n_det]; gate in [0, N).
 * ------------------------------------------------------------------------- */
mcr_status mcr_warp(mcr_handle* h, int32_t gate, const void* x, void* img);              /* D_i x     */
mcr_status mcr_warp_adjoint(mcr_handle* h, int32_t gate, const void* b, void* img);      /* D_i^T b   */
mcr_status mcr_project(mcr_handle* h, const void* x, void* sino);                        /* A x       */
mcr_status mcr_backproject(mcr_handle* h, const void* sino, void* img);                  /* A^T y     */
mcr_status mcr_apply_Ai(mcr_handle* h, int32_t gate, const void* x, void* sino);         /* A D_i x   */
mcr_status mcr_apply_Ai_adjoint(mcr_handle* h, int32_t gate, const void* sino, void* img); /* D_i^T A^T y */

/* ---------------------------------------------------------------------------
 * Algorithm 1. Each iteration with drawn gate set S:
 *   (i)   x <- (x - tau z-bar) / (1 + 2 tau alpha)                 (prox of tau g)
 *   (ii)  y_i <- (y_i + sigma_i (A_i x - d_i)) / (1 + sigma_i N/2), i in S (prox of sigma_i f_i^*)
 *   (iii) z <- z + sum_{i in S} A_i^*(y_i' - y_i);
 *         z-bar <- z + sum_{i in S} (theta / p_i) A_i^*(y_i' - y_i)   (z after the update)
 * with g(x) = alpha |x|^2 and f_i(u) = |u - d_i|^2 / N.
 * d: host array of N device pointers to the gated data d_i [n_angles][n_det].
 * sigma, p: host arrays of N doubles, sigma_i > 0, p_i in (0, 1]; tau > 0;
 * alpha > 0; theta >= 0; all finite.
 * ------------------------------------------------------------------------- */
/* SPDHG with serial sampling: n_iter iterations, iteration k updating the one
 * gate gate_seq[k] (host int32 array, entries in [0, N)).                    */
mcr_status mcr_spdhg_iterate(mcr_handle* h, const mcr_state* st, const void* const* d,
                             double alpha, const double* sigma, double tau, double theta,
                             const double* p, const int32_t* gate_seq, int32_t n_iter);
/* One SPDHG epoch: N iterations (the paper's epoch, Section II-A).            */
mcr_status mcr_spdhg_epoch(mcr_handle* h, const mcr_state* st, const void* const* d,
                           double alpha, const double* sigma, double tau, double theta,
                           const double* p, const int32_t* gate_seq);
/* One PDHG epoch = one iteration with S = all gates and p_i = 1. It runs the
 * same kernels as SPDHG, so PDHG with N = 1 equals SPDHG with N = 1 bit for bit. */
mcr_status mcr_pdhg_epoch(mcr_handle* h, const mcr_state* st, const void* const* d,
                          double alpha, const double* sigma, double tau, double theta);

/* ---------------------------------------------------------------------------
 * Batches of independent slices (one geometry): slice s has gates_per_slice[s]
 * gates; `motion` lists all gates slice after slice (global gate index =
 * first gate of the slice + local gate). The operator entry points accept the
 * global gate index. Workspaces hold one slot per slice; PDHG over all gates
 * and the stacked norm are not available on a batch handle (MCR_ERR_STATE).
 * ------------------------------------------------------------------------- */
mcr_status mcr_batch_create(const mcr_geometry* geom, int32_t n_slices, const int32_t* gates_per_slice,
                            const mcr_motion* motion, mcr_dtype dtype, void* stream, mcr_handle** out);
/* One SPDHG epoch of every slice (Algorithm 1 with serial sampling; slice s
 * runs N_s iterations): all slices take step (i), then max_s N_s rounds run
 * one launch per phase each over the round's slots; slice s takes its
 * iteration j in round floor(j max N / N_s), so every round holds about
 * sum N_s / max N slots and each slice's iterations keep their order (the
 * slices are independent problems, so the rounds only decide which slots
 * share a launch; the results are those of per-slice epochs). Device arrays
 * (handle dtype): x, z, zbar [S][n][n]; y, d [sum N_s][n_angles][n_det] in
 * global gate order. Host arrays: alpha, tau, theta [S]; sigma, p [sum N_s];
 * gate_seq [sum N_s], slice s's draws (local gate indices) at its first global
 * gate. use_graph != 0 replays the epoch as a HIP graph (captured on first use
 * and again whenever x, z or zbar move, or after mcr_set_variant,
 * mcr_autotune, mcr_set_motion or mcr_set_rigid_params; captured on a stream
 * of the handle) and launched on the handle's stream.                         */
mcr_status mcr_batch_spdhg_epoch(mcr_handle* h, void* x, void* z, void* zbar, void* y, const void* d,
                                 const double* alpha, const double* sigma, const double* tau,
                                 const double* theta, const double* p, const int32_t* gate_seq,
                                 int32_t use_graph);

/* ---------------------------------------------------------------------------
 * Differentiation through unrolled SPDHG iterations (reverse mode; not in the
 * paper, built on its Algorithm 1). Gradients and checkpoints have the
 * handle's dtype; rigid motion gradients are FP64.
 * ------------------------------------------------------------------------- */
/* As mcr_spdhg_iterate, and before iteration k (gate g = gate_seq[k]) has
 * touched the duals it stores x after step (i) into x1_ckpt[k] ([n][n]) and
 * y_g into y_ckpt[k] ([n_angles][n_det]): host arrays of n_iter device
 * pointers. b_ckpt (may be NULL; else n_iter device pointers of [n][n])
 * receives the iteration's backprojection A^T (y_g' - y_g), which spares
 * mcr_spdhg_step_backward its recomputation (one warp, projection and
 * backprojection per step). Same results as mcr_spdhg_iterate, bit for bit. */
mcr_status mcr_spdhg_iterate_ckpt(mcr_handle* h, const mcr_state* st, const void* const* d,
                                  double alpha, const double* sigma, double tau, double theta,
                                  const double* p, const int32_t* gate_seq, int32_t n_iter,
                                  void* const* x1_ckpt, void* const* y_ckpt, void* const* b_ckpt);
/* Reverse of one SPDHG iteration on `gate` from its checkpoint (x1, y_before)
 * and the gate's data d_gate, with that iteration's sigma (of the gate), tau,
 * theta, p (of the gate). On entry gx, gy_gate, gz, gzbar ([n][n] except
 * gy_gate [n_angles][n_det]) hold the adjoints of the iteration's outputs
 * x, y_gate, z, z-bar; on return those of its inputs. grad_motion (may be
 * NULL) accumulates d/d(motion of gate): device double[3] (phi, t_x, t_y) for
 * rigid gates, device [2][n][n] (u_x, u_y planes) for fields, unused for the
 * identity. b_ckpt (may be NULL): the iteration's backprojection stored by
 * mcr_spdhg_iterate_ckpt; given, the step costs one projection and one
 * backprojection, else it recomputes it (two of each; the same results bit
 * for bit). The reverse map is the transpose of the iteration (see
 * mcr_grad.h).                                                                */
mcr_status mcr_spdhg_step_backward(mcr_handle* h, int32_t gate, const void* x1,
                                   const void* y_before, const void* d_gate, double alpha,
                                   double sigma, double tau, double theta, double p, void* gx,
                                   void* gy_gate, void* gz, void* gzbar, void* grad_motion,
                                   const void* b_ckpt);
/* grad_motion += d/d(motion of gate) <img, D_gate v> (img, v: [n][n]); layout
 * of grad_motion as above.                                                     */
mcr_status mcr_warp_motion_grad(mcr_handle* h, int32_t gate, const void* img, const void* v,
                                void* grad_motion);

/* ---------------------------------------------------------------------------
 * Rigid registration: the preliminary step of Section I, which estimates the
 * displacement map from the reference motion state to each gate (the paper
 * does not say how). Reading: the rigid parameters (phi, t_x, t_y) of gate
 * `gate` minimise E = |D(theta) ref - target|^2 / 2 (D the library's warp),
 * by gradient descent in the scaled coordinates (phi (n - 1) / 2, t_x, t_y)
 * (pixels at the image's edge) with Barzilai-Borwein step lengths (the first
 * trial moves 1 px) and Armijo backtracking (sufficient decrease 1e-4, at most
 * 40 halvings); it stops after the first accepted step shorter than tol
 * pixels, at a zero gradient, or after max_iter steps. ref, target: device
 * [n][n] in the handle's dtype. params: host double[3], the start on entry and
 * the result on return; the gate's motion is set to the result. loss (may be
 * NULL): E at the result; steps (may be NULL): steps taken. The gate must be
 * rigid. Synchronises the stream at every evaluation (warp, residual, FP64
 * squared norm, motion gradient).
 * ------------------------------------------------------------------------- */
mcr_status mcr_register_rigid(mcr_handle* h, int32_t gate, const void* ref, const void* target,
                              double* params, int32_t max_iter, double tol, double* loss,
                              int32_t* steps);
/* The same for the chest experiment's non-rigid motion, a linear dilatation
 * (Section III), taken as the affine displacement field
 *   u(p) = A (p - c) + t,   x = column - c, y = row - c, c = (n - 1) / 2,
 * params = host double[6] (A00, A01, A10, A11, t_x, t_y), each component
 * evaluated as (A_r0 x + A_r1 y) + t_r and rounded to float32 (the field
 * precision); minimised over the scaled coordinates (A (n - 1) / 2, t). The
 * gate must be a field gate; its field is set to the result through
 * mcr_set_motion (which can fail if the map needs a wider gather window than
 * the transposed warp has). On any error after the start (a non-finite
 * energy, MCR_ERR_NONFINITE, included) the gate is reset to the identity, as
 * its field planes then hold a map whose gather windows were not set up.     */
mcr_status mcr_register_affine(mcr_handle* h, int32_t gate, const void* ref, const void* target,
                               double* params, int32_t max_iter, double tol, double* loss,
                               int32_t* steps);
/* Dense registration: the displacement field itself (the maps u_i of Section
 * II-A, estimated in Section I's preliminary step). Reading: u [2][n][n]
 * minimises
 *   E(u) = |D_u ref - target|^2 / 2 + lambda / 2 R(u),
 * R(u) the sum, over both components, of the squared differences between
 * horizontally and vertically adjacent pixels of the image (a discrete
 * Dirichlet energy), by the same descent directly on the field in pixels:
 * u is kept in FP64 and evaluated on its float32 rounding (the field
 * precision); tol bounds the Euclidean norm of the whole accepted step.
 * Scale-space schedule: for each width sigmas[l] (pixels; a host array of
 * n_levels in [0, 16], each in [0, 32]; 0 = no smoothing) both images are
 * smoothed with the separable Gaussian exp(-k^2 / (2 sigma^2)),
 * |k| <= int(3 sigma + 0.5), normalised, zero outside the image, and the
 * descent (max_iter, tol per level) runs on them from the previous level's
 * field; n_levels = 0: one level on the images themselves. loss: E of the
 * last level; steps: summed over the levels.
 * field: device float32 [2][n][n] (u_x plane, u_y plane), the start on
 * entry and the result on return; the gate's motion is then set to it
 * through mcr_set_motion (MCR_ERR_STATE, gate reset to the identity, if it
 * folds too strongly for the transposed warp's window). lambda >= 0. The
 * gate must be a field gate. Workspace: 8 n^2 doubles (3 n^2 more with
 * levels), allocated on the first call. Synchronises the stream at every
 * evaluation. On any error after the start the gate is reset to the
 * identity, as for mcr_register_affine.                                       */
mcr_status mcr_register_field(mcr_handle* h, int32_t gate, const void* ref, const void* target, void* field,
                              double lambda, const double* sigmas, int32_t n_levels, int32_t max_iter,
                              double tol, double* loss, int32_t* steps);

/* ---------------------------------------------------------------------------
 * FP64 diagnostics (Theorem 1 and the model of Section II-A), computed on the
 * device in double precision whatever the handle's dtype; they synchronise.
 * ------------------------------------------------------------------------- */
/* |A_i|^2 (gate >= 0) or |(A_1; ...; A_N)|^2 = lambda_max(sum_i A_i^* A_i)
 * (gate = -1) by power iteration from the device FP64 image v0 [n][n] (not
 * modified), stopping when the Rayleigh quotient changes by at most rtol
 * relative, or after max_iter iterations. *iters (may be NULL) receives the
 * iteration count.                                                            */
mcr_status mcr_power_norm_sq(mcr_handle* h, int32_t gate, const double* v0, int32_t max_iter,
                             double rtol, double* out, int32_t* iters);
/* O(x) = alpha |x|^2 + sum_i |A_i x - d_i|^2 / N.                              */
mcr_status mcr_objective(mcr_handle* h, const void* x, const void* const* d, double alpha,
                         double* out);
/* O(x) + |z|^2 / (4 alpha) + sum_i (<y_i, d_i> + (N/4) |y_i|^2) with
 * z = sum_i A_i^* y_i recomputed from y (>= 0; zero exactly at the saddle point). */
mcr_status mcr_duality_gap(mcr_handle* h, const mcr_state* st, const void* const* d,
                           double alpha, double* out);

/* ---------------------------------------------------------------------------
 * Step sizes (host only, no device work). Theorem 1 quotes the rates of
 * "well-chosen" step sizes; these attain them:
 *   algo 0 (SPDHG, p_i = 1/N): norms_sq = |A_i|^2 for i = 0..N-1;
 *     s_i = sqrt(1 + |A_i|^2 / (alpha N)), s = max s_i, rho = 1 - 2/(N (1 + s)),
 *     sigma_i = 2 / (N (s_i - 1)), tau = 1 / (2 N alpha rho (1 + s)), theta = rho,
 *     per-epoch rate rho^N = l(kappa^SPDHG, N).
 *   algo 1 (PDHG): norms_sq[0] = |(A_1; ...; A_N)|^2; s = sqrt(1 + norms_sq[0] / (alpha N)),
 *     sigma_i = 2 / (N (s - 1)), tau = 1 / (2 alpha (s - 1)), theta = (s - 1)/(s + 1),
 *     per-epoch rate theta = l(kappa^PDHG, 1).
 * sigma: host array of N doubles (out). Any of tau, theta, rate may be NULL.  */
mcr_status mcr_step_sizes(int32_t algo, int32_t n_gates, const double* norms_sq, double alpha,
                          double* sigma, double* tau, double* theta, double* rate_per_epoch);

/* ---------------------------------------------------------------------------
 * Sampling over gates x angle subsets (the next step named in the
 * Conclusions: sampling over both the gates and subsets of the data).
 * The angles are cut into M subsets: contiguous ones [k_s, k_{s+1}),
 * k_s = floor(s n_angles / M), or paired ones (mcr_set_subset_partition). Block b = i M + s (gate i, subset s) has the
 * operator A_b = R_s A D_i (R_s keeps the rows of subset s) and the data term
 * f_b(u) = |u - d_{i,s}|^2 / N, so the objective, its minimiser and the dual
 * solution are those of the gate problem; f_b^* keeps the modulus N/2, so the
 * dual step of a block is the gate formula (with N, the gate count) on the
 * block's rows. An epoch is N M block iterations (the operator work of one
 * PDHG iteration).
 * ------------------------------------------------------------------------- */
/* Sets the number of angle subsets (1 <= M <= n_angles; 1 at creation).
 * Rebuilds the float32 forward projector's work tables so that no work unit
 * crosses a subset boundary; the full-range operators are unchanged.
 * Synchronises the stream. Not available on batch handles (MCR_ERR_STATE).  */
mcr_status mcr_set_subsets(mcr_handle* h, int32_t n_subsets);
/* The same with a choice of partition: paired = 0 gives the contiguous
 * subsets above; paired != 0 (n_angles even, 1 <= M <= n_angles/2) gives
 * subset s = [h_s, h_{s+1}) and [h_s + n_angles/2, h_{s+1} + n_angles/2),
 * h_s = floor(s (n_angles/2) / M): every angle with its partner a quarter
 * turn away (the Conclusions leave the choice of subsets open; every
 * partition gives the same objective and minimiser). With paired subsets
 * the quarter-turn projector pair (forward 4, adjoint codes < 0) also runs
 * the block launches. Synchronises the stream.                               */
mcr_status mcr_set_subset_partition(mcr_handle* h, int32_t n_subsets, int32_t paired);
/* |A_b|^2 for block (gate, subset) by FP64 power iteration on A_b^* A_b, as
 * mcr_power_norm_sq.                                                          */
mcr_status mcr_block_norm_sq(mcr_handle* h, int32_t gate, int32_t subset, const double* v0,
                             int32_t max_iter, double rtol, double* out, int32_t* iters);
/* n_iter iterations of Algorithm 1 over blocks with serial sampling: iteration
 * k updates block block_seq[k] (host int32, entries in [0, N M)): step (i);
 * the rows of subset s of y_i become (y + sigma_b (A_b x - d)) / (1 + sigma_b N/2);
 * z += A_b^*(dy); z-bar = z + (theta / p_b) A_b^*(dy). sigma and p are host
 * arrays of N M doubles indexed by block; y and d stay per gate (full
 * [n_angles][n_det] arrays, only the block's rows are read or written).      */
mcr_status mcr_spdhg_blocks_iterate(mcr_handle* h, const mcr_state* st, const void* const* d,
                                    double alpha, const double* sigma, double tau, double theta,
                                    const double* p, const int32_t* block_seq, int32_t n_iter);
/* Host step sizes for serial uniform sampling over the N M blocks
 * (p = 1/(N M)): s_b = sqrt(1 + norms_sq[b] / (alpha N)), s = max_b s_b,
 * rho = 1 - 2p / (1 + s), sigma_b = 2 / (N (s_b - 1)),
 * tau = p / (2 alpha rho (1 + s)), theta = rho; per-epoch rate rho^(N M) =
 * l(max_b |A_b|^2 / (alpha N), N M). sigma: host array of N M doubles (out);
 * tau, theta, rate may be NULL.                                               */
mcr_status mcr_step_sizes_blocks(int32_t n_gates, int32_t n_subsets, const double* norms_sq,
                                 double alpha, double* sigma, double* tau, double* theta,
                                 double* rate_per_epoch);

/* ---------------------------------------------------------------------------
 * Kernel variants of the float32 projector pair (no effect on FP64 handles).
 * forward:  0 = one thread per ray, 1 = LDS-tiled (8 angles x 32 bins share a
 *           staged image band; only where every band window fits in LDS),
 *           2 = the same with the bands scheduled on the host and the next
 *           band prefetched while the current one is computed,
 *           3 = host-scheduled bands whose window shifts line by line with
 *           the chunk's mean ray slope (up to 16 angles x 32 bins, two rays
 *           per thread; the default where it applies),
 *           4 = the same over the row-stepping angles and half the bins, the
 *           warp also writing the image's three quarter turns: one crossing
 *           serves rays of angle k and k +- n_angles/2, bins j and
 *           n_det - 1 - j (even n and n_angles, and a padded image of under
 *           2^29 pixels, only; launches over a paired angle subset run it
 *           per subset, over a contiguous one variant 3),
 *           5 = variant 4 over the angles of 0 to 45 degrees, the warp also
 *           writing the transposed image's four quarter turns: one crossing
 *           serves eight rays, the transpose's ray (k, j) being the image's
 *           ray (n_angles/2 - k, j) (even n, n_angles a multiple of 4;
 *           angle-subset launches run variant 4 or 3);
 * adjoint:  adj_px = 0 one thread per pixel, or 1, 2, 4, 8 pixels per thread with
 *           LDS-staged sinogram chunks, the angles split into adj_s (1..16)
 *           shares whose partial images are summed in a fixed order;
 *           adj_px = -2, -4, -8: the quarter-turn kernel with 2, 4, 8 pixels
 *           per thread on 32 x 16, 32 x 32, 32 x 64 pixel tiles, -16: 4 pixels
 *           per thread on 32 x 64 tiles, -32: 4 pixels per thread on 64 x 64
 *           tiles (one detector coordinate serves a pixel of the top-left
 *           quadrant at angle k and its three quarter turns at angles k and
 *           k +- n_angles/2; needs an even n and n_angles,
 *           4 n_angles n_det < 2^31 and a launch over all angles or a paired
 *           angle subset, else the tiled kernel runs with 2, 4, 8, 8, 8
 *           pixels per thread).
 * A new handle starts with forward 4 where available (else 3, 2, 0) and the
 * adjoint -4 with 16 shares on even n and n_angles (else 8 pixels, 6 shares).
 * All variants compute the same weights; results differ only by summation
 * order. mcr_autotune times the variants on this geometry with
 * gates_per_launch gates per launch (1 for SPDHG, N for PDHG; at most the
 * gates one launch of the handle covers, N or the batch's slots, else
 * MCR_ERR_ARG), each forward with the warp that writes its planes, keeps the
 * first variant, in a fixed order of preference (forward 4, 3, 2, 1, 0;
 * variant 5 only through mcr_set_variant), that is within 3% of the fastest (remembered per geometry and
 * gates_per_launch for the life of the process) and returns the choice
 * (output pointers may be NULL). Synchronises the stream.
 * ------------------------------------------------------------------------- */
mcr_status mcr_autotune(mcr_handle* h, int32_t gates_per_launch, int32_t* fwd, int32_t* adj_px,
                        int32_t* adj_s);
mcr_status mcr_set_variant(mcr_handle* h, int32_t fwd, int32_t adj_px, int32_t adj_s);

/* ---------------------------------------------------------------------------
 * Kernel timing (diagnostic). While enabled, every kernel launch of the handle
 * is bracketed by HIP events on the handle's stream. mcr_profile_read waits
 * for the stream, then returns per kernel class the summed duration [ms] and
 * the launch count, and clears the records. total_ms and launches are host
 * arrays of MCR_KERNEL_CLASSES entries (either may be NULL).
 * ------------------------------------------------------------------------- */
typedef enum {
  MCR_KERNEL_WARP = 0,         /* D_i (a1)                                   */
  MCR_KERNEL_PROJECT = 1,      /* A, fused with the dual step (a2, a3)       */
  MCR_KERNEL_BACKPROJECT = 2,  /* A^T (a4)                                   */
  MCR_KERNEL_TWARP = 3,        /* D_i^T, fused with the z / z-bar / x update (a5, a6) */
  MCR_KERNEL_XSTEP = 4,        /* step (i) alone                             */
  MCR_KERNEL_OTHER = 5,        /* reductions, copies                         */
  MCR_KERNEL_CLASSES = 6
} mcr_kernel_class;
mcr_status mcr_profile_enable(mcr_handle* h, int32_t enable);
mcr_status mcr_profile_read(mcr_handle* h, double* total_ms, int64_t* launches);

/* ---------------------------------------------------------------------------
 * For callers that cannot allocate device memory at the time of the call
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): A x, the Joseph projection of mcr_project, in float32, with no
 * handle. geom: host struct, 1 <= n <= 1024, 1 <= n_angles <= 4096,
 * 1 <= n_det <= 16384 (larger sizes: MCR_ERR_ARG, nothing queued). x: device
 * float [n][n]; sino: device float [n_angles][n_det] (out); both caller-owned
 * and on the current device. stream: hipStream_t (NULL = the null stream);
 * the call is asynchronous on it. The work runs in a fixed scratch array of
 * the library (8.5 MiB of device memory per GPU, held from the first call
 * on that GPU until the process ends): no hipMalloc, hipFree or other
 * allocation happens in the call. Every call on one GPU shares that array, so
 * calls that overlap on one GPU (different streams or host threads without
 * ordering between them) race and must not be issued. The result equals
 * mcr_project of a float32 handle of the same geometry up to summation order
 * (it runs the one-thread-per-ray kernel, forward variant 0).                 */
mcr_status mcr_project_noalloc(const mcr_geometry* geom, const float* x, float* sino, void* stream);

/* Message describing the last non-OK status returned on the calling thread. */
const char* mcr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MCR_H */
