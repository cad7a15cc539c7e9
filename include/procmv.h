/*
 * procmv: block-procedural matrix-free Hamiltonian product on MI355X (gfx950).
 *
 * C ABI of libprocmv.so.  The library applies a dense Hermitian operator H of
 * dimension D to one or more vectors without ever holding the D x D matrix:
 * blocks H^[n,m] are generated on the fly from a seed or a closed form, or
 * read from a partial or full cache of canonical block pairs in device memory,
 * and applied inside the same kernel (paper: Sec. II, Eqs. blockham,
 * blockmatvec, blockmatvecindex; Sec. III, Eqs. single_block_apply,
 * output_block_apply, and the block sources "seeded generation", "analytic
 * generation", "fused action", "full caching", "partial caching").
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Vectors are complex64 (interleaved float re, im), vector-contiguous:
 *    vector v of a block of nvec vectors starts at base + v * ld complex
 *    elements, ld >= D.  In PyTorch terms: a (nvec, D) complex64 tensor.
 *  - Pointers named X, Y, psi, out_dev are DEVICE pointers owned by the caller
 *    (allocate them with PyTorch or hipMalloc).  The library never frees them.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Device work is enqueued on it and calls return without synchronising,
 *    except where a call says it synchronises.
 *  - Every call returns a procmv_status.  Argument errors are detected on the
 *    host before anything is enqueued; launch errors are reported by the call
 *    that launched; faults inside kernels surface at the next synchronisation.
 *    procmv_last_error() gives a message for the calling thread.
 *  - Results are deterministic: the same inputs give bit-identical outputs on
 *    every run (fixed-order reductions, no floating-point atomics).
 *  - An operator handle is not thread-safe: serialise calls on one handle.
 */
#ifndef PROCMV_H
#define PROCMV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct procmv_op* procmv_op_t;

typedef enum {
    PROCMV_OK = 0,
    PROCMV_ERR_INVALID_ARG = 1,
    PROCMV_ERR_OOM = 2,
    PROCMV_ERR_INFEASIBLE_PLAN = 3,
    PROCMV_ERR_NOT_PLANNED = 4,
    PROCMV_ERR_HIP = 5,
    PROCMV_ERR_INTERNAL = 6
} procmv_status;

/* Block sources (paper Sec. III): seeded Philox-GUE and analytic sinc-DVR. */
typedef enum {
    PROCMV_GEN_PHILOX_GUE = 0,
    PROCMV_GEN_SINC_DVR = 1
} procmv_generator;

/* Storage modes (paper Sec. III, "full caching", "partial caching"). */
typedef enum {
    PROCMV_PROCEDURAL = 0,
    PROCMV_PARTIAL = 1,
    PROCMV_FULL = 2
} procmv_strategy;

/* Arithmetic of the block products.
 * PROCMV_FP32_COMPENSATED (sinc-DVR operators only; paper Sec. VII centered
 * Chebyshev propagation with the analytic blocks of Sec. III): the same
 * binary32 entries and binary32 operations, arranged against the
 * cancellation of the kinetic stencil (entries ~1/dx^2 with vanishing row
 * sums acting on smooth states).  The tile kernels apply the operator
 * without the band 0 < |i - j| < W (W = min(32, D)); the reduction adds the
 * band in difference form, sum_band t(i-j) (x_j - x_i), and the rest of the
 * row as the per-row constant C_i = d + sum_band t(i-j) + V_i (binary64 sum
 * of the binary32 entries, applied as a hi + lo binary32 pair), which is the
 * same operator.  Chebyshev recurrence vectors are carried as hi + lo
 * binary32 pairs updated with exact products and two-sums; the coefficient
 * sum and the norms stay binary64.  Products, propagation, the imaginary-
 * time filter and the Lanczos bounds all use it; batches do not. */
typedef enum {
    PROCMV_FP32 = 0,             /* binary32 entries, binary32 accumulation        */
    PROCMV_SPLIT_BF16 = 1,       /* hi/lo bfloat16 split on MFMA, fp32 accumulation */
    PROCMV_FP32_COMPENSATED = 2  /* binary32, difference-form band, hi + lo vectors */
} procmv_precision;

/* Sinc-DVR parameters (analytic generation, paper Sec. III).  Grid
 * x_i = x_min + i dx, dx = (x_max - x_min)/(D - 1); entries
 * T_ij = (-1)^(i-j) / (mass dx^2 (i-j)^2) for i != j and
 * H_ii = pi^2/(6 mass dx^2) + mass omega^2 x_i^2 / 2.  With compensate != 0
 * the constant diagonal also absorbs the binary32 rounding error of the
 * off-diagonal kinetic entries (keeps the exact zero row sum of the kinetic
 * stencil).  Pass NULL for the defaults x in [-20, 20], mass = omega = 1,
 * compensate = 1. */
typedef struct {
    double x_min, x_max, mass, omega;
    int32_t compensate;
} procmv_dvr_params;

/* Create an operator.  Philox-GUE (paper Sec. III, seeded generation; keyed
 * on global (i, j) so the matrix does not depend on the partition, Sec. II):
 * H_ij for i < j has re, im ~ N(0, 1/(2D)), H_ji = conj(H_ij), H_ii ~
 * N(0, 1/D) real, drawn from Philox4x32-10 with key (seed & 0xffffffff,
 * seed >> 32) and counter (i, j, 0, 0).  gen_params: NULL for GUE,
 * procmv_dvr_params* (or NULL) for DVR.  D in [1, 2^31).  No device memory is
 * touched until procmv_plan.  *out receives the handle. */
procmv_status procmv_create_operator(procmv_generator gen, uint64_t seed,
                                     int64_t D, const void* gen_params,
                                     procmv_op_t* out);

/* Choose the execution plan (paper Sec. IV: block size, storage mode, cache
 * budget / number of cached canonical pairs, Eq. partial_cache_pairs).
 * block_size b: multiple of 64, 64 <= b; the last block is ragged when
 * D % b != 0.  strategy PROCMV_PARTIAL caches P = floor(cache_fraction *
 * N_pair) canonical pairs (n <= m) of the N_pair = N_blk (N_blk + 1) / 2,
 * spread over block rows; PROCMV_FULL caches all; PROCMV_PROCEDURAL none.
 * Allocates the cache and fills it on `stream`, then SYNCHRONISES the stream.
 * Returns PROCMV_ERR_OOM if the cache cannot be allocated.  Re-planning
 * releases the previous plan's memory. */
procmv_status procmv_plan(procmv_op_t H, int32_t block_size,
                          procmv_strategy strategy, double cache_fraction,
                          procmv_precision precision, void* stream);

/* Y = H X for nvec vectors (paper Eq. generic_multivector, Y = A X).  X and Y
 * are device complex64 (nvec, ld*) buffers that must not overlap.  Needs a
 * plan.  Enqueues on `stream`; does not synchronise. */
procmv_status procmv_apply(procmv_op_t H, const void* X, int64_t ldx,
                           void* Y, int64_t ldy, int32_t nvec, void* stream);

/* Allocation-free form of procmv_apply, for callers that cannot allocate
 * device memory during the call (code under HIP stream capture, tight
 * serving loops, harnesses that forbid hipMalloc).  Same arguments, kernels
 * and results as procmv_apply (bit-identical outputs), but the partial slots
 * of the product live in a static device workspace of 64 MiB that the
 * library's code object holds on every device it runs on until the process
 * ends, instead of the operator's own buffer; the call allocates and frees
 * nothing and records no timing events (procmv_profile_enable does not
 * cover it).  The operator must already be created and planned (those calls
 * allocate).  Every call on one device shares that device's workspace and
 * overwrites it (every partial slot is written before it is read, so no
 * clearing is needed): calls that overlap on one device, on different
 * streams or threads, race and give wrong results.  PROCMV_ERR_INVALID_ARG
 * when a vector block's partial slots (slots x vectors per launch x D x 8
 * bytes: e.g. 8.4 MB for the procedural sinc-DVR operator at D = 32768 and
 * one vector, 33.8 MB per vector for a Philox-GUE operator at D = 32768)
 * exceed the workspace, and for the argument errors of procmv_apply. */
procmv_status procmv_apply_noalloc(procmv_op_t H, const void* X, int64_t ldx,
                                   void* Y, int64_t ldy, int32_t nvec, void* stream);

/* Default spectral bounds used by procmv_chebyshev_propagate when spec_R is
 * not positive: GUE c = 0, R = 2.5 (semicircle edge 2 plus margin); DVR
 * E_min = 0, E_max = pi^2/(2 mass dx^2) + max V. */
procmv_status procmv_spectral_bounds(procmv_op_t H, double* c, double* R);

/* Largest Lanczos step count accepted by procmv_lanczos_bounds. */
#define PROCMV_LANCZOS_MAX_STEPS 256

/* Matrix-free Lanczos estimate of the spectral bounds (paper Sec. VII: a short
 * Lanczos run, m = 40 in the paper, gives E_min and E_max and hence the
 * Chebyshev shift c = (E_max + E_min)/2 and half-width R = (E_max - E_min)/2).
 * Plain three-term recurrence without reorthogonalisation from the start
 * vector v0: v_1 = v0/||v0||, w = H v_j, alpha_j = Re <v_j, w>,
 * w -= alpha_j v_j + beta_{j-1} v_{j-1}, beta_j = ||w||, v_{j+1} = w/beta_j.
 * The products run in the tile kernels of the current plan (binary32 entries
 * and vectors); inner products and norms are binary64; the m x m tridiagonal
 * eigenproblem is solved on the host.  The extreme Ritz values are widened by
 * their residual estimates |beta_m s_m| (s = unit eigenvector of T_m):
 *   bounds_out (HOST, 6 doubles): E_min, E_max, theta_min, theta_max,
 *                                 r_min, r_max.
 * v0: device complex64, D entries, not modified (any nonzero vector; the
 * tests draw a seeded complex Gaussian).  1 <= m <= min(D, 256).
 * alpha_out, beta_out (HOST, m doubles each, may be NULL) receive the
 * recurrence coefficients; steps_out (may be NULL) the step count, which is
 * below m only if some beta_j is exactly zero.  Requires a plan.  Workspace
 * (3 D complex64 + (1024 + 2m) doubles) is allocated on first use and kept
 * with H.  SYNCHRONISES the stream.  PROCMV_ERR_INVALID_ARG for a null v0 or
 * bounds_out or m out of range; PROCMV_ERR_INTERNAL if a coefficient is not
 * finite (v0 zero or not finite). */
procmv_status procmv_lanczos_bounds(procmv_op_t H, const void* v0, int32_t m,
                                    double* bounds_out, double* alpha_out,
                                    double* beta_out, int32_t* steps_out, void* stream);

/* Limits of procmv_kron_apply. */
#define PROCMV_KRON_MAX_SYS 8
#define PROCMV_KRON_MAX_INT 3

/* System-bath Kronecker product Y = H X (paper Sec. VII example:
 * H = H_S (x) I_B + I_S (x) H_B + g sum_a A_a (x) B_a, applied without forming
 * H; Sec. IV-A: the bath operators act on R = d_S vectors at once).  X, Y:
 * device complex64 of d_S * d_B entries, X[s * d_B + j] = component
 * |s> (x) |j> (the d_S x d_B matrix, row-major); X and Y must not overlap.
 * HB: the bath Hamiltonian, B[0..n_int): the interaction bath operators, all
 * planned operators of the same D = d_B (any generator and plan; each product
 * runs in its own plan's tile kernels, on the d_S rows of X).  HS (HOST,
 * complex128 interleaved, d_S x d_S row-major) and A (HOST, n_int such
 * matrices) are used as given (Hermitian for a Hermitian H) and rounded to
 * binary32 in the mixing kernel.  1 <= d_S <= 8, 0 <= n_int <= 3.
 * Workspace (1 + n_int) d_S d_B complex64 is allocated on first use and kept
 * with HB.  Asynchronous on the stream.  PROCMV_ERR_INVALID_ARG for null
 * pointers, sizes out of range, mismatched D or overlapping X and Y;
 * PROCMV_ERR_NOT_PLANNED if an operator has no plan. */
procmv_status procmv_kron_apply(procmv_op_t HB, const procmv_op_t* B, int32_t n_int,
                                int32_t dS, const double* HS, const double* A, double g,
                                const void* X, void* Y, void* stream);

/* Real-time propagation of a system-bath state, psi <- exp(-i H dt)^nsteps
 * psi, with H the operator of procmv_kron_apply (same arguments HB, B, n_int,
 * d_S, HS, A, g) and the centered Chebyshev expansion of
 * procmv_chebyshev_propagate (paper Sec. VII: the example propagates its
 * system-bath state this way).  Every term is one procmv_kron_apply plus one
 * binary32 vector kernel (q_{k+1} = 2 alpha (H q_k - c q_k) - q_{k-1},
 * alpha = 1/R rounded down to a binary32 value and R widened to 1/alpha,
 * alpha c as a hi + lo pair; binary64 coefficient sum).  spec_c, spec_R: the caller's
 * spectral centre and half-width (R > 0; they must enclose the spectrum, e.g.
 * from procmv_lanczos_bounds-style estimates with a margin).  K <= 0:
 * procmv_cheb_order(R dt, 1e-10).  psi: device complex64, d_S * d_B entries
 * (layout of procmv_kron_apply), in place.  norms_out (HOST, may be NULL):
 * nsteps binary64 norms, SYNCHRONISES the stream when given.  Workspace
 * (2 d_S d_B complex64 + d_S d_B complex128) is kept with HB.
 * PROCMV_ERR_INVALID_ARG as procmv_kron_apply, or for R <= 0, dt < 0,
 * nsteps < 0 or d_S d_B >= 2^31. */
procmv_status procmv_kron_propagate(procmv_op_t HB, const procmv_op_t* B, int32_t n_int,
                                    int32_t dS, const double* HS, const double* A, double g,
                                    void* psi, double dt, int32_t K, int32_t nsteps,
                                    double spec_c, double spec_R, double* norms_out,
                                    void* stream);

/* Chebyshev order for argument x = R dt and coefficient tolerance tol: the
 * first k >= x with 2|J_k(x)| < tol and 2|J_{k+1}(x)| < tol. */
int32_t procmv_cheb_order(double x, double tol);

/* Real-time propagation psi <- exp(-i H dt)^nsteps psi by the centered
 * Chebyshev expansion (paper Sec. VII: Ht = (H - c)/R, q_0 = psi,
 * q_1 = Ht q_0, q_{l+1} = 2 Ht q_l - q_{l-1}; coefficients
 * (2 - delta_k0)(-i)^k J_k(R dt), Tal-Ezer & Kosloff).  Each step runs K + 1
 * terms (K <= 0: procmv_cheb_order(R dt, 1e-10)); the coefficient sum is
 * accumulated in binary64 and rounded to complex64 once per step.  psi:
 * device complex64 (nvec, ld), updated in place.  spec_R <= 0 selects
 * procmv_spectral_bounds.  norms_out (HOST, may be NULL): nsteps * nvec
 * binary64 norms ||psi|| after each step.  SYNCHRONISES the stream when
 * norms_out is given. */
procmv_status procmv_chebyshev_propagate(procmv_op_t H, void* psi, int64_t ld,
                                         int32_t nvec, double dt, int32_t K,
                                         int32_t nsteps, double spec_c,
                                         double spec_R, double* norms_out,
                                         void* stream);

/* Chebyshev order of the imaginary-time filter for z = R tau: the first k
 * with 2 e^{-z} I_k(z) < tol and 2 e^{-z} I_{k+1}(z) < tol (at least 1);
 * -1 for z < 0 or tol <= 0. */
int32_t procmv_filter_order(double z, double tol);

/* Imaginary-time Chebyshev filter psi <- exp(-tau H) psi (paper Sec. I/VII:
 * the TPQ states are prepared by an imaginary-time Chebyshev filter
 * e^{-beta H/2} applied to random vectors; here tau = beta/2).  Same
 * recurrence as procmv_chebyshev_propagate (Ht = (H - c)/R, q_0 = psi,
 * q_1 = Ht q_0, q_{l+1} = 2 Ht q_l - q_{l-1}) with the coefficients of
 * e^{-z x} = I_0(z) + 2 sum_k (-1)^k I_k(z) T_k(x), z = R tau, used in the
 * exponentially scaled form e^{-z} I_k(z) with the factor
 * e^{-tau (c - R)} = e^{-tau E_min} applied once at the end; binary64
 * accumulation.  The result is NOT normalised: norms_out (HOST, may be NULL)
 * receives the nvec binary64 norms ||exp(-tau H) psi||, and SYNCHRONISES
 * the stream when given.  K <= 0: procmv_filter_order(R tau, 1e-10).
 * spec_R <= 0 selects procmv_spectral_bounds (c, R must enclose the spectrum,
 * or the expansion grows).  psi: device complex64 (nvec, ld), in place.
 * PROCMV_ERR_INVALID_ARG for bad sizes, tau < 0, or a factor e^{-tau E_min}
 * that overflows or underflows binary64. */
procmv_status procmv_chebyshev_filter(procmv_op_t H, void* psi, int64_t ld, int32_t nvec,
                                      double tau, int32_t K, double spec_c, double spec_R,
                                      double* norms_out, void* stream);

/* Test hook: the generated binary32 entries H[r0:r0+nr, c0:c0+nc] written to
 * out_dev (device, complex64, row-major nr x nc), through the same generator
 * code as the products.  Needs no plan. */
procmv_status procmv_get_entries(procmv_op_t H, int64_t r0, int64_t c0,
                                 int32_t nr, int32_t nc, void* out_dev,
                                 void* stream);

/* Test hook for the generator's binary32 definition (paper Sec. III seeded
 * generation; the transform is fixed as IEEE operations): the kernels divide
 * and take square roots with short sequences (reciprocal or root estimate
 * plus one residual correction) and evaluate the logarithm, sine and cosine
 * in a rearranged but bitwise equal form (uniform scaled by 2^32, factor -2
 * folded into the series constants, quadrant signs by XOR).  This runs, for
 * all 2^23 uniforms the generator can draw, the logarithm with the short
 * division against the compiler's IEEE division, the rearranged -2 ln u,
 * sine and cosine against the plain ones (counted with the logarithm), and
 * the short square root of -2 ln u against the IEEE square root, and returns
 * the numbers of bitwise mismatches (host int32s; both 0 means the entries
 * equal the IEEE definition).  Allocates
 * and frees 8 bytes of device memory; SYNCHRONISES the stream. */
procmv_status procmv_selftest_generator(int32_t* ln_mismatches,
                                        int32_t* sqrt_mismatches, void* stream);

/* Plan summary (host): block size, block count, canonical pairs, cached
 * pairs, cache bytes, workspace bytes. */
typedef struct {
    int64_t D;
    int32_t block_size, n_blk;
    int64_t n_pair, p_cache;
    int64_t cache_bytes, work_bytes;
    int32_t strategy, precision;
} procmv_plan_info_t;
procmv_status procmv_plan_info(procmv_op_t H, procmv_plan_info_t* info);

/* Measurement hook (paper Sec. IV-C: measured time per product, timed
 * with device-side events).  With every > 0, the library records a pair of
 * HIP events on the launch stream around every `every`-th launch of the
 * block-product (tile) kernel and of the partial-reduction kernel issued
 * through this handle; every <= 0 switches recording off and clears the
 * record.  procmv_profile_read synchronises the recorded events and returns
 * the summed durations (ms) and the number of timed launches of each kernel,
 * then clears the record. */
procmv_status procmv_profile_enable(procmv_op_t H, int32_t every);
procmv_status procmv_profile_read(procmv_op_t H, double* tile_ms,
                                  int64_t* tile_launches, double* reduce_ms,
                                  int64_t* reduce_launches);

/* Measured tile-shape tuning (paper Sec. IV-C, Algorithm 2, applied to the
 * kernel's launch shape): times `reps` products of nvec scratch vectors for
 * each VALU tile shape (-1, 0, 1, 2; see procmv_set_tile_shape) and keeps the
 * fastest for this handle.  Allocates and frees its scratch vectors;
 * SYNCHRONISES the stream.  *shape_out / *best_ms (host, may be NULL) receive
 * the choice and its mean time per product. */
procmv_status procmv_autotune(procmv_op_t H, int32_t nvec, int32_t reps,
                              void* stream, int32_t* shape_out, double* best_ms);

/* Set the VALU tile shape (0, 1, 2: 8, 16, 32 direct values per lane and
 * vector block) explicitly, or -1 for the default that procmv_plan sets:
 * shape 0 for every class of super-tiles (all canonical pairs cached, none
 * cached, mixed when the block size is below the super-tile edge), one
 * launch per class.
 * Shapes whose tile rows exceed the super-tile edge (64 entries for
 * D <= 5632, 128 for D <= 11264, else 256) are reduced to the largest that
 * fits.  With one explicit shape, products are bit-identical across storage
 * modes and block sizes. */
procmv_status procmv_set_tile_shape(procmv_op_t H, int32_t shape);

/* Kernel of the procedural sinc-DVR product (paper Sec. III analytic
 * generation fused with the block product; the operator is Toeplitz plus a
 * diagonal): kind 1 = VALU Toeplitz kernel (symbol window in LDS, binary32
 * FMA), kind 2 = matrix-core Toeplitz kernel for one-vector launches (32 x 32
 * Toeplitz blocks T_d shared by every output block, binary32 MFMA
 * 32x32x2), kind 3 = the same blocks on the bfloat16 matrix cores: every
 * binary32 entry and vector component is split exactly into three bfloat16
 * pieces (hi + mid + lo, each rounded to nearest) and the six piece products
 * down to the binary32 rounding level (hh, hm, mh, hl, lh, mm) are
 * accumulated in binary32 by MFMA 32x32x16, the hh products and the smaller
 * ones in separate sums (split-BF16 application with a third piece; the
 * dropped products are at most 2^-23 of each entry's product, about 2^-27
 * in root mean square, and of either sign), kind 0 =
 * automatic (kind 3 for one vector from D = 16384 on, VALU otherwise).
 * Launches of several vectors always take the VALU kernel.  All apply the
 * same binary32 entries; kinds 1 and 2 differ in summation order only, and
 * kind 3's products are as accurate as theirs (measured at D = 32768: error
 * 6.8e-11 R |x| per product, against 2.5e-10 for kind 2). */
procmv_status procmv_set_dvr_kernel(procmv_op_t H, int32_t kind);

/* Tile shape the VALU tile kernel runs for a requested shape (0-2), a launch
 * of nvec vectors (1, 2, 4 or 8) on an operator of dimension D: the largest
 * shape not above `shape` whose tile rows 4 RW (RW = (8, 16, 32) / (2 nvec))
 * fit the super-tile edge (64, 128 or 256, from D) and, when the super-tiles
 * read a block cache of block size cache_block (0 = none), divide
 * cache_block, so that a cached tile never leaves its b x b slot.  Host
 * only; -1 for arguments out of range. */
int32_t procmv_tile_shape_fit(int32_t nvec, int32_t shape, int64_t D, int32_t cache_block);

/* Measured microbenchmark of one (operator, plan) pair (paper Sec. IV-C,
 * Eq. measured_matvec_time): creates the operator, plans it, times the cache
 * fill (the fill kernels re-run on the allocated slots: allocation is left
 * out, its time depends on the allocator's history) and the mean of `reps`
 * products of nvec vectors after `warmup` untimed ones, then releases
 * everything.  Times in ms (host outputs; fill 0 without a cache).  Returns
 * PROCMV_ERR_OOM when the plan or the vectors do not fit.  SYNCHRONISES the
 * stream. */
procmv_status procmv_measure(procmv_generator gen, uint64_t seed, int64_t D,
                             const void* gen_params, int32_t nvec,
                             int32_t block_size, procmv_strategy strategy,
                             double cache_fraction, procmv_precision precision,
                             int32_t warmup, int32_t reps, void* stream,
                             double* t_fill_ms, double* t_apply_ms);

/* ---- Execution planner (paper Sec. IV). ----------------------------------
 * Candidates: block size b in {128, ..., 4096} x storage mode {procedural,
 * partial f = 0.25 / 0.5 / 0.75, full}; index = 5 * log2(b / 128) + mode.
 * Memory model: cache = cached canonical pairs x b^2 x bytes per entry
 * (Eq. planner_partial_cache over canonical pairs); workspace (Eq.
 * planner_workspace) = partial slots + input/output vectors (+ Chebyshev
 * vectors when reuse > 1); a plan is feasible when cache + workspace <=
 * 0.9 x budget (Eq. planner_memory_constraint). */
int32_t procmv_plan_candidate_count(void);
procmv_status procmv_plan_candidate(int32_t idx, int32_t* block_size,
                                    int32_t* strategy, double* cache_fraction);

/* Surrogate features of (problem, plan) (paper Sec. IV-D, feature vector
 * x(p); this library's 8): log2 D, log2 nvec, log2(1 + cache MB), log2 reuse,
 * family (0 GUE, 1 DVR), log2 b, cached fraction (procedural 0, full 1),
 * M_tot / budget (the budget enters through this ratio and the memory test).
 * x_out: 8 floats (host).  *feasible_out = memory test. */
procmv_status procmv_plan_features(int64_t D, int32_t nvec, double budget_bytes,
                                   int64_t reuse, int32_t family,
                                   int32_t block_size, int32_t strategy,
                                   double cache_fraction, float* x_out,
                                   double* m_tot_out, int32_t* feasible_out);

/* Machine constants of the analytic cost model (paper Eqs. runtime_overlap,
 * seed_source_time, analytic_source_time: the throughput R_eff of the
 * cost score made concrete), measured by microbenchmarks. */
typedef struct {
    double gen_rate[2];  /* canonical entries produced per second: GUE, DVR */
    double dvr_rate;     /* sinc-DVR Toeplitz-kernel matrix elements per s   */
    double cache_bw;     /* bytes per second read from the block cache        */
    double flop_rate;    /* binary32 product flop/s (8 per complex element)   */
    double launch_s;     /* fixed cost of one product (launches, reduction)   */
} procmv_machine_model;

/* Analytic (Algorithm 1) time of a plan: fill and per-product time (s). */
procmv_status procmv_plan_model_time(const procmv_machine_model* mm, int64_t D,
                                     int32_t nvec, int32_t family,
                                     int32_t block_size, int32_t strategy,
                                     double cache_fraction, int64_t reuse,
                                     double* t_fill_s, double* t_apply_s);

/* Rank the memory-feasible candidates (paper Sec. IV-B, Algorithm 1's
 * enumeration and memory test, Eq. planner_memory_constraint; block sizes
 * above D are skipped except the smallest) by a model score, best first:
 * planner 0 = analytic t_fill + reuse t_apply (Algorithm 1 with the
 * procmv_plan_model_time model), planner 1 = learned exp(f(z)), the
 * surrogate's predicted total time (Algorithm 3, Eq. nn_pred_time).
 * mlp_params: procmv_mlp_param_count() floats; mlp_norm: 16 floats
 * (feature means then deviations).  order_out / score_out (HOST, room for
 * procmv_plan_candidate_count() entries, may be NULL) receive the candidate
 * indices and scores; *n_out the number of feasible candidates.
 * PROCMV_ERR_INFEASIBLE_PLAN when no candidate fits. */
procmv_status procmv_plan_rank(int32_t planner, const procmv_machine_model* mm,
                               const float* mlp_params, const float* mlp_norm,
                               int64_t D, int32_t nvec, double budget_bytes,
                               int64_t reuse, int32_t family, int32_t* order_out,
                               double* score_out, int32_t* n_out);

/* The best-ranked candidate of procmv_plan_rank (planner 0 or 1) and its
 * score.  Planners 2 and 3 time plans of an operator and are only offered by
 * procmv_plan_auto (PROCMV_ERR_INVALID_ARG here). */
procmv_status procmv_plan_choose(int32_t planner, const procmv_machine_model* mm,
                                 const float* mlp_params, const float* mlp_norm,
                                 int64_t D, int32_t nvec, double budget_bytes,
                                 int64_t reuse, int32_t family,
                                 int32_t* best_idx, double* best_score);

/* Candidates timed by the measured planners of procmv_plan_auto. */
#define PROCMV_PLAN_K_BENCH 4

/* Choose a plan for this operator and apply it (procmv_plan, binary32):
 *   planner 0: analytic (Algorithm 1), the best of procmv_plan_rank(0);
 *   planner 1: learned (Algorithm 3, direct), the best of procmv_plan_rank(1);
 *   planner 2: measured (Algorithm 2): the PROCMV_PLAN_K_BENCH best analytic
 *              candidates are each timed with procmv_measure on this
 *              operator's generator, seed and parameters (1 warm-up, 3 timed
 *              products), and the smallest measured t_fill + reuse t_apply
 *              wins (Eq. bench_argmin; one task, W = 1);
 *   planner 3: hybrid (Algorithm 3 with local measurement): the same over
 *              the PROCMV_PLAN_K_BENCH best learned candidates.
 * Planners 2 and 3 allocate and free the measured plans' memory and
 * SYNCHRONISE the stream; a timed candidate that does not fit is skipped.
 * *chosen_idx (may be NULL) receives the candidate index. */
procmv_status procmv_plan_auto(procmv_op_t H, int32_t nvec, double budget_bytes,
                               int64_t reuse, int32_t planner,
                               const procmv_machine_model* mm,
                               const float* mlp_params, const float* mlp_norm,
                               void* stream, int32_t* chosen_idx);

/* Surrogate network on the GPU (hand-written kernels): 8 inputs, two hidden
 * layers of 64 ReLU units, one output; parameters packed as W1 (8x64,
 * row-major), b1, W2 (64x64), b2, W3 (64), b3.  z: n x 8 normalised
 * features, t: n targets (log time), all HOST arrays; the calls copy to and
 * from the device and synchronise. */
int32_t procmv_mlp_param_count(void);
/* One forward/backward pass: gradient of the mean squared error (Eq.
 * nn_loss) with respect to every parameter, and the loss. */
procmv_status procmv_mlp_grad(const float* params, const float* z,
                              const float* t, int32_t n, float* grad_out,
                              float* loss_out);
/* `epochs` full-batch Adam steps from params_inout (updated in place);
 * loss_hist (may be NULL): loss before each step. */
procmv_status procmv_mlp_train(const float* z, const float* t, int32_t n,
                               int32_t epochs, float lr, float* params_inout,
                               float* loss_hist);
procmv_status procmv_mlp_predict(const float* params, const float* z,
                                 int32_t n, float* y_out);

/* ---- Batches of independent operators (single-GPU form of the paper's
 * parameter-parallel execution, Sec. IV-G and Eq. planner_waves: independent
 * tasks share the device instead of waiting for waves). -------------------
 * All operators of a batch are planned, binary32, of one generator family,
 * and must outlive the batch.  Vectors are PACKED in one device complex64
 * buffer: instance k holds nvec vectors of length D_k, each contiguous,
 * starting at element off_k = sum_{l<k} nvec * D_l.  One persistent launch
 * walks every (instance, super-tile) item (super-tiles of edge 256; VALU or
 * matrix cores by the routing rule of procmv_apply);
 * a second launch reduces all partials in a fixed order.  A batched product
 * does not depend on the grid or the item order, and is bit-identical to an
 * instance's own product when that runs the same kernel on the same
 * super-tiles (same tile shape; D > 11264). */
typedef struct procmv_batch* procmv_batch_t;

/* nvec in {1, 2, 4, 8}.  Allocates the packed partial buffers. */
procmv_status procmv_batch_create(const procmv_op_t* ops, int32_t n,
                                  int32_t nvec, procmv_batch_t* out);

/* Packed element count, number of work items and the launch configuration
 * (tile shape 0-2, persistent grid size, item order 0 = round-robin over
 * instances largest first, 1 = instance by instance).  Any pointer may be
 * NULL. */
procmv_status procmv_batch_info(procmv_batch_t B, int64_t* total,
                                int64_t* items, int32_t* shape, int32_t* grid,
                                int32_t* order);
procmv_status procmv_batch_configure(procmv_batch_t B, int32_t shape,
                                     int32_t grid, int32_t order);

/* Y_k = H_k X_k for every instance (packed X, Y; no overlap).  Async. */
procmv_status procmv_batch_apply(procmv_batch_t B, const void* X, void* Y,
                                 void* stream);

/* Autotuner of the batched launch: times `reps` batched products for every
 * (item order, tile shape, grid = {1,2,4,8} x compute units) and keeps the
 * fastest.  SYNCHRONISES the stream. */
procmv_status procmv_batch_autotune(procmv_batch_t B, const void* X, void* Y,
                                    int32_t reps, void* stream,
                                    double* best_ms);

/* nsteps Chebyshev steps (as procmv_chebyshev_propagate) of every instance
 * with one (c, R), dt and order K for all (K <= 0: the coefficient rule,
 * tol 1e-10).  With use_graph != 0 one step is captured once as a HIP graph
 * (re-captured when psi, dt, K, c or R change) and replayed nsteps times.
 * norms_out (HOST, may be NULL): n * nvec binary64 norms after the last
 * step; SYNCHRONISES the stream when given. */
procmv_status procmv_batch_propagate(procmv_batch_t B, void* psi, double dt,
                                     int32_t K, int32_t nsteps, double spec_c,
                                     double spec_R, int32_t use_graph,
                                     double* norms_out, void* stream);

void procmv_batch_destroy(procmv_batch_t B);

/* Release the operator and every device buffer it owns. NULL is ignored. */
void procmv_destroy(procmv_op_t H);

/* Message of the calling thread's last error ("" if none). */
const char* procmv_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PROCMV_H */
