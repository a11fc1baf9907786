/*
 * cpamg.h -- C ABI of the gfx950 hot path for multigrid CP decomposition.
 *
 * Method: H. De Sterck and K. Miller, "An adaptive algebraic multigrid
 * algorithm for low-rank canonical tensor decomposition".  The library runs the
 * ALS relaxation sweep (Section 3), the multilinear restriction and
 * prolongation of the setup phase (Section 4.1) and the CP-FAS V-cycle of the
 * solve phase (Section 5, Algorithm 2) on one AMD Instinct MI355X.
 *
 * Conventions shared by every call
 * --------------------------------
 * Pointers are DEVICE pointers unless a parameter says (host).
 * Tensor layout: dense, mode 1 fastest: entry (i_1..i_N) sits at
 *   i_1 + I_1*(i_2 + I_2*(i_3 + ...)), 0-based indices.
 * Factor layout: A^(n) is I_n x R, row-major with r fastest (leading dim R).
 * Mode numbers in this interface are 0-based (mode n here is mode n+1 of the
 * paper).  Rank R <= CP_MAX_RANK, order 2 <= N <= CP_MAX_ORDER.
 *
 * Ownership: the caller owns every tensor, factor and output buffer.  The
 * library allocates only its own workspace inside the context; it grows on
 * demand (the stream is synchronized before a reallocation) and is released by
 * cp_ctx_destroy.  No caller pointer is retained after a call returns.
 *
 * Asynchrony: every compute call only enqueues work on the context's stream and
 * returns; outputs are valid once that stream has been synchronized.  Scalar
 * results (f, g, norms) are written to device memory, so no call synchronizes
 * except cp_get_status and workspace growth.
 *
 * Errors: argument errors are found on the host before anything is enqueued:
 * the call returns a negative cp_status, writes nothing, and cp_last_error()
 * describes the problem.  Numerical events found on the device are OR-ed into
 * a device flag word read by cp_get_status().  No exception or abort crosses
 * the ABI.  A context is used by one host thread at a time.
 *
 * Precision: CP_FP64 computes everything in IEEE double.  CP_MIXED runs the
 * tensor contractions (MTTKRP GEMM stage, restriction GEMMs) in FP32 on the
 * matrix cores with FP32 accumulation, reading the FP32 shadows z32 / a32;
 * the Hadamard-reduce stage, Gram matrices, R x R solves, objective and FAS
 * right-hand sides stay in FP64.
 */
#ifndef CPAMG_H
#define CPAMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CP_MAX_ORDER 8
#define CP_MAX_RANK 32

typedef enum {
  CP_OK = 0,
  CP_ERR_INVALID = -1,     /* NULL or inconsistent argument */
  CP_ERR_SHAPE = -2,       /* dimension / rank outside the supported range */
  CP_ERR_NOT_SPD = -3,     /* reported by cp_get_status when a solve failed */
  CP_ERR_NONFINITE = -4,   /* reported by cp_get_status on NaN/Inf */
  CP_ERR_HIP = -5,         /* a HIP runtime call failed (message in cp_last_error) */
  CP_ERR_NOMEM = -6,       /* workspace allocation failed */
  CP_ERR_UNSUPPORTED = -7  /* valid request that the library does not implement */
} cp_status;

typedef enum { CP_FP64 = 0, CP_MIXED = 1 } cp_prec;
typedef enum { CP_SOLVE_CHOL = 0, CP_SOLVE_GS = 1 } cp_solver;

/* Device flag bits reported by cp_get_status(). */
#define CP_FLAG_PINV_FALLBACK 1u  /* a Gamma had a pivot <= R*eps*max(diag): pseudoinverse used */
#define CP_FLAG_NOT_SPD 2u        /* a Gamma was zero: the update left A unchanged */
#define CP_FLAG_NONFINITE 4u      /* a non-finite value appeared in a solve */

typedef struct cp_ctx_s* cp_ctx;

/* Tensor.  Dense form (nnz == 0): z64: FP64 master (required by CP_FP64
 * calls); z32: FP32 shadow (required by CP_MIXED contractions; fill it with
 * cp_cast_f32).  norm2: device scalar holding ||Z||^2 in FP64 (cp_norm2
 * writes it); it is needed only where a call says so, NULL otherwise.
 *
 * Sparse form (nnz >= 1; Section 6.2: a relaxation then costs about N R nnz
 * operations): the tensor is given by its nonzero entries, FP64 only, and
 * z64 / z32 are ignored.
 *   idx:  nnz x order int32, row-major (entry k has indices idx[k*order + m]),
 *         0-based; no index tuple may appear twice.
 *   vals: nnz FP64 values.
 *   rowptr[m], perm[m] (m < order): the entries ordered by their mode-m index:
 *         perm[m][rowptr[m][i] .. rowptr[m][i+1]-1] are the ids k of the
 *         entries with index i in mode m, in increasing k (rowptr[m] has
 *         I_m + 1 int64 offsets, perm[m] nnz int32 ids); cp_sparse_index
 *         builds both on the host.
 * Calls that accept the sparse form say so; the others return
 * CP_ERR_UNSUPPORTED for it.  Every sparse call runs in FP64 (CP_MIXED:
 * CP_ERR_UNSUPPORTED). */
typedef struct {
  int32_t order;
  int64_t dims[CP_MAX_ORDER];
  const double* z64;
  const float* z32;
  const double* norm2;
  int64_t nnz;
  const int32_t* idx;
  const double* vals;
  const int64_t* rowptr[CP_MAX_ORDER];
  const int32_t* perm[CP_MAX_ORDER];
} cp_tensor;

/* Kruskal factors A^(0..N-1), each I_n x R row-major (FP64 master).  a32[n] is
 * the FP32 shadow used by CP_MIXED contractions (updated by the library
 * whenever it writes a[n]); may be NULL for CP_FP64. */
typedef struct {
  int32_t rank;
  double* a[CP_MAX_ORDER];
  float* a32[CP_MAX_ORDER];
} cp_factors;

/* One level of a multigrid hierarchy (Section 4.1, Algorithm 1/2).  z: the
 * level tensor (level 0 is the finest).  phat[n]: dense P^ = P L^{-T} of mode
 * n mapping the next coarser level to this one, I_n x I_{n,c} row-major, or
 * NULL when mode n is not coarsened on this level (n in I_c').  The coarsest
 * level has every phat[n] NULL. */
typedef struct {
  cp_tensor z;
  const double* phat[CP_MAX_ORDER];
} cp_level;

/* CP-FAS parameters (Table 1: nu1 = nu2 = 1, nuc = 50; Section 5.2: 10
 * Gauss-Seidel iterations).  ic_rule: coarse right-hand side for modes that
 * are not coarsened: 0 = tau-corrected F - H(A) + H_c(A~_c) (keeps the FAS
 * fixed point), 1 = Algorithm 2 as printed (F_c = F). */
typedef struct {
  int32_t nu1, nu2, nuc, gs_iters;
  int32_t ic_rule;
} cp_fas_params;

/* ---- context ---------------------------------------------------------- */

/* Create a context bound to the current HIP device and to `hip_stream`
 * (a hipStream_t; NULL = the legacy default stream).  *out receives the
 * handle. */
cp_status cp_ctx_create(cp_ctx* out, void* hip_stream);
/* Synchronize the context's stream, free its workspace and the handle. */
cp_status cp_ctx_destroy(cp_ctx ctx);
/* Re-bind the context to another stream (work already enqueued stays where it is). */
cp_status cp_set_stream(cp_ctx ctx, void* hip_stream);

/* Context options (host values):
 *   CP_OPT_DIMTREE (default 1): ALS/BNGS sweeps of order N >= 3 reuse the
 *     stage-1 GEMM tiles of the mode-1 MTTKRP, Y = Z x_1 A^(1)T (exact in exact
 *     arithmetic), for the MTTKRPs of modes >= 2, so a sweep streams Z twice
 *     instead of N times; used when Y takes at most a quarter of Z's bytes.
 *     0: every mode streams Z.
 *   CP_OPT_GRAPHS (default 1): cp_fas_vcycle records its launch sequence into
 *     a HIP graph the first time it sees an argument set (level tensors,
 *     transfer operators, factors, parameters, precision) and replays the graph
 *     on later calls with the same set; changing an option or growing the
 *     workspace drops the recorded graphs.  Not while per-kernel profiling is
 *     on.  0: every call launches its kernels one by one.
 *   CP_OPT_SMALL_LEVELS (default 1): Gauss-Seidel relaxations without
 *     normalization (every coarse level of cp_fas_vcycle, and cp_als_sweep with
 *     CP_SOLVE_GS, normalize == 0 and no f_hist) on a tensor that fits in LDS
 *     with its stage-1 tiles (about 150 KB; R <= 16) run all their sweeps in one
 *     workgroup, tensor and factors resident in LDS, arithmetic in FP64.
 *     0: the general per-mode kernels.
 * Returns CP_ERR_INVALID for an unknown option or value. */
#define CP_OPT_DIMTREE 1
#define CP_OPT_GRAPHS 2
#define CP_OPT_SMALL_LEVELS 3
cp_status cp_set_option(cp_ctx ctx, int32_t option, int32_t value);
/* Text of the last host-side error of this context ("" if none); owned by ctx. */
const char* cp_last_error(cp_ctx ctx);
/* Synchronize the stream, return the OR of device flag bits since the last call
 * in *flags (host) and clear them. */
cp_status cp_get_status(cp_ctx ctx, int32_t* flags);

/* ---- utilities -------------------------------------------------------- */

/* dst[i] = (float)src[i], i < count (FP32 shadow of a tensor or factor). */
cp_status cp_cast_f32(cp_ctx ctx, const double* src, float* dst, int64_t count);
/* *out (device) = ||Z||^2 accumulated in FP64 from Z->z64 (sparse form: from
 * the stored values). */
cp_status cp_norm2(cp_ctx ctx, const cp_tensor* Z, double* out);

/* Mode orderings of a sparse tensor (host only, no device work).  idx (host):
 * nnz x order int32 0-based indices as in cp_tensor; dims (host): order
 * extents.  Writes rowptr (host, sum over m of dims[m] + 1 int64: the rowptr
 * arrays of modes 0, 1, ... back to back) and perm (host, order x nnz int32:
 * perm of mode m at perm + m*nnz), ordering each mode's entries by index and,
 * within one index, by entry id.  ctx may be NULL (no device is touched; the
 * error message is then not kept).  Errors: CP_ERR_SHAPE for an order or extent
 * outside the supported range or nnz outside [1, 2^31 - 1]; CP_ERR_INVALID for
 * NULL pointers, an index outside its extent or an index tuple stored twice. */
cp_status cp_sparse_index(cp_ctx ctx, int32_t order, const int64_t* dims, int64_t nnz,
                          const int32_t* idx, int64_t* rowptr, int32_t* perm);

/* ---- hot path (the calls named by the method) -------------------------- */

/* MTTKRP of eq. (6): M = Z_(n) Phi^(n), Phi^(n) the Khatri-Rao product of all
 * factors but n in the order of eq. (7).  Computed as a matrix-core GEMM that
 * contracts one mode with its factor, followed by a Hadamard-reduce over the
 * remaining modes; the Khatri-Rao matrix is never formed.  M: I_n x R
 * row-major FP64 (written, not accumulated).  CP_MIXED reads z32/a32.  Sparse
 * form (FP64): the workgroups of output row i of mode n sum their share of the
 * entries with index i (in perm[n] order) into per-split partial sums that a
 * second launch adds in a fixed order; no atomics, so results repeat bit for
 * bit. */
cp_status cp_mttkrp(cp_ctx ctx, const cp_tensor* Z, const cp_factors* A, int32_t n,
                    double* M, cp_prec prec);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): cp_mttkrp
 * without any allocation.  Same arguments, launch configuration, kernels and
 * result as cp_mttkrp; the per-split partial sums go to a static device array
 * of CP_NOALLOC_SCRATCH_BYTES bytes that the library holds on every device it
 * has run on until the process ends (its address is looked up once per device
 * by cp_ctx_create), never to the context's workspace.  The call allocates no
 * device memory and calls no allocating routine.  Every call on one device
 * shares that device's array and leaves its contents behind (each call
 * overwrites what it reads, so nothing needs to start at zero): calls that
 * overlap on one device (two streams, two contexts, two host threads) race
 * and must be ordered by the caller.  Errors: as cp_mttkrp; CP_ERR_SHAPE when
 * the partial sums of this mode's launch (splits x I_n x R doubles) exceed the
 * array; CP_ERR_HIP when no context was ever created on the current device. */
#define CP_NOALLOC_SCRATCH_BYTES (32u << 20)
cp_status cp_mttkrp_noalloc(cp_ctx ctx, const cp_tensor* Z, const cp_factors* A, int32_t n,
                            double* M, cp_prec prec);
/* (Dense form only.) */

/* `nsweeps` iterations of block nonlinear Gauss-Seidel (Section 3 ALS, or the
 * FAS relaxation of Section 5.2 when F != NULL) on A^(n) Gamma^(n) =
 * Z_(n) Phi^(n) + F^(n), n = 0..N-1, updating A (and its shadows) in place.
 * solver: CP_SOLVE_CHOL = A^(n) <- (M + F) Gamma^dagger (Cholesky factor L,
 * applied through W = L^-1 as (M + F) W^T W; pseudoinverse fallback when a
 * pivot fails the test); CP_SOLVE_GS = `gs_iters` Gauss-Seidel iterations warm-started from
 * the current A^(n).  normalize != 0 applies eq. (10) after every sweep.
 * F: NULL for plain ALS, else F->a[n] (I_n x R FP64).  f_hist (optional,
 * device, nsweeps doubles): f = 1/2||Z - [[A]]||^2 after each sweep from the
 * fused identity (needs Z->norm2; with CP_MIXED it uses the FP32 MTTKRP).
 * Accepts the sparse form (FP64). */
cp_status cp_als_sweep(cp_ctx ctx, const cp_tensor* Z, cp_factors* A, const cp_factors* F,
                       int32_t nsweeps, cp_solver solver, int32_t gs_iters, int32_t normalize,
                       cp_prec prec, double* f_hist);

/* Objective eq. (2) and stopping measure eq. (30) at fixed A.  exact != 0:
 * f from one streaming pass over Z->z64 forming the residual on the fly;
 * exact == 0: fused identity 1/2(||Z||^2 - 2<A^(N), M^(N)> + 1^T(*Upsilon)1)
 * (needs Z->norm2).  f (device scalar, optional), g (device scalar, optional;
 * needs Z->norm2; N MTTKRPs in precision `prec`).  Sparse form (FP64): g as
 * above; f from the fused identity whatever `exact` says (the residual has
 * prod I_n entries, most of them outside the stored ones), with its relative
 * rounding error of about eps ||Z||^2 / f. */
cp_status cp_objective(cp_ctx ctx, const cp_tensor* Z, const cp_factors* A, int32_t exact,
                       double* f, double* g, cp_prec prec);

/* Coarse tensor eq. (15): Zc = Z x_{n : phat[n] != NULL} phat[n]^T, applied as
 * one mode-n matrix-core GEMM after another.  phat[n]: I_n x I_{n,c}
 * row-major, or NULL (identity).  Zc->dims must equal the coarse dims; CP_FP64
 * writes Zc->z64 from Z->z64, CP_MIXED writes Zc->z32 from Z->z32.  A sparse Z
 * (FP64) is first scattered into a dense workspace copy (the coarse tensor is
 * dense anyway: P^ = P L^{-T} has no zero entries). */
cp_status cp_restrict(cp_ctx ctx, const cp_tensor* Z, const double* const phat[CP_MAX_ORDER],
                      cp_tensor* Zc, cp_prec prec);

/* The same coarse tensor eq. (15) in factored form: with P^^T = L^{-1} P^T
 * (Section 4.1), each coarsened mode applies the interpolation stencil P^T
 * (three terms per coarse entry) and then forward substitution with the
 * bidiagonal Cholesky factor L of B = P^T P: one pass over the tensor and
 * about five flops per coarse entry, against 2 I_c flops of the dense GEMM.
 * w[n]: the interpolation weights of mode n as taken by cp_transfer_build
 * (I_n x 2, device), or NULL (identity).  Arithmetic is FP64 whatever the
 * storage; CP_MIXED reads Z->z32 and writes Zc->z32.  Sparse Z (FP64): as
 * cp_restrict.  Errors: as cp_restrict; a coarsened mode of extent < 2. */
cp_status cp_restrict_factored(cp_ctx ctx, const cp_tensor* Z, const double* const w[CP_MAX_ORDER],
                               cp_tensor* Zc, cp_prec prec);

/* Prolongation.  Ac_tilde == NULL: A = P^ Ac (eq. (18), coarse-grid correction
 * of the setup phase); else A += P^ (Ac - Ac_tilde) (eq. (28), FAS).  phat:
 * I x Ic row-major; Ac, Ac_tilde: Ic x R; A: I x R; all FP64.  With phat ==
 * NULL the identity is used (Ic must equal I). */
cp_status cp_prolong(cp_ctx ctx, int64_t I, int64_t Ic, int32_t R, const double* phat,
                     const double* Ac, const double* Ac_tilde, double* A);

/* Restriction of factors, eq. (21): Ac = P^^T A (Ic x R), FP64. */
cp_status cp_restrict_factor(cp_ctx ctx, int64_t I, int64_t Ic, int32_t R, const double* phat,
                             const double* A, double* Ac);

/* Least-squares interpolation weights of the setup phase (Section 4.4,
 * eqs. (19)-(20); Algorithm 1 step 3) for mode n.  A holds `groups` factor
 * sets side by side as column groups (group k: columns [k R_g, (k+1) R_g) of
 * every factor, R_g = A->rank / groups): the relaxed test blocks and, last,
 * the boot factors.  Groups 0..nfit-1 are fitted, group k with weight
 * ||A_k^(n)||^2 / ||G_k^(n)||^2 for the gradient G_k^(n) = A_k^(n) Gamma_k^(n) -
 * M_k^(n), M_k^(n) = Z_(n) Phi_k^(n), of f at that block (eq. (23)); ||G_k^(n)|| is
 * floored at 1e-8 ||M_k^(n)|| (the mode an ALS sweep solved last has a gradient
 * that vanishes identically: its computed norm is rounding noise).  For every fine point i (odd
 * 0-based index) w[i][0], w[i][1] (I_n x 2 row-major, device) are the weights of
 * the coarse points (i-1)/2 and (i+1)/2 (the latter absent at the right end of
 * an even extent: w[i][1] = 0) minimizing the weighted misfit of every fitted
 * column at i against its injected values at i - 1 and i + 1; rows of coarse
 * points are zero.  The output feeds cp_transfer_build.  FP64 (Z->z64, or the
 * sparse form).
 * Errors: bad group split, nfit outside [1, groups], mode extent < 2. */
cp_status cp_interp_weights(cp_ctx ctx, const cp_tensor* Z, const cp_factors* A, int32_t groups,
                            int32_t nfit, int32_t n, double* w);

/* Transfer operator of Section 4.1 / Algorithm 1 steps 4-6 for geometric
 * coarsening (Section 4.3): from per-row weights w (I x 2; row i odd (0-based)
 * interpolates from coarse points (i-1)/2 and (i+1)/2 with weights w[i][0],
 * w[i][1]; the last row of an even I uses w[i][0] only; rows of coarse points
 * are ignored) builds B = P^T P (tridiagonal), L = chol(B) (bidiagonal) and
 * writes phat = P L^{-T} (I x Ic row-major, Ic = ceil(I/2)). */
cp_status cp_transfer_build(cp_ctx ctx, int64_t I, const double* w, double* phat);

/* One CP-FAS V-cycle (Algorithm 2) from level 0 with F = 0 there, updating A
 * (level-0 factors, and shadows) in place.  levels[0..nlevels-1]: finest to
 * coarsest; each level tensor needs z64 (CP_FP64) or z32 (CP_MIXED).  Level 0
 * may be in the sparse form (CP_FP64; the coarser levels are dense).
 * Relaxation is BNGS with Gauss-Seidel inner solves; eq. (10) normalization is
 * applied on level 0 only.  params NULL = Table 1 defaults. */
cp_status cp_fas_vcycle(cp_ctx ctx, const cp_level* levels, int32_t nlevels, cp_factors* A,
                        const cp_fas_params* params, cp_prec prec);

/* ---- per-kernel timing ------------------------------------------------ */

/* Kernel classes reported by cp_profile_read (index into its arrays). */
enum {
  CP_PROF_MTTKRP_MODE0_F64 = 0, CP_PROF_MTTKRP_MODE1_F64, CP_PROF_MTTKRP_MODEN_F64,
  CP_PROF_MTTKRP_MODE0_F32, CP_PROF_MTTKRP_MODE1_F32, CP_PROF_MTTKRP_MODEN_F32,
  CP_PROF_UPDATE, CP_PROF_EPILOGUE_OTHER, CP_PROF_GAMMA_PREP, CP_PROF_NORMALIZE, CP_PROF_GRAM,
  CP_PROF_OTHER, CP_PROF_CLASSES
};

/* on != 0: from now on bracket every kernel launch of this context with a pair
 * of HIP events recorded on the context's stream (clears earlier records);
 * on == 0: stop recording (records are kept until read).  Not for use while
 * the stream is being captured into a graph. */
cp_status cp_profile_enable(cp_ctx ctx, int32_t on);
/* Synchronize the stream and return, per kernel class, the summed elapsed
 * milliseconds and the number of launches (host arrays of CP_PROF_CLASSES
 * entries); clears the records. */
cp_status cp_profile_read(cp_ctx ctx, double* ms, int32_t* counts);

/* Measurement aid: enqueue `reps` back-to-back launches of the MTTKRP kernel
 * of mode n exactly as cp_als_sweep launches it (same launch configuration,
 * with the sweep-bookkeeping workgroup working on scratch Grams and scales;
 * partial sums land in the workspace, neither M nor A is written), between two
 * HIP events recorded on the context's stream; synchronize and return the
 * mean milliseconds per launch in *ms (host).  When the dimension tree applies
 * (CP_OPT_DIMTREE on, order >= 3, Y at most a quarter of Z's bytes), mode 1 is
 * the launch that also stores Y into the workspace and modes >= 2 are the
 * launches that contract Y, which one untimed mode-1 launch fills first. */
cp_status cp_time_mttkrp(cp_ctx ctx, const cp_tensor* Z, const cp_factors* A, int32_t n,
                         cp_prec prec, int32_t reps, double* ms);

/* ---- launch-configuration autotuner ----------------------------------- */

/* Time candidate launch configurations (streaming workgroups, contraction
 * split, rows per wave, FP32 lane width, contracted factor staged in LDS or
 * read from global memory) of the MTTKRP kernel of every mode of Z at precision
 * `prec` and rank A->rank, `reps` launches each, with HIP events on the
 * context's stream, and keep the fastest per mode in the context.  When a
 * sweep of Z would use the dimension tree, the mode-1 launch that also stores
 * the stage-1 tiles is tuned on its own too (key suffix ";y").  Later calls
 * on tensors of the same shape, rank and precision use them. */
cp_status cp_autotune(cp_ctx ctx, const cp_tensor* Z, const cp_factors* A, cp_prec prec,
                      int32_t reps);
/* The tuned configurations as text, one line per (shape, rank, precision,
 * mode, and the tile-storing mode-1 launch):
 * "<key> <workgroups> <split> <rows> <lane width> <unstaged>"; owned by ctx,
 * valid until the next call on ctx. */
const char* cp_plans_export(cp_ctx ctx);
/* Load configurations in the cp_plans_export format (replaces matching keys;
 * the last field may be omitted: staged). */
cp_status cp_plans_import(cp_ctx ctx, const char* text);

/* Stable sort of the rank-one terms by decreasing lambda_r (remark after
 * eq. (10)); permutes the columns of every A^(n) (and shadows) in place. */
cp_status cp_sort(cp_ctx ctx, const int64_t* dims /*host, N*/, int32_t order, cp_factors* A);

/* ---- batched solves ------------------------------------------------------ */

#define CP_MAX_RESTARTS 8

/* One problem of a batch: its tensor (z64; z32 too for CP_MIXED; norm2 set,
 * e.g. by cp_norm2) and one factor set of rank restarts * R holding every
 * restart side by side: restart k owns columns [k R, (k + 1) R) of each A^(n)
 * (FP64, plus FP32 shadows for CP_MIXED), initialised by the caller. */
typedef struct {
  cp_tensor z;
  cp_factors a;
} cp_batch_problem;

/* Stopping rules of a batched solve, applied per restart after every sweep
 * (fit = 1 - sqrt(2 f / ||Z||^2) from the fused objective of the sweep):
 *   CP_MIXED: FP32-contraction sweeps in windows of `window32` sweeps until
 *   (fit_last - fit_first) / (window32 - 1) <= tol32 * fit_last over a window,
 *   then FP64 sweeps (all restarts of the problem together) until
 *   |fit_k - fit_{k-1}| <= tol64 * fit_k;  CP_FP64: the FP64 phase only.
 * A restart stops after max_sweeps sweeps over both phases (at least one FP64
 * sweep runs in the mixed form).  `chunk` sweeps are enqueued between two host
 * checks of whether any restart still runs. */
typedef struct {
  int32_t restarts;   /* 1..CP_MAX_RESTARTS, restarts * R <= CP_MAX_RANK */
  cp_prec prec;
  int32_t window32;   /* >= 2 */
  double tol32;
  double tol64;
  int32_t max_sweeps; /* >= 1 */
  int32_t chunk;      /* >= 1 */
  int32_t wg_kib;     /* tensor KiB each streaming workgroup of the batched
                         MTTKRP launches covers: 16..4096, 0 = 192 (the tile
                         size a tuner such as drivers.tune_batched picks) */
} cp_batch_params;

/* Batched form of the ALS solve (Section 3, stopping as in cp_batch_params):
 * `nprob` independent problems (host array of descriptors with device
 * pointers), each with `restarts` starts that share every pass over their
 * tensor: the MTTKRP of a problem runs at rank restarts * R and Gamma is kept
 * block-diagonal, so the restarts never couple.  One launch per mode covers
 * every problem.  The factor sets are updated in place (normalized as in
 * eq. (10), not sorted).  Outputs (device, optional): fits[b * restarts + k],
 * the fit after the last sweep of restart k of problem b (fused objective);
 * sweeps[(b * restarts + k) * 2 + phase], sweeps run in the FP32 (0) and FP64
 * (1) phases.  Blocks until every restart has stopped.  Errors: invalid
 * descriptors or parameters (nothing enqueued), a contracted mode too large
 * to stage in LDS (CP_ERR_UNSUPPORTED). */
cp_status cp_als_batched(cp_ctx ctx, const cp_batch_problem* probs, int32_t nprob,
                         const cp_batch_params* params, double* fits, int32_t* sweeps);

#ifdef __cplusplus
}
#endif

#endif /* CPAMG_H */
