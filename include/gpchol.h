/*
 * gpchol: dense Cholesky factorisation of symmetric positive-definite
 * covariance matrices and its reverse-mode derivative on AMD Instinct MI355X
 * (gfx950), with the triangular solves and log-determinant a Gaussian-process
 * log-density needs.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Matrices are row-major FP64 with a leading dimension
 *   max(1, n) <= ld <= 2^20: element (i, j) of X is X[i * ld + j].  (Row-major
 *   lower is the same memory as column-major upper.)  A leading dimension out
 *   of that range is GPC_ERR_ARG, found before anything is enqueued.
 * - Symmetric inputs are given by their lower triangle including the
 *   diagonal; the strict upper triangle of an input is never read.
 *   Triangular outputs are lower; their strict upper triangle is written as 0.
 * - Every data pointer is a DEVICE pointer on the handle's device and is owned
 *   by the caller; the library never frees caller memory.  Pointers named
 *   `*_host` are host memory read during the call only.
 * - Calls are asynchronous: they validate arguments on the host, enqueue work
 *   on the handle's HIP stream and return.  Results are ready when that stream
 *   reaches the enqueued work.  No exception crosses this interface.
 * - Status codes report argument and runtime errors; numerical failure of the
 *   factorisation (a non-positive or NaN pivot) is data, reported through the
 *   device integer `info`, as in LAPACK.
 * - n == 0 is valid everywhere and enqueues nothing (except that `info` and
 *   device scalar outputs are still written).
 * - A handle is not thread-safe; use one handle per host thread.
 */
#ifndef GPCHOL_H
#define GPCHOL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GPC_OK = 0,
    GPC_ERR_ARG = 1,        /* invalid argument: n < 0, ld outside [max(1,n), 2^20], NULL pointer,
                               bad enum, an output overlapping an input */
    GPC_ERR_NO_DEVICE = 2,  /* no HIP device is visible */
    GPC_ERR_ARCH = 3,       /* the current device is not gfx950 */
    GPC_ERR_HIP = 4,        /* a HIP runtime call failed; gpc_last_error() has the message */
    GPC_ERR_REFINE = 5,     /* iterative refinement did not reach its tolerance */
    GPC_ERR_ALLOC = 6,      /* workspace allocation failed */
    GPC_ERR_SWEEP = 7,      /* a one-launch solve sweep ran out of time; its results are NaN
                               (reported by gpc_check and gpc_solve_refined) */
    GPC_ERR_CAPTURE = 8     /* the stream is capturing a graph and the call would need work
                               that cannot be captured (see the batched entry points) */
} gpc_status;

typedef enum {
    GPC_FP64 = 0,   /* every step in FP64 */
    GPC_MIXED = 1   /* trailing SYRK/GEMM updates of factor and adjoint in FP32 on MFMA
                       (FP32 accumulation, subtracted from FP64 storage); diagonal
                       blocks, panels and log-determinant stay FP64 */
} gpc_precision;

typedef enum { GPC_NOTRANS = 0, GPC_TRANS = 1 } gpc_trans;

typedef struct {
    int32_t precision;     /* gpc_precision; default GPC_FP64 */
    int32_t block;         /* outer block size b of the blocked algorithms; 0 = library default
                              (factor: 512 in FP64 from n = 8192 up, else 256; adjoint: 512
                              from n = 8192 up in both forms, else 256; the adjoint uses at
                              most 512) */
    int32_t lookahead;     /* 1 = overlap the next diagonal step with the trailing update */
    int32_t refine_maxit;  /* maximum refinement iterations of gpc_solve_refined (default 10) */
    double  refine_tol;    /* stop when the normwise backward error eta_inf <= refine_tol (default 1e-12) */
    int32_t mixed_fallback; /* GPC_MIXED factor: 0 (default) = none: a lost pivot of the
                               FP32-updated Schur complement is reported in info, and a caller
                               that still holds A factors it again in FP64; 1 = the library
                               keeps a copy of A and does that itself (see gpc_factor and
                               gpc_get_fallback) */
    int32_t test_flags;    /* 0; 1 = start every one-launch solve sweep (a single right-hand
                              side) with its error flag raised: its waits return at once and
                              its solution entries are NaN, which tests the failure path */
    int32_t gemm_max_splits; /* largest split-K count of gpc_gemm (gpchol_ops.h); 0 = 32
                                (default), 1 = never split */
    int32_t batched_schedule; /* batched calls: 0 = library choice (default: grouped when the
                                 largest member has order >= 256, else persistent);
                                 1 = persistent (one workgroup per matrix, one launch);
                                 2 = grouped (every block step one launch over all members) */
    int32_t adjoint_group; /* gpc_adjoint: the B-bar updates of G consecutive reverse-sweep
                              steps are applied together, as products of inner dimension up to
                              G b (b a multiple of 128); 0 = library default (2 below
                              512-blocks, else 1), 1 = one
                              product of inner dimension b per step, 2..8 = G */
} gpc_options;

typedef struct gpc_handle gpc_handle;

/* Create a handle bound to the current HIP device and to `hip_stream`
 * (a hipStream_t; NULL = the default stream).  The handle owns a device
 * workspace that grows on demand and is freed by gpc_destroy.
 * Errors: GPC_ERR_ARG (h NULL), GPC_ERR_NO_DEVICE, GPC_ERR_ARCH, GPC_ERR_HIP. */
gpc_status gpc_create(gpc_handle** h, void* hip_stream);

/* Wait for the handle's stream, free its workspace and the handle. */
gpc_status gpc_destroy(gpc_handle* h);

/* Rebind the handle to another stream of the same device.  The new stream
 * first waits (a HIP event, no host wait) for all work enqueued on the old
 * one, because every call shares the handle's workspace; when either stream
 * is capturing a graph there is no such wait, and ordering the captured work
 * against the handle's other work is up to the caller. */
gpc_status gpc_set_stream(gpc_handle* h, void* hip_stream);

/* Wait for the handle's stream and report whether a one-launch solve sweep
 * (gpc_trsm with one right-hand side, gpc_gp_value, gpc_solve_refined) has
 * run out of time since the last check: GPC_ERR_SWEEP (the record is then
 * cleared; the results of that sweep are NaN) or GPC_OK. */
gpc_status gpc_check(gpc_handle* h);

/* Replace the handle's options (copied).  GPC_ERR_ARG on NULL, an unknown
 * precision, block not in {0, 32, 64, 128, 256, 512}, refine_maxit < 0 or
 * refine_tol <= 0. */
gpc_status gpc_set_options(gpc_handle* h, const gpc_options* opt);
gpc_status gpc_get_options(const gpc_handle* h, gpc_options* opt);

/* Factor (section 3.3.1: L11 = chol(A11), L21 = A21 L11^-T, then the Schur
 * complement A22 - L21 L21^T is factored the same way).  In place: on return
 * the lower triangle of A holds L and its strict upper triangle holds 0.
 * info_dev (device int32) receives 0, or j+1 for the first column j whose pivot
 * is not positive or is NaN; L is then unspecified.
 * Uses the handle's precision (GPC_MIXED: trailing updates in FP32).
 * GPC_MIXED with mixed_fallback set: A is first copied to a handle-owned
 * buffer (n x n doubles, grow-only), the call waits for the stream once to
 * read info, and on a failed pivot restores A and factors it again in FP64;
 * info then reports the FP64 result (so a matrix that is not SPD in FP64
 * still gets its failing column).  Such a call returns GPC_ERR_CAPTURE if
 * the stream is capturing a graph. */
gpc_status gpc_factor(gpc_handle* h, int64_t n, double* A, int64_t lda, int32_t* info_dev);

/* gpc_factor without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  The same FP64 factor as gpc_factor with lookahead off:
 * one stream (the handle's), no ordering events, no launch trace, no growth
 * of the handle's workspace.  Its only device memory beyond A and info_dev is
 * a library-owned static array of 128 x 128 doubles (128 KiB per GPU, held
 * until the process ends) for the inverse of the current diagonal block;
 * that need does not depend on n, so every n the argument checks accept fits.
 * All calls on one GPU share that array: calls that overlap in time on the
 * same GPU (from different streams or handles) race and give wrong results.
 * Errors: GPC_ERR_ARG as gpc_factor, and when the handle's precision is not
 * GPC_FP64 (the mixed form needs n-sized FP32 panel copies); GPC_ERR_HIP if
 * the array's device address cannot be found. */
gpc_status gpc_factor_noalloc(gpc_handle* h, int64_t n, double* A, int64_t lda, int32_t* info_dev);

/* *fell_back = 1 if the last gpc_factor on this handle was a GPC_MIXED call
 * whose FP32-updated factor failed and was redone in FP64, else 0. */
gpc_status gpc_get_fallback(const gpc_handle* h, int32_t* fell_back);

/* Reverse-mode derivative of the factor (section 3.3.2: the blocked gradient
 * with the diagonal of each diagonal block's adjoint halved and its upper
 * triangle zeroed).  Inputs: L (lower, not modified) and Lbar, the adjoint of
 * the lower triangle of L.  In place: the lower triangle of Lbar becomes Abar,
 * the gradient with respect to the independent lower-triangle entries a_ij
 * (i >= j) of the symmetric A (a perturbation of a_ij, i > j, moves both A_ij
 * and A_ji); its strict upper triangle becomes 0.  L and Lbar must not overlap
 * (GPC_ERR_ARG if their byte ranges intersect). */
gpc_status gpc_adjoint(gpc_handle* h, int64_t n, const double* L, int64_t ldl,
                       double* Lbar, int64_t ldlb);

/* Triangular solve with the factor (section 3.2, A x = b with A triangular):
 * B <- L^-1 B (trans = GPC_NOTRANS) or B <- L^-T B (GPC_TRANS).
 * B is n x nrhs row-major with leading dimension ldb >= max(1, nrhs); B must
 * not overlap L.  A single column is solved in one launch whose workgroups
 * wait on each other; every wait is bounded in time (100 ms): were one ever
 * to run out, the entries it guards are NaN and gpc_check (or the next
 * gpc_solve_refined) returns GPC_ERR_SWEEP. */
gpc_status gpc_trsm(gpc_handle* h, int32_t trans, int64_t n, int64_t nrhs,
                    const double* L, int64_t ldl, double* B, int64_t ldb);

/* log|A| = 2 * sum_i log L_ii (section 1: the GP log-density needs the
 * determinant of the covariance, taken here through its factor), accumulated
 * in FP64 in a fixed order (independent of launch shape).  out_dev: one
 * device double. */
gpc_status gpc_logdet(gpc_handle* h, int64_t n, const double* L, int64_t ldl, double* out_dev);

/* Iterative refinement (mixed precision): solve K x = y in FP64 with a
 * factor L of K that may carry FP32 rounding in its trailing updates
 * (GPC_MIXED).  x_0 = 0; then repeat d = L^-T L^-1 r, x += d, r = y - K x
 * (residual in FP64 from the lower triangle of K) until the normwise
 * backward error eta_inf = |r|_inf / (|K|_inf |x|_inf + |y|_inf) is at most
 * the handle's refine_tol, or refine_maxit iterations have run.  y, x: device
 * n-vectors; iters_dev (int32) and eta_dev (double): device scalars.  Waits
 * for the stream once per iteration to read eta.  Returns GPC_ERR_REFINE if
 * the tolerance was not reached (x, iters and eta are still written), and
 * GPC_ERR_SWEEP if one of its sweeps ran out of time (x is then not a
 * solution).  x must not overlap K, L or y. */
gpc_status gpc_solve_refined(gpc_handle* h, int64_t n, const double* K, int64_t ldk, const double* L,
                             int64_t ldl, const double* y, double* x, int32_t* iters_dev, double* eta_dev);

/* GP covariance (squared-exponential with one lengthscale per input
 * dimension, the kernel of the GP regression example, section 4.2):
 * K_ij = s2 exp(-1/2 sum_q (x_iq - x_jq)^2 / l_q^2) + sn2 [i == j], written to
 * the lower triangle of K (strict upper := 0).  X: n x d row-major device
 * array, 1 <= d <= 16.  theta: d+2 device doubles (s2, l_1..l_d, sn2). */
gpc_status gpc_gp_kgen_se(gpc_handle* h, int64_t n, int32_t d, const double* X, const double* theta,
                          double* K, int64_t ldk);

/* GP log-density pieces from the factor L of K (section 1: the density needs
 * the inverse and the determinant of the covariance, through its factor):
 * z = L^-1 y, alpha = L^-T z (device n-vectors), logdet = 2 sum log L_ii and
 * f = -1/2 z^T z - 1/2 logdet (device scalars; the constant -n/2 log 2 pi is
 * left out).  All sums in a fixed order. */
gpc_status gpc_gp_value(gpc_handle* h, int64_t n, const double* L, int64_t ldl, const double* y, double* z,
                        double* alpha, double* logdet_dev, double* f_dev);

/* The same pieces when L carries FP32 rounding (GPC_MIXED): alpha solves
 * K alpha = y by FP64 iterative refinement against K (gpc_solve_refined; its
 * iters_dev and eta_dev), z = L^T alpha (so that alpha = L^-T z holds for
 * this L, which keeps gpc_gp_lbar's seed the adjoint of y^T K^-1 y / 2 at
 * the refined alpha), logdet = 2 sum log L_ii and
 * f = -1/2 y^T alpha - 1/2 logdet.  K and L: lower triangles read.  Returns
 * gpc_solve_refined's status (GPC_ERR_REFINE: the outputs are still
 * written).  z must not overlap alpha, K, L or y. */
gpc_status gpc_gp_value_refined(gpc_handle* h, int64_t n, const double* K, int64_t ldk, const double* L,
                                int64_t ldl, const double* y, double* z, double* alpha, double* logdet_dev,
                                double* f_dev, int32_t* iters_dev, double* eta_dev);

/* Adjoint of the factor for that density: Lbar = tril(alpha z^T) - diag(1/L_ii)
 * (lower triangle; strict upper := 0). */
gpc_status gpc_gp_lbar(gpc_handle* h, int64_t n, const double* L, int64_t ldl, const double* alpha,
                       const double* z, double* Lbar, int64_t ldlb);

/* Chain rule from Abar (the adjoint of the lower-triangle entries of K, as
 * returned by gpc_adjoint) to theta:
 * grad_q = scale * sum_{i>=j} Abar_ij dK_ij / dtheta_q  (d+2 device doubles;
 * scale: device double or NULL for 1).  Fixed summation order. */
gpc_status gpc_gp_hypergrad_se(gpc_handle* h, int64_t n, int32_t d, const double* X, const double* theta,
                               const double* Abar, int64_t ldab, const double* scale_dev, double* grad_dev);

/* Batched forms: nb matrices of uneven order n_host[i] (>= 0), each stored
 * row-major with leading dimension n_host[i] at element offset off_host[i]
 * from the base pointer (the caller keeps them disjoint).  Two schedules
 * (gpc_options.batched_schedule) run the same blocked algorithms as
 * gpc_factor / gpc_adjoint (section 3.3) on every member:
 *  - persistent: one launch; workgroups take matrices from a device queue,
 *    largest first, and factor / differentiate each alone (inner block chosen
 *    per size bucket by gpc_autotune_batched, default 64);
 *  - grouped (the default once a member has order >= 256): block size 64,
 *    every block step one launch over all members that have it (the
 *    diagonal blocks one workgroup each, the products one workgroup per
 *    64 x 64 output tile of every member), so a large member is spread over
 *    many CUs.
 * The launches are captured once into a HIP graph per distinct (sizes,
 * offsets, pointers, schedule) and replayed on later calls.  If the handle's stream is itself being captured, the launch
 * is recorded into the caller's graph instead, provided the same call (same
 * sizes, offsets and pointers) has been made once outside the capture, which
 * prepares its plan; otherwise the call returns GPC_ERR_CAPTURE and enqueues
 * nothing.  The buffers of a plan recorded into a caller's graph stay
 * allocated until gpc_destroy (the graph must not be launched after that).
 * Concurrent launches of one handle's plan (graph replays on two streams)
 * share its queue counter and race.  Results are bitwise independent of
 * queue order.  info_dev: nb device int32 (0 or first failing column + 1).
 * The handle's precision applies: GPC_MIXED runs the trailing update and the
 * B-bar / R-bar products in FP32 on MFMA (operands rounded from FP64 on load,
 * FP32 accumulation subtracted from FP64 storage); diagonal blocks, panels and
 * the diagonal reverse step stay FP64.  The batched mixed factor has no FP64
 * fallback: a matrix whose FP32-updated Schur complement loses definiteness
 * reports it in info. */
gpc_status gpc_factor_batched(gpc_handle* h, int32_t nb, const int32_t* n_host, const int64_t* off_host,
                              double* base, int32_t* info_dev);
gpc_status gpc_adjoint_batched(gpc_handle* h, int32_t nb, const int32_t* n_host, const int64_t* off_host,
                               const double* Lbase, double* Lbarbase);
/* Factor then adjoint of every matrix in one launch (Lbar given, Abar out). */
gpc_status gpc_factor_adjoint_batched(gpc_handle* h, int32_t nb, const int32_t* n_host, const int64_t* off_host,
                                      double* base, double* Lbarbase, int32_t* info_dev);

/* Autotuner of the batched path: for each size bucket (n < 128, 256, 512,
 * 1024, larger) time factor+adjoint of a synthetic diagonally dominant batch
 * with inner blocks 32 and 64 (median of 3) and keep the faster.  If
 * cache_path is not NULL the choices are written there; handles read the file
 * named by the environment variable GPC_TUNE_CACHE at creation.  Waits for
 * the stream (GPC_ERR_CAPTURE if it is capturing).  gpc_get_tuning returns
 * the 5 bucket blocks and whether they come from tuning. */
gpc_status gpc_autotune_batched(gpc_handle* h, const char* cache_path);
gpc_status gpc_get_tuning(const gpc_handle* h, int32_t* blocks_out, int32_t* tuned);

/* Kernel classes reported by the launch trace below. */
typedef enum {
    GPC_K_DIAG_FACTOR = 0,      /* diagonal-block factor + inverse (one workgroup) */
    GPC_K_PANEL_SOLVE = 1,      /* L21 = A21 inv(L11)^T */
    GPC_K_TRAILING_UPDATE = 2,  /* A22 -= L21 L21^T (lower tiles, all but the next block's columns) */
    GPC_K_DIAG_INVERSE = 3,     /* inverses of all diagonal blocks (reverse sweep, solves) */
    GPC_K_ADJ_PANEL_SOLVE = 4,  /* Cbar <- Cbar D^-1 */
    GPC_K_ADJ_LEFT_UPDATE = 5,  /* Bbar -= Cbar R */
    GPC_K_ADJ_DIAG_PRODUCT = 6, /* split-K slices of Cbar^T C */
    GPC_K_ADJ_DIAG_BLOCK = 7,   /* Dbar <- Phi(D^-T sym(D^T Dbar) D^-1) (4 launches) */
    GPC_K_ADJ_ROW_UPDATE = 8,   /* split-K slices of [M; Cbar]^T [R; B] */
    GPC_K_REDUCE = 9,           /* fixed-order sum of split-K slices into Rbar */
    GPC_K_BATCHED = 10,         /* one persistent batched launch (graph replay) */
    GPC_K_TRAILING_NARROW = 11, /* trailing update of the next block's columns only */
    GPC_K_OPS = 12,             /* the entry points of gpchol_ops.h, one record per call */
    GPC_K_COUNT = 13
} gpc_kernel_class;

/* Launch trace, for measurement: while enabled, every launch of the classes
 * above is bracketed by a pair of HIP events on the handle's stream and its
 * algorithmic flops and bytes (the useful work of that launch, counted on the
 * host) are recorded.  gpc_trace_read waits for the stream and returns, for
 * one class, the number of launches, the sum of their event-measured
 * durations (ms), and the summed flops and bytes.  gpc_trace_reset waits for
 * the stream and forgets all records.  Tracing is off by default. */
gpc_status gpc_trace_enable(gpc_handle* h, int32_t on);
gpc_status gpc_trace_reset(gpc_handle* h);
gpc_status gpc_trace_read(gpc_handle* h, int32_t kclass, int64_t* launches, double* ms,
                          double* flops, double* bytes);

/* Static description of a status code (never NULL). */
const char* gpc_status_string(gpc_status s);

/* Message of the last GPC_ERR_HIP / GPC_ERR_ALLOC on this handle ("" if none). */
const char* gpc_last_error(const gpc_handle* h);

#ifdef __cplusplus
}
#endif
#endif /* GPCHOL_H */
