/*
 * gpchol operations beside the Cholesky path: the lower-triangular inverse
 * and the reverse modes of the triangular solve and of the inverse
 * (section 3.2), general matrix products with their reverse mode and the
 * special case C = A A^T (section 3.1), and the Bernoulli-logit GLM
 * log-likelihood with its gradient (section 3.4).
 *
 * The conventions of gpchol.h apply: row-major FP64 with leading dimensions
 * in [max(1, columns), 2^20], device pointers owned by the caller, calls
 * asynchronous on the handle's stream, status codes for argument and runtime
 * errors, outputs that must not overlap inputs (GPC_ERR_ARG otherwise, found
 * before anything is enqueued).  Triangular inputs are read from their lower
 * triangle only; triangular outputs have their strict upper triangle written
 * as 0.  Workspace is the handle's (grown on demand, which waits for the
 * stream once).  Every call is one record of the launch trace class
 * GPC_K_OPS.
 */
#ifndef GPCHOL_OPS_H
#define GPCHOL_OPS_H

#include "gpchol.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Lower-triangular inverse (section 3.2, the solve whose right-hand side is
 * the identity, by the divide-and-conquer step C3 = -C2 A3 C1 applied level
 * by level over the diagonal blocks): X <- L^-1, n x n, lower.  The inverses
 * of the 128 x 128 diagonal blocks come first, then each level doubles the
 * block size with two batched matrix products.  X must not overlap L.  A zero
 * or non-finite diagonal of L gives non-finite entries (no check). */
gpc_status gpc_trtri(gpc_handle* h, int64_t n, const double* L, int64_t ldl, double* X, int64_t ldx);

/* Reverse mode of gpc_trtri (section 3.2): given X = L^-1 and the adjoint
 * Xbar of its lower triangle (the strict upper triangle of Xbar is not read),
 * Lbar <- -tril(X^T tril(Xbar) X^T), lower, strict upper 0.  Workspace: n x n
 * doubles.  Lbar must not overlap X or Xbar. */
gpc_status gpc_trtri_adjoint(gpc_handle* h, int64_t n, const double* X, int64_t ldx, const double* Xbar,
                             int64_t ldxb, double* Lbar, int64_t ldlb);

/* Reverse mode of gpc_trsm (section 3.2; the printed first step is read as
 * the transposed solve): for C = L^-1 B (trans = GPC_NOTRANS) or C = L^-T B
 * (GPC_TRANS), with C and its adjoint Cbar (n x nrhs), in place
 * Cbar <- Bbar = L^-T Cbar (GPC_NOTRANS) or L^-1 Cbar (GPC_TRANS), and
 * Lbar <- -tril(Bbar C^T) (GPC_NOTRANS) or -tril(C Bbar^T) (GPC_TRANS),
 * n x n lower, strict upper 0.  The solve is gpc_trsm's (its sweep status
 * is reported by gpc_check).  No output may overlap an input. */
gpc_status gpc_trsm_adjoint(gpc_handle* h, int32_t trans, int64_t n, int64_t nrhs, const double* L, int64_t ldl,
                            const double* C, int64_t ldc, double* Cbar, int64_t ldcb, double* Lbar, int64_t ldlb);

/* Matrix product (section 3.1): C <- op(A) op(B) + beta C with beta 0 or 1,
 * op(A) M x K (A is M x K, or K x M read transposed when ta = 1), op(B)
 * K x N (B is K x N, or N x K when tb = 1).  128 x 128 MFMA tiles; when the
 * output has few tiles for a long inner dimension (section 3.1, "large k")
 * the inner dimension is split into s slices whose partial products go to
 * the workspace (s M N doubles) and are added in a fixed order, so results
 * repeat bit for bit.  gpc_get_last_splits returns the s of the last call. */
gpc_status gpc_gemm(gpc_handle* h, int32_t ta, int32_t tb, int64_t M, int64_t N, int64_t K, const double* A,
                    int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc);
gpc_status gpc_get_last_splits(const gpc_handle* h, int32_t* splits);

/* Reverse mode of gpc_gemm (section 3.1): given Cbar (M x N),
 * Abar <- d<Cbar, C>/dA + beta Abar (Cbar op(B)^T, or its transpose when
 * ta = 1) and Bbar <- d<Cbar, C>/dB + beta Bbar (op(A)^T Cbar, or its
 * transpose when tb = 1), each shaped like its input; either may be NULL to
 * skip it.  Each is one gpc_gemm call (so split along k when its inner
 * dimension is long). */
gpc_status gpc_gemm_adjoint(gpc_handle* h, int32_t ta, int32_t tb, int64_t M, int64_t N, int64_t K, const double* A,
                            int64_t lda, const double* B, int64_t ldb, const double* Cbar, int64_t ldcb, double beta,
                            double* Abar, int64_t ldab, double* Bbar, int64_t ldbb);

/* C <- A A^T (section 3.1, multiply_transpose): A is M x K; C is the full
 * symmetric M x M product, its lower tiles computed and mirrored. */
gpc_status gpc_multiply_transpose(gpc_handle* h, int64_t M, int64_t K, const double* A, int64_t lda, double* C,
                                  int64_t ldc);

/* Reverse mode of gpc_multiply_transpose: Abar <- (Cbar + Cbar^T) A + beta Abar. */
gpc_status gpc_multiply_transpose_adjoint(gpc_handle* h, int64_t M, int64_t K, const double* A, int64_t lda,
                                          const double* Cbar, int64_t ldcb, double beta, double* Abar, int64_t ldab);

/* Bernoulli-logit GLM (section 3.4; the likelihood of the logistic
 * regression example, section 4.1): with mu_i = alpha + sum_j X_ij beta_j
 * and s the logistic function,
 *   lp = sum_i y_i log s(mu_i) + (1 - y_i) log(1 - s(mu_i)),
 *   dalpha = sum_i d_i,  dbeta_j = sum_i X_ij d_i,  dX_ij = d_i beta_j,
 *   d_i = y_i - s(mu_i).
 * X: n x k (device), y: n device int32 (0 or 1), alpha: device double,
 * beta: k device doubles; lp, dalpha: device doubles; dbeta: k device
 * doubles; dX (n x k) may be NULL to skip it.  X is read once when
 * k <= 2048 (the row's linear term, likelihood and gradient contribution in
 * one pass), twice beyond.  Sums run in a fixed order. */
gpc_status gpc_glm_bernoulli_logit(gpc_handle* h, int64_t n, int64_t k, const double* X, int64_t ldx,
                                   const int32_t* y, const double* alpha, const double* beta, double* lp,
                                   double* dalpha, double* dbeta, double* dX, int64_t lddx);

#ifdef __cplusplus
}
#endif
#endif /* GPCHOL_OPS_H */
