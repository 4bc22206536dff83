/*
 * Plain CPU oracle for the Cholesky factor, its reverse-mode adjoint, the
 * triangular solves, the log-determinant and the GP pieces built on them.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may use it.  It shares no code, header, table or helper with
 * the HIP path.
 *
 * Every routine is the plain definition written out as loops, in FP64 (the
 * paper computes in double precision throughout, section 2.3 and 3.5), with a
 * long-double "referee" variant of the factor and the adjoint that measures the
 * rounding floor of the FP64 versions.  Storage is row-major with a leading
 * dimension (element (i,j) of X is X[i*ldx + j]); only the lower triangle of
 * symmetric inputs is read, and the strict upper triangle of triangular outputs
 * is written as zero (the lower/upper "view" convention of section 2.2).
 *
 * Parallel loops (OpenMP) only split work whose results are independent of one
 * another; every reduction runs in a fixed order, so results do not depend on
 * the thread count.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define AT(X, ld, i, j) ((X)[(int64_t)(i) * (ld) + (j)])

/* Thread count of the parallel loops (for timing; results do not depend on it). */
int orc_max_threads(void) { return omp_get_max_threads(); }
void orc_set_threads(int t) { if (t > 0) omp_set_num_threads(t); }

/* Rows per fixed chunk of the column reductions in the adjoint. */
#define ORC_CHUNK 64

/* ------------------------------------------------------------------------ */
/* Factor: section 3.3.1.  L is the unique lower-triangular matrix with a
 * positive diagonal and L*L^T = A; the paper's block identities
 * (L11 = chol(A11), L21 = A21*L11^-T, then the Schur complement A22 - L21*L21^T
 * factored recursively) reach the same L, and for blocks of width one they are
 * the column-by-column (Crout) recurrence written here:
 *   s_j  = A_jj - sum_{k<j} L_jk^2          (k increasing)
 *   L_jj = sqrt(s_j)                        (requires s_j > 0)
 *   L_ij = (A_ij - sum_{k<j} L_ik L_jk) / L_jj   for i > j.
 * Returns 0, or j+1 for the first column j whose pivot s_j is not > 0 (this
 * includes NaN); L is then unspecified from column j on.                      */
int orc_potrf(int64_t n, const double* A, int64_t lda, double* L, int64_t ldl)
{
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j)
            AT(L, ldl, i, j) = (j <= i) ? AT(A, lda, i, j) : 0.0;

    for (int64_t j = 0; j < n; ++j) {
        double acc = 0.0;
        for (int64_t k = 0; k < j; ++k)
            acc += AT(L, ldl, j, k) * AT(L, ldl, j, k);
        double s = AT(L, ldl, j, j) - acc;
        if (!(s > 0.0))
            return (int)(j + 1);
        double ljj = sqrt(s);
        AT(L, ldl, j, j) = ljj;
#pragma omp parallel for schedule(static)
        for (int64_t i = j + 1; i < n; ++i) {
            double dot = 0.0;
            for (int64_t k = 0; k < j; ++k)
                dot += AT(L, ldl, i, k) * AT(L, ldl, j, k);
            AT(L, ldl, i, j) = (AT(L, ldl, i, j) - dot) / ljj;
        }
    }
    return 0;
}

/* Same recurrence with every sum and quotient carried in long double; the
 * result is rounded to double once at the end (referee of the FP64 floor).   */
int orc_potrf_ref(int64_t n, const double* A, int64_t lda, double* L, int64_t ldl)
{
    long double* W = (long double*)malloc(sizeof(long double) * (size_t)(n * n + 1));
    if (!W) return -1;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j)
            W[i * n + j] = (j <= i) ? (long double)AT(A, lda, i, j) : 0.0L;
    int info = 0;
    for (int64_t j = 0; j < n && !info; ++j) {
        long double acc = 0.0L;
        for (int64_t k = 0; k < j; ++k)
            acc += W[j * n + k] * W[j * n + k];
        long double s = W[j * n + j] - acc;
        if (!(s > 0.0L)) { info = (int)(j + 1); break; }
        long double ljj = sqrtl(s);
        W[j * n + j] = ljj;
#pragma omp parallel for schedule(static)
        for (int64_t i = j + 1; i < n; ++i) {
            long double dot = 0.0L;
            for (int64_t k = 0; k < j; ++k)
                dot += W[i * n + k] * W[j * n + k];
            W[i * n + j] = (W[i * n + j] - dot) / ljj;
        }
    }
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j)
            AT(L, ldl, i, j) = (double)W[i * n + j];
    free(W);
    return info;
}

/* ------------------------------------------------------------------------ */
/* Adjoint: section 3.3.2.  Given L and the adjoint Lbar of the lower-triangular
 * output, Abar is the gradient of f(A) = sum_{i>=j} Lbar_ij * L_ij(A) with
 * respect to the independent lower-triangle entries a_ij (i >= j) of the
 * symmetric A: the derivative the paper's blocked gradient returns once it has
 * halved the diagonal and zeroed the upper triangle of each diagonal block.
 *
 * It is computed by running the factor's recurrence backwards (reverse-mode
 * differentiation of each assignment, last assignment first).  G holds the
 * running adjoints of the entries of L.  For column j = n-1 down to 0:
 *   for each i > j, from the quotient L_ij = (A_ij - sum_k L_ik L_jk) / L_jj:
 *       t = G_ij / L_jj;   Abar_ij = t;   G_jj -= t * L_ij;
 *       G_ik -= t * L_jk and G_jk -= t * L_ik   for every k < j;
 *   then from L_jj = sqrt(A_jj - sum_k L_jk^2):
 *       sbar = G_jj / (2 L_jj);  Abar_jj = sbar;  G_jk -= 2 sbar L_jk  (k < j).
 * Row i's own updates are private to i (parallel over i); the updates of row j
 * are sums over i taken in fixed chunks of ORC_CHUNK rows, added in chunk
 * order.                                                                       */
void orc_potrf_adjoint(int64_t n, const double* L, int64_t ldl,
                       const double* Lbar, int64_t ldlb,
                       double* Abar, int64_t ldab)
{
    double* G = (double*)malloc(sizeof(double) * (size_t)(n * n + 1));
    int64_t nchunk = (n + ORC_CHUNK - 1) / ORC_CHUNK + 1;
    double* part = (double*)malloc(sizeof(double) * (size_t)(nchunk * (n + 1) + 1));
    double* t = (double*)malloc(sizeof(double) * (size_t)(n + 1));
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            G[i * n + j] = (j <= i) ? AT(Lbar, ldlb, i, j) : 0.0;
            AT(Abar, ldab, i, j) = 0.0;
        }

    for (int64_t j = n - 1; j >= 0; --j) {
        const double ljj = AT(L, ldl, j, j);
        for (int64_t i = j + 1; i < n; ++i) {
            t[i] = G[i * n + j] / ljj;
            AT(Abar, ldab, i, j) = t[i];
        }
        /* the diagonal adjoint collects t_i * L_ij, i increasing */
        double gdiag = 0.0;
        for (int64_t i = j + 1; i < n; ++i)
            gdiag += t[i] * AT(L, ldl, i, j);
        G[j * n + j] -= gdiag;

        int64_t nrows = n - (j + 1);
        int64_t nc = (nrows + ORC_CHUNK - 1) / ORC_CHUNK;
#pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < nc; ++c) {
            double* p = part + c * (n + 1);
            for (int64_t k = 0; k < j; ++k) p[k] = 0.0;
            int64_t i0 = j + 1 + c * ORC_CHUNK;
            int64_t i1 = i0 + ORC_CHUNK < n ? i0 + ORC_CHUNK : n;
            for (int64_t i = i0; i < i1; ++i) {
                const double ti = t[i];
                double* gi = G + i * n;
                const double* li = L + i * ldl;
                const double* lj = L + j * ldl;
                for (int64_t k = 0; k < j; ++k) {
                    gi[k] -= ti * lj[k];
                    p[k] += ti * li[k];
                }
            }
        }
        for (int64_t c = 0; c < nc; ++c) {
            const double* p = part + c * (n + 1);
            for (int64_t k = 0; k < j; ++k) G[j * n + k] -= p[k];
        }

        const double sbar = G[j * n + j] / (2.0 * ljj);
        AT(Abar, ldab, j, j) = sbar;
        for (int64_t k = 0; k < j; ++k)
            G[j * n + k] -= 2.0 * sbar * AT(L, ldl, j, k);
    }
    free(t);
    free(part);
    free(G);
}

/* The same reverse sweep with long-double running adjoints (referee).        */
void orc_potrf_adjoint_ref(int64_t n, const double* L, int64_t ldl,
                           const double* Lbar, int64_t ldlb,
                           double* Abar, int64_t ldab)
{
    long double* G = (long double*)malloc(sizeof(long double) * (size_t)(n * n + 1));
    long double* R = (long double*)malloc(sizeof(long double) * (size_t)(n * n + 1));
    long double* t = (long double*)malloc(sizeof(long double) * (size_t)(n + 1));
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            G[i * n + j] = (j <= i) ? (long double)AT(Lbar, ldlb, i, j) : 0.0L;
            R[i * n + j] = 0.0L;
        }
    for (int64_t j = n - 1; j >= 0; --j) {
        const long double ljj = AT(L, ldl, j, j);
        for (int64_t i = j + 1; i < n; ++i) {
            t[i] = G[i * n + j] / ljj;
            R[i * n + j] = t[i];
        }
        long double gdiag = 0.0L;
        for (int64_t i = j + 1; i < n; ++i)
            gdiag += t[i] * (long double)AT(L, ldl, i, j);
        G[j * n + j] -= gdiag;
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < j; ++k) {
            long double acc = 0.0L;
            for (int64_t i = j + 1; i < n; ++i)
                acc += t[i] * (long double)AT(L, ldl, i, k);
            G[j * n + k] -= acc;
        }
#pragma omp parallel for schedule(static)
        for (int64_t i = j + 1; i < n; ++i)
            for (int64_t k = 0; k < j; ++k)
                G[i * n + k] -= t[i] * (long double)AT(L, ldl, j, k);
        const long double sbar = G[j * n + j] / (2.0L * ljj);
        R[j * n + j] = sbar;
        for (int64_t k = 0; k < j; ++k)
            G[j * n + k] -= 2.0L * sbar * (long double)AT(L, ldl, j, k);
    }
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j)
            AT(Abar, ldab, i, j) = (double)R[i * n + j];
    free(t);
    free(R);
    free(G);
}

/* ------------------------------------------------------------------------ */
/* Triangular solves: section 3.2 (a triangular system A x = b with the lower
 * triangular factor; the upper case is the transposed system).
 * trans == 0:  B <- L^-1 B  by forward substitution,
 *              x_i = (b_i - sum_{k<i} L_ik x_k) / L_ii,  i increasing;
 * trans == 1:  B <- L^-T B  by back substitution,
 *              x_i = (b_i - sum_{k>i} L_ki x_k) / L_ii,  i decreasing.
 * B is n x nrhs, row-major with leading dimension ldb; columns are independent. */
void orc_trsm(int trans, int64_t n, int64_t nrhs, const double* L, int64_t ldl,
              double* B, int64_t ldb)
{
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nrhs; ++c) {
        if (trans == 0) {
            for (int64_t i = 0; i < n; ++i) {
                double acc = 0.0;
                for (int64_t k = 0; k < i; ++k)
                    acc += AT(L, ldl, i, k) * AT(B, ldb, k, c);
                AT(B, ldb, i, c) = (AT(B, ldb, i, c) - acc) / AT(L, ldl, i, i);
            }
        } else {
            for (int64_t i = n - 1; i >= 0; --i) {
                double acc = 0.0;
                for (int64_t k = i + 1; k < n; ++k)
                    acc += AT(L, ldl, k, i) * AT(B, ldb, k, c);
                AT(B, ldb, i, c) = (AT(B, ldb, i, c) - acc) / AT(L, ldl, i, i);
            }
        }
    }
}

/* log|A| = log|L L^T| = 2 * sum_i log L_ii, i increasing (section 1: the GP
 * log-density needs the determinant of the covariance through its factor).  */
double orc_logdet(int64_t n, const double* L, int64_t ldl)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i)
        s += log(AT(L, ldl, i, i));
    return 2.0 * s;
}

/* ------------------------------------------------------------------------ */
/* GP pieces (section 4.2 motivates the GP regression workload; the kernel is
 * the squared-exponential with one lengthscale per input dimension).
 * K_ij = sigma2 * exp(-1/2 sum_d (x_id - x_jd)^2 / ell_d^2) + noise * [i == j].
 * X is n x d row-major.  Lower triangle and diagonal written, upper zeroed.   */
void orc_gp_kgen_se(int64_t n, int64_t d, const double* X, double sigma2,
                    const double* ell, double noise, double* K, int64_t ldk)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            if (j > i) { AT(K, ldk, i, j) = 0.0; continue; }
            double r2 = 0.0;
            for (int64_t q = 0; q < d; ++q) {
                double diff = X[i * d + q] - X[j * d + q];
                r2 += diff * diff / (ell[q] * ell[q]);
            }
            double v = sigma2 * exp(-0.5 * r2);
            if (i == j) v += noise;
            AT(K, ldk, i, j) = v;
        }
    }
}

/* Adjoint of the lower-triangular factor for the GP log-density
 *   f = -1/2 z^T z - 1/2 log|K|,  z = L^-1 y,  alpha = L^-T z,  log|K| = 2 sum log L_ii.
 * Differentiating: d(-1/2 z^T z) = alpha^T dL z and d(-sum log L_ii) = -sum dL_ii/L_ii,
 * so Lbar = tril(alpha z^T) - diag(1 / L_ii).                                  */
void orc_gp_lbar(int64_t n, const double* L, int64_t ldl, const double* alpha,
                 const double* z, double* Lbar, int64_t ldlb)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            double v = 0.0;
            if (j <= i) v = alpha[i] * z[j];
            if (j == i) v -= 1.0 / AT(L, ldl, i, i);
            AT(Lbar, ldlb, i, j) = v;
        }
}

/* Chain rule from the lower-triangle adjoint Abar to the SE-ARD hyperparameters
 * theta = (sigma2, ell_1..ell_d, noise):  df/dtheta = sum_{i>=j} Abar_ij dK_ij/dtheta,
 *   dK_ij/dsigma2 = exp(-r2_ij/2),
 *   dK_ij/dell_q  = sigma2 exp(-r2_ij/2) (x_iq - x_jq)^2 / ell_q^3,
 *   dK_ij/dnoise  = [i == j].
 * grad has d + 2 entries.  Each row's contribution is formed independently and
 * the rows are added in increasing order.                                      */
void orc_gp_hypergrad_se(int64_t n, int64_t d, const double* X, double sigma2,
                         const double* ell, const double* Abar, int64_t ldab,
                         double* grad)
{
    int64_t m = d + 2;
    double* rowc = (double*)calloc((size_t)(n * m + 1), sizeof(double));
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double* g = rowc + i * m;
        for (int64_t j = 0; j <= i; ++j) {
            double a = AT(Abar, ldab, i, j);
            double r2 = 0.0;
            for (int64_t q = 0; q < d; ++q) {
                double diff = X[i * d + q] - X[j * d + q];
                r2 += diff * diff / (ell[q] * ell[q]);
            }
            double e = exp(-0.5 * r2);
            g[0] += a * e;
            for (int64_t q = 0; q < d; ++q) {
                double diff = X[i * d + q] - X[j * d + q];
                g[1 + q] += a * sigma2 * e * diff * diff / (ell[q] * ell[q] * ell[q]);
            }
            if (i == j) g[m - 1] += a;
        }
    }
    for (int64_t q = 0; q < m; ++q) grad[q] = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t q = 0; q < m; ++q) grad[q] += rowc[i * m + q];
    free(rowc);
}

/* ------------------------------------------------------------------------ */
/* Lower-triangular inverse: section 3.2 (the special case of a triangular
 * solve whose right-hand side is the identity).  X = L^-1 is the lower
 * triangular matrix with L X = I; column j is the forward substitution of
 * L x = e_j:
 *   X_ij = 0 (i < j),   X_jj = 1 / L_jj,
 *   X_ij = -(sum_{k=j}^{i-1} L_ik X_kj) / L_ii   (i > j, k increasing).
 * Columns are independent (parallel over j).                                 */
void orc_trtri(int64_t n, const double* L, int64_t ldl, double* X, int64_t ldx)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < j; ++i) AT(X, ldx, i, j) = 0.0;
        AT(X, ldx, j, j) = 1.0 / AT(L, ldl, j, j);
        for (int64_t i = j + 1; i < n; ++i) {
            double acc = 0.0;
            for (int64_t k = j; k < i; ++k)
                acc += AT(L, ldl, i, k) * AT(X, ldx, k, j);
            AT(X, ldx, i, j) = -acc / AT(L, ldl, i, i);
        }
    }
}

/* Reverse mode of the triangular solve: section 3.2.  For C = L^-1 B
 * (trans 0) the adjoints are Bbar = L^-T Cbar and Lbar = -tril(Bbar C^T);
 * for C = L^-T B (trans 1) they are Bbar = L^-1 Cbar and
 * Lbar = -tril(C Bbar^T).  (From dC = -L^-1 dL C, resp. dC = -L^-T dL^T C:
 * <Cbar, dC> = -<L^-T Cbar C^T, dL>, resp. -<C (L^-1 Cbar)^T, dL>, and only
 * the lower triangle of L is a variable.)  C, Cbar, Bbar: n x nrhs; Bbar is
 * formed by the substitutions of orc_trsm; Lbar is n x n, lower, with
 *   Lbar_ij = -sum_c Bbar_ic C_jc   (trans 0)   or   -sum_c C_ic Bbar_jc   (trans 1)
 * for i >= j (c increasing) and 0 above the diagonal.                          */
void orc_trsm_adjoint(int trans, int64_t n, int64_t nrhs, const double* L, int64_t ldl,
                      const double* C, int64_t ldc, const double* Cbar, int64_t ldcb,
                      double* Bbar, int64_t ldbb, double* Lbar, int64_t ldlb)
{
    for (int64_t i = 0; i < n; ++i)
        for (int64_t c = 0; c < nrhs; ++c) AT(Bbar, ldbb, i, c) = AT(Cbar, ldcb, i, c);
    orc_trsm(trans ? 0 : 1, n, nrhs, L, ldl, Bbar, ldbb);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            double acc = 0.0;
            if (j <= i)
                for (int64_t c = 0; c < nrhs; ++c)
                    acc += trans ? AT(C, ldc, i, c) * AT(Bbar, ldbb, j, c)
                                 : AT(Bbar, ldbb, i, c) * AT(C, ldc, j, c);
            AT(Lbar, ldlb, i, j) = j <= i ? -acc : 0.0;
        }
}

/* Reverse mode of the lower-triangular inverse X = L^-1 (section 3.2): from
 * dX = -X dL X, <Xbar, dX> = -<X^T Xbar X^T, dL>, so with the adjoint of the
 * lower triangle of X (its strict upper part is not a variable and is
 * ignored),  Lbar = -tril(X^T tril(Xbar) X^T):
 *   T_kj    = sum_{l} tril(Xbar)_kl X_jl          (l increasing)
 *   Lbar_ij = -sum_k X_ki T_kj   for i >= j       (k increasing), 0 above.     */
void orc_trtri_adjoint(int64_t n, const double* X, int64_t ldx, const double* Xbar, int64_t ldxb,
                       double* Lbar, int64_t ldlb)
{
    double* T = (double*)malloc(sizeof(double) * (size_t)(n * n + 1));
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k)
        for (int64_t j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int64_t l = 0; l <= k; ++l)
                acc += AT(Xbar, ldxb, k, l) * AT(X, ldx, j, l);
            T[k * n + j] = acc;
        }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            double acc = 0.0;
            if (j <= i)
                for (int64_t k = 0; k < n; ++k)
                    acc += AT(X, ldx, k, i) * T[k * n + j];
            AT(Lbar, ldlb, i, j) = j <= i ? -acc : 0.0;
        }
    free(T);
}

/* ------------------------------------------------------------------------ */
/* Matrix product: section 3.1.  C = op(A) op(B) + beta C with op(A) M x K
 * (A, or A^T when ta) and op(B) K x N (B, or B^T when tb):
 *   C_ij = beta C_ij + sum_{k} op(A)_ik op(B)_kj   (k increasing).            */
void orc_gemm(int ta, int tb, int64_t M, int64_t N, int64_t K, const double* A, int64_t lda,
              const double* B, int64_t ldb, double beta, double* C, int64_t ldc)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < M; ++i)
        for (int64_t j = 0; j < N; ++j) {
            double acc = 0.0;
            for (int64_t k = 0; k < K; ++k)
                acc += (ta ? AT(A, lda, k, i) : AT(A, lda, i, k)) * (tb ? AT(B, ldb, j, k) : AT(B, ldb, k, j));
            AT(C, ldc, i, j) = (beta == 0.0 ? 0.0 : beta * AT(C, ldc, i, j)) + acc;
        }
}

/* The special case C = A A^T of section 3.1 (multiply_transpose): A is M x K,
 * C the full symmetric M x M product, C_ij = C_ji = sum_k A_ik A_jk.          */
void orc_multiply_transpose(int64_t M, int64_t K, const double* A, int64_t lda, double* C, int64_t ldc)
{
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < M; ++i)
        for (int64_t j = 0; j <= i; ++j) {
            double acc = 0.0;
            for (int64_t k = 0; k < K; ++k)
                acc += AT(A, lda, i, k) * AT(A, lda, j, k);
            AT(C, ldc, i, j) = acc;
            AT(C, ldc, j, i) = acc;
        }
}

/* ------------------------------------------------------------------------ */
/* Bernoulli-logit GLM log-likelihood and its gradient: section 3.4 (the
 * likelihood of the logistic regression example, section 4.1):
 *   mu_i = alpha + sum_j X_ij beta_j                       (j increasing)
 *   lp   = sum_i [ y_i log s(mu_i) + (1 - y_i) log(1 - s(mu_i)) ],
 * with s the logistic function, log s(t) = -softplus(-t),
 * log(1 - s(t)) = -softplus(t), softplus(t) = max(t, 0) + log1p(exp(-|t|));
 *   d_i = y_i - s(mu_i)                (dlp / dmu_i)
 *   dalpha = sum_i d_i,   dbeta_j = sum_i X_ij d_i,   dX_ij = d_i beta_j.
 * Sums over i run in increasing i.  dX may be NULL.  y holds 0/1 integers.  */
static double orc_softplus(double t) { return (t > 0.0 ? t : 0.0) + log1p(exp(-fabs(t))); }

void orc_glm_bernoulli_logit(int64_t n, int64_t k, const double* X, int64_t ldx, const int32_t* y,
                             double alpha, const double* beta, double* lp, double* dalpha,
                             double* dbeta, double* dX, int64_t lddx)
{
    double* d = (double*)malloc(sizeof(double) * (size_t)(n + 1));
    double* lpi = (double*)malloc(sizeof(double) * (size_t)(n + 1));
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double mu = alpha;
        for (int64_t j = 0; j < k; ++j) mu += AT(X, ldx, i, j) * beta[j];
        const double yi = (double)y[i];
        lpi[i] = -yi * orc_softplus(-mu) - (1.0 - yi) * orc_softplus(mu);
        d[i] = yi - 1.0 / (1.0 + exp(-mu));
        if (dX)
            for (int64_t j = 0; j < k; ++j) AT(dX, lddx, i, j) = d[i] * beta[j];
    }
    double s = 0.0, sa = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        s += lpi[i];
        sa += d[i];
    }
    *lp = s;
    *dalpha = sa;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < k; ++j) {
        double acc = 0.0;
        for (int64_t i = 0; i < n; ++i) acc += AT(X, ldx, i, j) * d[i];
        dbeta[j] = acc;
    }
    free(lpi);
    free(d);
}
