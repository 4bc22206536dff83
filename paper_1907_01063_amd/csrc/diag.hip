// Diagonal-block kernels: one workgroup owns one kb x kb block (kb <= 128)
// held entirely in LDS (128 x 129 doubles = 132 KB of the CU's 160 KB).
//
// potrf_diag: the classic unblocked Cholesky of the diagonal block, the
// "chol" step of section 3.3.1, and in the same sweep the inverse of the
// resulting triangle (needed by the panel solve L21 = A21 L11^-T, done as a
// product with the inverse as the paper does with its lower-triangular
// inverse, section 3.2).  Held in registers, see potrf_diag_kernel.
//
// trtri_diag_batched: inverses of all diagonal blocks of a given factor, one
// workgroup per block (the D^-1 of each step of the reverse sweep, 3.3.2);
// block q goes to Dinv + q*b*b with leading dimension b.
#include "internal.hpp"

namespace gpc {
namespace {

constexpr int P = kDiagMax + 1;   // LDS row pitch (odd: spreads column walks over banks)

// X = L^-1 for the lower triangle L in S.  X[i][c] (i > c) is kept in the
// strict upper triangle at S[c][i], the diagonal of X in xd.  Row j of X is
// final once divided by L_jj; it is then subtracted, times L_ij, from every
// later row i (forward substitution on all columns at once).  The division of
// row j is deferred to step j+1, one barrier per step.
__device__ void invert_in_lds(double* S, double* xd, int kb)
{
    const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
    for (int i = tid; i < kb; i += 256) xd[i] = 1.0;
    for (int idx = tid; idx < kb * kb; idx += 256) {
        const int r = idx / kb, c = idx % kb;
        if (c > r) S[r * P + c] = 0.0;
    }
    __syncthreads();
    for (int j = 0; j < kb; ++j) {
        if (j > 0) {
            const double l = S[(j - 1) * P + (j - 1)];
            for (int c = tid; c < j; c += 256) {
                if (c == j - 1) xd[j - 1] /= l;
                else S[c * P + (j - 1)] /= l;
            }
        }
        const double ljj = S[j * P + j];
        const int m = kb - j - 1;
        for (int q = tx; q <= j; q += 16) {
            const double xjc = (q == j ? xd[j] : S[q * P + j]) / ljj;
            for (int p = ty; p < m; p += 16) {
                const int i = j + 1 + p;
                S[q * P + i] -= S[i * P + j] * xjc;
            }
        }
        __syncthreads();
    }
    {
        const double l = S[(kb - 1) * P + (kb - 1)];
        for (int c = tid; c < kb; c += 256) {
            if (c == kb - 1) xd[kb - 1] /= l;
            else S[c * P + (kb - 1)] /= l;
        }
    }
    __syncthreads();
}

// Factor + inverse of one diagonal block with the block held in registers.
// Thread (ty, tx) of a 16 x 16 grid owns the elements (i, c) = (ty + 16a, tx + 16b)
// with a >= b (the lower triangle, up to 36 per thread) in E[a][b] for the
// whole kernel.  Step j (one column):
//   A. the owner of (j, j) takes d = E(j,j), records a failed pivot, publishes
//      L_jj = sqrt(d) and writes it out;                              barrier
//   B. owners of column j publish L_ij = E(i,j) / L_jj (i > j) and write them
//      out, then restart those registers as the inverse's column j; owners of
//      row j publish the now-final inverse row Xh_jc = X_jc / L_jj (c < j)
//      and 1 / L_jj, and write them out;                              barrier
//   C. every thread updates its elements with one multiply-add:
//      c > j:  E -= L_ij L_cj       (trailing Schur complement)
//      c <= j: E -= L_ij Xh_jc      (forward substitution of the inverse)
// so the factor of section 3.3.1's diagonal step and its inverse (used by the
// panel solve) come out of the same sweep.  E(i, c) for c < j holds the
// inverse's running entry X_ic once column c of L has been written out.
__global__ void __launch_bounds__(256)
potrf_diag_kernel(int kb, double* A, int64_t lda, double* Linv, int64_t ldi, int32_t* info, int64_t col0)
{
    __shared__ double colbuf[kDiagMax];
    __shared__ double rowbuf[kDiagMax];
    __shared__ double sljj;
    const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;

    // strict upper triangles of both outputs are zero
    for (int idx = tid; idx < kb * kb; idx += 256) {
        const int r = idx / kb, c = idx % kb;
        if (c > r) {
            A[r * lda + c] = 0.0;
            Linv[r * ldi + c] = 0.0;
        }
    }

    double E[8][8];
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b) {
            const int i = ty + 16 * a, c = tx + 16 * b;
            E[a][b] = (i < kb && c <= i) ? A[i * lda + c] : 0.0;
        }

#pragma unroll
    for (int aj = 0; aj < 8; ++aj) {
        if (aj * 16 >= kb) break;
        for (int rj = 0; rj < 16; ++rj) {
            const int j = aj * 16 + rj;
            if (j >= kb) break;
            // A: pivot
            if (ty == rj && tx == rj) {
                const double d = E[aj][aj];
                if (!(d > 0.0) && *info == 0) *info = (int32_t)(col0 + j + 1);
                const double l = sqrt(d);
                sljj = l;
                A[j * lda + j] = l;
            }
            __syncthreads();
            const double ljj = sljj;
            const double rl = 1.0 / ljj;
            // B: publish column j of L and row j of the inverse
            if (tx == rj) {
#pragma unroll
                for (int a = aj; a < 8; ++a) {
                    const int i = ty + 16 * a;
                    if (i > j && i < kb) {
                        const double l = E[a][aj] * rl;
                        colbuf[i] = l;
                        A[i * lda + j] = l;
                        E[a][aj] = 0.0;
                    }
                }
            }
            if (ty == rj) {
#pragma unroll
                for (int b = 0; b <= aj; ++b) {
                    const int c = tx + 16 * b;
                    if (c < j) {
                        const double xh = E[aj][b] * rl;
                        rowbuf[c] = xh;
                        Linv[j * ldi + c] = xh;
                    } else if (c == j) {
                        rowbuf[j] = rl;
                        Linv[j * ldi + j] = rl;
                    }
                }
            }
            __syncthreads();
            // C: one multiply-add per owned element
            double g[8], f[8];
#pragma unroll
            for (int a = 0; a < 8; ++a) {
                const int i = ty + 16 * a;
                g[a] = (i > j && i < kb) ? colbuf[i] : 0.0;
            }
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const int c = tx + 16 * b;
                f[b] = c >= kb ? 0.0 : (c > j ? colbuf[c] : rowbuf[c]);
            }
#pragma unroll
            for (int a = 0; a < 8; ++a)
#pragma unroll
                for (int b = 0; b <= a; ++b)
                    E[a][b] -= g[a] * f[b];
        }
    }
}

__global__ void __launch_bounds__(256)
trtri_batched_kernel(int64_t n, int b, const double* L, int64_t ldl, double* Dinv)
{
    __shared__ double S[kDiagMax * P];
    __shared__ double xd[kDiagMax];
    const int tid = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * b;
    const int kb = (int)min((int64_t)b, n - r0);
    const double* D = L + r0 * ldl + r0;
    double* X = Dinv + (int64_t)blockIdx.x * b * b;
    for (int idx = tid; idx < kb * kb; idx += 256) {
        const int r = idx / kb, c = idx % kb;
        S[r * P + c] = c <= r ? D[r * ldl + c] : 0.0;
    }
    __syncthreads();
    invert_in_lds(S, xd, kb);
    for (int idx = tid; idx < kb * kb; idx += 256) {
        const int r = idx / kb, c = idx % kb;
        X[r * b + c] = c < r ? S[c * P + r] : (c == r ? xd[r] : 0.0);
    }
}

}  // namespace

hipError_t potrf_diag(hipStream_t s, int kb, double* A, int64_t lda, double* Linv, int64_t ldi,
                      int32_t* info, int64_t col0)
{
    if (kb <= 0) return hipSuccess;
    if (kb > kDiagMax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(potrf_diag_kernel, dim3(1), dim3(256), 0, s, kb, A, lda, Linv, ldi, info, col0);
    return hipGetLastError();
}

hipError_t trtri_diag_batched(hipStream_t s, int64_t n, int b, const double* L, int64_t ldl, double* Dinv)
{
    if (n <= 0) return hipSuccess;
    if (b <= 0 || b > kDiagMax) return hipErrorInvalidValue;
    const int64_t nblk = (n + b - 1) / b;
    hipLaunchKernelGGL(trtri_batched_kernel, dim3((unsigned)nblk), dim3(256), 0, s, n, b, L, ldl, Dinv);
    return hipGetLastError();
}

}  // namespace gpc
