// Register-resident diagonal-block routines shared by the stand-alone kernels
// and the persistent batched kernel (256 threads as a 16 x 16 grid).
#pragma once

#include "internal.hpp"

namespace gpc {

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
// NA: number of 16-row groups (block edge up to 16 * NA); 256 threads.
// colbuf, rowbuf: LDS arrays of 16 * NA doubles; sljj: one LDS double.
template <int NA>
__device__ void diag_factor_inverse(int kb, double* A, int64_t lda, double* Linv, int64_t ldi, int32_t* info,
                                    int64_t col0, double* colbuf, double* rowbuf, double* sljj)
{
    const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;

    // strict upper triangles of both outputs are zero
    for (int idx = tid; idx < kb * kb; idx += 256) {
        const int r = idx / kb, c = idx % kb;
        if (c > r) {
            A[r * lda + c] = 0.0;
            Linv[r * ldi + c] = 0.0;
        }
    }

    double E[NA][NA];
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b) {
            const int i = ty + 16 * a, c = tx + 16 * b;
            E[a][b] = (i < kb && c <= i) ? A[i * lda + c] : 0.0;
        }

#pragma unroll
    for (int aj = 0; aj < NA; ++aj) {
        if (aj * 16 >= kb) break;
        for (int rj = 0; rj < 16; ++rj) {
            const int j = aj * 16 + rj;
            if (j >= kb) break;
            // A: pivot
            if (ty == rj && tx == rj) {
                const double d = E[aj][aj];
                if (!(d > 0.0) && *info == 0) *info = (int32_t)(col0 + j + 1);
                const double l = sqrt(d);
                *sljj = l;
                A[j * lda + j] = l;
            }
            __syncthreads();
            const double ljj = *sljj;
            const double rl = 1.0 / ljj;
            // B: publish column j of L and row j of the inverse
            if (tx == rj) {
#pragma unroll
                for (int a = aj; a < NA; ++a) {
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
            double g[NA], f[NA];
#pragma unroll
            for (int a = 0; a < NA; ++a) {
                const int i = ty + 16 * a;
                g[a] = (i > j && i < kb) ? colbuf[i] : 0.0;
            }
#pragma unroll
            for (int b = 0; b < NA; ++b) {
                const int c = tx + 16 * b;
                f[b] = c >= kb ? 0.0 : (c > j ? colbuf[c] : rowbuf[c]);
            }
#pragma unroll
            for (int a = 0; a < NA; ++a)
#pragma unroll
                for (int b = 0; b <= a; ++b)
                    E[a][b] -= g[a] * f[b];
        }
    }
}


// Inverse X = L^-1 of a lower-triangular block (edge kb <= 16 * NA) read from
// global memory; the block sits in LDS (Ls, pitch 16*NA + 1) and thread
// (ty, tx) keeps the inverse's entries (ty + 16a, tx + 16b), a >= b, in
// registers.  Step j: the owners of row j publish the final row
// X_jc = E(j,c) / L_jj (c < j) and X_jj = 1 / L_jj; then every thread does
// E(i,c) -= L_ij X_jc for i > j, c <= j (forward substitution on all
// columns at once).  X is written with leading dimension ldx, upper := 0.
template <int NA>
__device__ void diag_inverse(int kb, const double* L, int64_t ldl, double* X, int64_t ldx, double* Ls,
                             double* rowbuf)
{
    constexpr int P = 16 * NA + 1;
    const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
    for (int idx = tid; idx < kb * kb; idx += 256) {
        const int r = idx / kb, c = idx % kb;
        Ls[r * P + c] = c <= r ? L[r * ldl + c] : 0.0;
        if (c > r) X[r * ldx + c] = 0.0;
    }
    double E[NA][NA];
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b)
            E[a][b] = (ty + 16 * a == tx + 16 * b) ? 1.0 : 0.0;
    __syncthreads();
#pragma unroll
    for (int aj = 0; aj < NA; ++aj) {
        if (aj * 16 >= kb) break;
        for (int rj = 0; rj < 16; ++rj) {
            const int j = aj * 16 + rj;
            if (j >= kb) break;
            const double rl = 1.0 / Ls[j * P + j];
            if (ty == rj) {
#pragma unroll
                for (int b = 0; b <= aj; ++b) {
                    const int c = tx + 16 * b;
                    if (c <= j) {
                        const double xh = E[aj][b] * rl;
                        rowbuf[c] = xh;
                        X[j * ldx + c] = xh;
                    }
                }
            }
            __syncthreads();
            double g[NA], f[NA];
#pragma unroll
            for (int a = 0; a < NA; ++a) {
                const int i = ty + 16 * a;
                g[a] = (i > j && i < kb) ? Ls[i * P + j] : 0.0;
            }
#pragma unroll
            for (int b = 0; b < NA; ++b) {
                const int c = tx + 16 * b;
                f[b] = c <= j ? rowbuf[c] : 0.0;
            }
#pragma unroll
            for (int a = 0; a < NA; ++a)
#pragma unroll
                for (int b = 0; b <= a; ++b)
                    E[a][b] -= g[a] * f[b];
            __syncthreads();
        }
    }
}

}  // namespace gpc
