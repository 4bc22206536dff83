// Register-resident diagonal-block routines shared by the stand-alone kernels
// and the persistent batched kernel (256 threads as a 16 x 16 grid).
#pragma once

#include "internal.hpp"

namespace gpc {

// 1/sqrt(d) to working precision: the hardware estimate refined by two
// Newton steps y <- y + y (1 - d y^2) / 2 (each one doubles the correct bits).
// NaN for d < 0 and NaN, +inf for d = 0, like 1/sqrt.
__device__ __forceinline__ double rsqrt_refined(double d)
{
    double y = __builtin_amdgcn_rsq(d);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double e = fma(-d * y, y, 1.0);
        y = fma(0.5 * y, e, y);
    }
    return y;
}

// Factor + inverse of one diagonal block with the block held in registers.
// Thread (ty, tx) of a 16 x 16 grid owns the elements (i, c) = (ty + 16a, tx + 16b)
// with a >= b (the lower triangle, up to 36 per thread) in E[a][b] for the
// whole kernel.  Column j takes one barrier:
//   publish  the owners of column j put the unscaled E(i, j) in colbuf (zero
//            for i <= j and i >= kb) and restart those registers as the
//            inverse's column j; the owners of row j put the inverse's
//            unscaled row X_jc (c < j), 1 at c = j and zeros beyond in rowbuf;
//            the owner of (j, j) takes d = E(j,j), records a failed pivot,
//            writes L_jj = sqrt(d) and publishes 1/d and 1/L_jj;        barrier
//   update   the owners of column j write L_ij = E(i,j) / L_jj; every thread
//            updates its elements in rows i > j with one multiply-add,
//            f_c = (c > j ? colbuf_c : rowbuf_c) / d:
//              c > j:  E -= E(i,j) E(c,j) / d = L_ij L_cj   (Schur complement)
//              c <= j: E -= E(i,j) X_jc / d = L_ij Xh_jc    (inverse by forward
//                      substitution, Xh_jc = X_jc / L_jj)
// so the factor of section 3.3.1's diagonal step and its inverse (used by the
// panel solve) come out of the same sweep.  E(i, c), c < i, ends as the
// inverse's unscaled entry X_ic; the inverse is written once at the end as
// Xh_ic = X_ic / L_ii.  The broadcast buffers alternate between columns: a
// thread that publishes column j + 2 has passed the barrier of column j + 1,
// which every thread reaches only after its update with column j.  LDS use
// is small (about 5 KB at NA = 8), so the kernel can share a CU with the
// product kernels that run beside it.
// NA: number of 16-row groups (block edge up to 16 * NA); 256 threads.
// colbuf, rowbuf: 2 * 16 * NA doubles; piv: 4 doubles; rls: 16 * NA doubles
// (all LDS).  A and Linv: byte offsets of a 16 NA row band fit in 31 bits.
template <int NA>
__device__ void diag_factor_inverse(int kb, double* A, int64_t lda, double* Linv, int64_t ldi, int32_t* info,
                                    int64_t col0, double* colbuf, double* rowbuf, double* piv, double* rls)
{
    constexpr int NB = 16 * NA;
    const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
    const __amdgpu_buffer_rsrc_t ra =
        __builtin_amdgcn_make_buffer_rsrc(A, (short)0, 0x7fffffff, 0x00020000);

    double E[NA][NA];
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b) {
            const int i = ty + 16 * a, c = tx + 16 * b;
            E[a][b] = (i < kb && c <= i) ? A[i * lda + c] : 0.0;
        }
    // byte offset of row ty + 16a of A
    uint32_t rowoff[NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) rowoff[a] = (uint32_t)((ty + 16 * a) * lda) * 8u;

#pragma unroll
    for (int aj = 0; aj < NA; ++aj) {
        if (aj * 16 >= kb) break;
        for (int rj = 0; rj < 16; ++rj) {
            const int j = aj * 16 + rj;
            if (j >= kb) break;
            double* cb = colbuf + (j & 1) * NB;
            double* rb = rowbuf + (j & 1) * NB;
            double* pv = piv + (j & 1) * 2;
            // publish
            if (tx == rj) {
#pragma unroll
                for (int a = aj; a < NA; ++a) {
                    const int i = ty + 16 * a;
                    const bool below = i > j && i < kb;
                    cb[i] = below ? E[a][aj] : 0.0;
                    if (below) E[a][aj] = 0.0;
                }
            }
            if (ty == rj) {
#pragma unroll
                for (int b = 0; b < NA; ++b) {
                    const int c = tx + 16 * b;
                    rb[c] = b <= aj ? (c < j ? E[aj][b] : (c == j ? 1.0 : 0.0)) : 0.0;
                }
                if (tx == rj) {
                    const double d = E[aj][aj];
                    if (!(d > 0.0) && *info == 0) *info = (int32_t)(col0 + j + 1);
                    const double y = rsqrt_refined(d);
                    double l = d * y;                      // sqrt(d), one correction step
                    l = fma(0.5 * y, fma(-l, l, d), l);
                    pv[0] = y * y;
                    pv[1] = y;
                    rls[j] = y;
                    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, l),
                                                          ra, (int)(rowoff[aj] + 8u * j), 0, 0);
                }
            }
            __syncthreads();
            // update (rows i > j only: a >= aj)
            const double rd = pv[0], rl = pv[1];
            double g[NA], f[NA];
#pragma unroll
            for (int a = aj; a < NA; ++a) g[a] = cb[ty + 16 * a];
            if (tx == rj) {
#pragma unroll
                for (int a = aj; a < NA; ++a) {
                    const int i = ty + 16 * a;
                    if (i > j && i < kb)
                        __builtin_amdgcn_raw_buffer_store_b64(
                            __builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, g[a] * rl), ra,
                            (int)(rowoff[a] + 8u * j), 0, 0);
                }
            }
#pragma unroll
            for (int b = 0; b < NA; ++b) {
                // colbuf is fresh only in rows >= 16 aj; columns c < 16 aj are <= j
                const int c = tx + 16 * b;
                f[b] = (b < aj ? rb[c] : (b > aj ? cb[c] : (c > j ? cb[c] : rb[c]))) * rd;
            }
#pragma unroll
            for (int a = aj; a < NA; ++a)
#pragma unroll
                for (int b = 0; b <= a; ++b)
                    E[a][b] -= g[a] * f[b];
        }
    }
    __syncthreads();

    // write out the inverse (row i scaled by 1/L_ii) and zero both upper halves
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b) {
            const int i = ty + 16 * a, c = tx + 16 * b;
            if (i < kb && c <= i) Linv[i * ldi + c] = c < i ? E[a][b] * rls[i] : rls[i];
        }
    for (int idx = tid; idx < kb * kb; idx += 256) {
        const int r = idx / kb, c = idx % kb;
        if (c > r) {
            A[r * lda + c] = 0.0;
            Linv[r * ldi + c] = 0.0;
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
