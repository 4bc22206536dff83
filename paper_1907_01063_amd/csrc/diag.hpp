// Register-resident diagonal-block routines shared by the stand-alone kernels
// and the persistent batched kernel (256 threads as a 16 x 16 grid).
#pragma once

#include <type_traits>

#include "internal.hpp"

namespace gpc {

// f(std::integral_constant<int, I>()) for I = B .. E-1, unrolled at compile time.
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>());
        static_for<B + 1, E>(f);
    }
}

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
    // wait for the block's loads here, once: otherwise the wait for them sits
    // inside the column loop, where it also waits for every store of L issued
    // by the previous columns
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
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


// Same factor + inverse with columns eliminated four at a time (fewer
// barriers, more registers: used where no product kernel runs beside it).
// Thread (ty, tx) of a 16 x 16 grid owns the elements (i, c) = (ty + 16a, tx + 16b)
// with a >= b (the lower triangle, up to 36 per thread) in E[a][b] for the
// whole kernel.  Columns are eliminated four at a time (J = j .. j+3), one
// barrier per group:
//   publish  the owners of the group's columns put their Schur-complement
//            entries P_r = E(r, J) (zero above the diagonal) in colbuf; the
//            owners of the group's rows put their running inverse entries
//            Q_c = E(J, c), c < j, in rowbuf;                          barrier
//   update   every thread factors the 4 x 4 diagonal block S = l l^T itself
//            (refined 1/sqrt for the pivots; a failed pivot is recorded) and
//            forms Y = l^-1, then for the rows i and columns c it owns
//            L(i, J) = P_i Y^T and F(c) = Y V_c, with V_c = P_c below the
//            group, Q_c left of it and the unit vector inside it, so that F(c)
//            is L(c, J) below the group (Schur complement), the final rows J of
//            the inverse left of it, and Y's columns inside it (inverse by
//            forward substitution).  Rows below the group take
//            E(i, c) -= L(i, J) F(c) (the group's own columns restart at 0 as
//            inverse columns); rows of the group finish their inverse row:
//            E(i, c) = l_ii F_i(c), c < i.
// so the factor of section 3.3.1's diagonal step and its inverse (used by the
// panel solve) come out of the same sweep.  E(i, c), c < i, ends as the
// inverse's entry scaled by l_ii; the inverse is written once at the end and
// the columns of L as each group is done.  The broadcast buffers alternate
// between groups (a thread that publishes group g + 2 has passed the barrier
// of group g + 1, which every thread reaches only after its update with group
// g).  LDS use is small (about 17 KB at NA = 8), so the kernel can share a CU
// with the product kernels that run beside it.  Columns past kb act as an
// identity block (unit pivots, zero coupling).
// NA: number of 16-row groups (block edge up to 16 * NA); 256 threads.
// colbuf, rowbuf: 2 * 4 * 16 * NA doubles; rls: 16 * NA doubles (all LDS).
// A: byte offsets of a 16 NA row band fit in 31 bits.
template <int NA>
__device__ void diag_factor_inverse_g4(int kb, double* A, int64_t lda, double* Linv, int64_t ldi, int32_t* info,
                                    int64_t col0, double* colbuf, double* rowbuf, double* rls)
{
    constexpr int NB = 16 * NA, G = 4;
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
    // wait for the block's loads here, once: otherwise the wait for them sits
    // inside the column loop, where it also waits for every store of L issued
    // by the previous columns
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
    // byte offset of row ty + 16a of A
    uint32_t rowoff[NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) rowoff[a] = (uint32_t)((ty + 16 * a) * lda) * 8u;

    // block columns aj = 0 .. NA-1 with aj a compile-time constant, so that
    // every index into E stays static and E stays in registers
    static_for<0, NA>([&](auto ajc) {
        constexpr int aj = decltype(ajc)::value;
        if (aj * 16 >= kb) return;
        for (int rg = 0; rg < 16 / G; ++rg) {
            const int j = aj * 16 + rg * G;
            if (j >= kb) break;
            double* cb = colbuf + ((j / G) & 1) * NB * G;
            double* rb = rowbuf + ((j / G) & 1) * NB * G;
            const int tc = tx - G * rg;   // group column of this thread's block-aj column (0..3 if in J)
            const int tr = ty - G * rg;   // group row of this thread's block-aj row
            // publish
            if (tc >= 0 && tc < G) {
#pragma unroll
                for (int a = aj; a < NA; ++a) {
                    const int r = ty + 16 * a;
                    cb[r * G + tc] = r >= j + tc ? E[a][aj] : 0.0;
                }
            }
            if (tr >= 0 && tr < G) {
#pragma unroll
                for (int b = 0; b <= aj; ++b) {
                    const int c = tx + 16 * b;
                    rb[c * G + tr] = c < j ? E[aj][b] : 0.0;
                }
            }
            __syncthreads();

            // 4 x 4 diagonal block: S = l l^T, Y = l^-1 (every thread)
            double S[G][G], l[G][G], y[G], Y[G][G];
#pragma unroll
            for (int s2 = 0; s2 < G; ++s2)
#pragma unroll
                for (int t = 0; t <= s2; ++t) S[s2][t] = cb[(j + s2) * G + t];
#pragma unroll
            for (int t = 0; t < G; ++t) {
                double dt = S[t][t];
#pragma unroll
                for (int u = 0; u < t; ++u) dt -= l[t][u] * l[t][u];
                const bool valid = j + t < kb;
                if (tid == 0 && valid && !(dt > 0.0) && *info == 0) *info = (int32_t)(col0 + j + t + 1);
                dt = valid ? dt : 1.0;
                y[t] = rsqrt_refined(dt);
                double lt = dt * y[t];
                l[t][t] = fma(0.5 * y[t], fma(-lt, lt, dt), lt);
#pragma unroll
                for (int s2 = t + 1; s2 < G; ++s2) {
                    double v = S[s2][t];
#pragma unroll
                    for (int u = 0; u < t; ++u) v -= l[s2][u] * l[t][u];
                    l[s2][t] = v * y[t];
                }
            }
#pragma unroll
            for (int t = 0; t < G; ++t) {
                Y[t][t] = y[t];
#pragma unroll
                for (int s2 = 0; s2 < t; ++s2) {
                    double v = 0.0;
#pragma unroll
                    for (int u = s2; u < t; ++u) v += l[t][u] * Y[u][s2];
                    Y[t][s2] = -y[t] * v;
                }
            }
            if (tid < G && j + tid < kb) rls[j + tid] = tid == 0 ? y[0] : tid == 1 ? y[1] : tid == 2 ? y[2] : y[3];

            // L(i, J) for the owned rows (a >= aj), F(c) for the owned columns
            double Lr[NA][G], F[NA][G];
#pragma unroll
            for (int a = aj; a < NA; ++a) {
                double P[G];
#pragma unroll
                for (int s2 = 0; s2 < G; ++s2) P[s2] = cb[(ty + 16 * a) * G + s2];
#pragma unroll
                for (int t = 0; t < G; ++t) {
                    double v = 0.0;
#pragma unroll
                    for (int s2 = 0; s2 <= t; ++s2) v += Y[t][s2] * P[s2];
                    Lr[a][t] = v;
                }
            }
#pragma unroll
            for (int b = 0; b < NA; ++b) {
                const int c = tx + 16 * b;
                double V[G];
#pragma unroll
                for (int s2 = 0; s2 < G; ++s2) {
                    if (b < aj) V[s2] = rb[c * G + s2];
                    else if (b > aj) V[s2] = cb[c * G + s2];
                    else V[s2] = c >= j + G ? cb[c * G + s2] : (c < j ? rb[c * G + s2] : (c - j == s2 ? 1.0 : 0.0));
                }
#pragma unroll
                for (int t = 0; t < G; ++t) {
                    double v = 0.0;
#pragma unroll
                    for (int s2 = 0; s2 <= t; ++s2) v += Y[t][s2] * V[s2];
                    F[b][t] = v;
                }
            }
            // columns J of L, written by their owners
            if (tc >= 0 && tc < G && j + tc < kb) {
#pragma unroll
                for (int a = aj; a < NA; ++a) {
                    const int i = ty + 16 * a;
                    if (i >= j + tc && i < kb) {
                        const double v = tc == 0 ? Lr[a][0] : tc == 1 ? Lr[a][1] : tc == 2 ? Lr[a][2] : Lr[a][3];
                        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v),
                                                              ra, (int)(rowoff[a] + 8u * (j + tc)), 0, 0);
                    }
                }
            }
            // updates: rows below the group; rows of the group finish their inverse row
#pragma unroll
            for (int a = aj; a < NA; ++a) {
                const int i = ty + 16 * a;
                const bool below = a > aj || tr >= G;
                const bool inJ = a == aj && tr >= 0 && tr < G;
                double lii = 0.0;
                if (a == aj) lii = tr == 0 ? l[0][0] : tr == 1 ? l[1][1] : tr == 2 ? l[2][2] : l[3][3];
#pragma unroll
                for (int b = 0; b <= a; ++b) {
                    const int c = tx + 16 * b;
                    if (below) {
                        double v = (b == aj && tc >= 0 && tc < G) ? 0.0 : E[a][b];
#pragma unroll
                        for (int t = 0; t < G; ++t) v -= Lr[a][t] * F[b][t];
                        E[a][b] = v;
                    } else if (inJ && c < i) {
                        const double f = tr == 0 ? F[b][0] : tr == 1 ? F[b][1] : tr == 2 ? F[b][2] : F[b][3];
                        E[a][b] = lii * f;
                    }
                }
            }
        }
    });
    __syncthreads();

    // write out the inverse (row i scaled by 1/l_ii) and zero both upper halves
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
